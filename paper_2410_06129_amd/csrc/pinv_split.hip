// Split-precision (BF16x3) products forming R (Eq. 8) and the few-frame apply
// (Eq. 3) on split-packed operands: each FP32 value is split into bf16 hi/lo
// once, where it is produced, and stored "split-packed" (SP: per 8 consecutive
// k of a row, the re_hi, re_lo, im_hi and im_lo planes, 64 bytes).
//
//   L^-1 and L^-H (SP, rows n, k = n')  <- the FP64 factor, split once
//   W^T[m][n]  = sum_{n' <= n} conj(E[m][n']) Li[n][n']    (SP rows m, k = n)
//   R[n][m]    = sum_{n' >= n} conj(Li[n'][n]) W[n'][m]    (SP rows n, k = m)
// The W product's tiles are W tiles (rows n, columns m) and the R product's
// tiles are R^T tiles (rows m, columns n): the MFMA result layout gives each
// lane four consecutive tile rows of one column, which is the k direction of
// the SP matrix each product writes.
#include "pinv_internal.h"

namespace pinv {

// ---------------------------------------------------------------------------
// Pack / unpack
// ---------------------------------------------------------------------------
// dst row r, 8-group g = split(src(r, 8g .. 8g+7)), zero beyond K, where
// src(r, k) = src[r*ld + k] or, with TRANS, src[k*ld + r]; conjugated with
// CONJ.  Non-transposed, consecutive threads take consecutive groups of a row
// (contiguous reads and writes); transposed, consecutive rows of a group
// (contiguous reads for each k).
template <typename S, bool TRANS, bool CONJ>
__global__ __launch_bounds__(256) void k_sp_pack(const S* __restrict__ src, int64_t ld, int rows,
                                                 int K, int64_t gpr, uint4* __restrict__ dst) {
  const cx<S>* z = reinterpret_cast<const cx<S>*>(src);
  const int64_t total = (int64_t)rows * gpr;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
       u += (int64_t)gridDim.x * blockDim.x) {
    int64_t r, g;
    if constexpr (TRANS) {
      g = u / rows;
      r = u - g * rows;
    } else {
      r = u / gpr;
      g = u - r * gpr;
    }
    float re[8], im[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t k = g * 8 + j;
      re[j] = im[j] = 0.f;
      if (k < K) {
        const cx<S> v = TRANS ? z[k * ld + r] : z[r * ld + k];
        re[j] = float(v.re);
        im[j] = CONJ ? -float(v.im) : float(v.im);
      }
    }
    uint4 o[4];
    sp_group(re, im, o);
#pragma unroll
    for (int p = 0; p < 4; ++p) dst[(r * gpr + g) * 4 + p] = o[p];
  }
}

// dst[r][k] (complex64, row length K) = hi + lo of SP row r.
__global__ __launch_bounds__(256) void k_sp_unpack(const uint4* __restrict__ sp, int64_t gpr,
                                                   int rows, int K, float* __restrict__ dst) {
  cx<float>* d = reinterpret_cast<cx<float>*>(dst);
  const int64_t total = (int64_t)rows * gpr;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = u / gpr, g = u - r * gpr;
    uint4 q[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) q[p] = sp[u * 4 + p];
    const uint32_t rh[4] = {q[0].x, q[0].y, q[0].z, q[0].w}, rl[4] = {q[1].x, q[1].y, q[1].z, q[1].w};
    const uint32_t ih[4] = {q[2].x, q[2].y, q[2].z, q[2].w}, il[4] = {q[3].x, q[3].y, q[3].z, q[3].w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t k = g * 8 + j;
      if (k < K) d[r * K + k] = cx<float>{join2(rh[j >> 1], rl[j >> 1], j & 1), join2(ih[j >> 1], il[j >> 1], j & 1)};
    }
  }
}

static int pack_blocks(int64_t total) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384));
}

template <typename S>
hipError_t launch_sp_pack(const S* src, int64_t ld, int rows, int K, bool trans, bool conj,
                          void* dst, hipStream_t s) {
  const int64_t gpr = sp_cols(K) / 8, total = (int64_t)rows * gpr;
  if (total <= 0) return hipSuccess;
  uint4* o = reinterpret_cast<uint4*>(dst);
  const dim3 grid(pack_blocks(total)), block(256);
  if (trans && conj)
    hipLaunchKernelGGL((k_sp_pack<S, true, true>), grid, block, 0, s, src, ld, rows, K, gpr, o);
  else if (trans)
    hipLaunchKernelGGL((k_sp_pack<S, true, false>), grid, block, 0, s, src, ld, rows, K, gpr, o);
  else if (conj)
    hipLaunchKernelGGL((k_sp_pack<S, false, true>), grid, block, 0, s, src, ld, rows, K, gpr, o);
  else
    hipLaunchKernelGGL((k_sp_pack<S, false, false>), grid, block, 0, s, src, ld, rows, K, gpr, o);
  return hipGetLastError();
}

hipError_t launch_sp_unpack(const void* sp, int rows, int K, float* dst, hipStream_t s) {
  const int64_t gpr = sp_cols(K) / 8, total = (int64_t)rows * gpr;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sp_unpack, dim3(pack_blocks(total)), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(sp), gpr, rows, K, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// W^T = (L^-1 E^H)^T, written SP with rows m and k = n
// ---------------------------------------------------------------------------
// conj(E) is first written split-packed, a slab of samples at a time (rows m,
// k = n, zero past N), and the product then loads both operands as the R
// product does.  Generating E inside the product's loop (two complex
// multiplies, the split and the table loads per element: 295 vector
// instructions per chunk against the R product's 132) held the bf16 pipe at
// 0.43 busy against R's 0.56; the slab costs one write and one read of
// 8 Np bytes per sample, about 1% of the product.
//
// Slab rows r0 .. r0 + 64 of workgroup b, columns (b % nbc) kGenChunks 32 ..
// for kGenChunks chunks of 32: thread t generates columns 8 (t / 64) .. + 8 of
// row t % 64 of each chunk, as the generated-row loader does for a tile, and
// writes the 64-byte group.
constexpr int kGenChunks = 16;

template <int FEAT, bool AL>
__global__ __launch_bounds__(256) void k_gen_e_sp(EncDev<float> e, int m0, int rows, int64_t gn,
                                                  uint4* __restrict__ Es) {
  typedef B3Cfg Cfg;   // 256 threads, chunks of BK = 32 columns
  const int64_t kp = gn * 8;
  const int nbc = (int)((kp + 32 * kGenChunks - 1) / (32 * kGenChunks));
  const int r0 = (int)(blockIdx.x / nbc) * 64, cb = (int)(blockIdx.x % nbc);
  LoadGenRowSP<Cfg, 64, true, FEAT, AL> g;   // conj(E[m][n]), zero past M and N
  g.init(e, m0 + r0);
  const int o = threadIdx.x % 64, kk0 = (int)(threadIdx.x / 64) * 8;
  const bool live = r0 + o < rows;
  for (int c = 0; c < kGenChunks; ++c) {
    const int k0 = (cb * kGenChunks + c) * 32;
    if (k0 >= kp) break;   // the same for every thread of the workgroup
    g.fetch(k0, e.N);
    g.finish(0, 1);
    if (live) {
      uint4* d = Es + ((int64_t)(r0 + o) * gn + (k0 + kk0) / 8) * 4;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        d[pl] = uint4{g.pk[0][pl][0], g.pk[0][pl][1], g.pk[0][pl][2], g.pk[0][pl][3]};
    }
  }
}

// W^T tiles for samples m0 .. m0 + rows from the slab Es (its rows 0 ..).
__global__ __launch_bounds__(B3Cfg::NT, B3Cfg::MIN_BLOCKS) void k_trmm_w_sp(
    const uint4* __restrict__ Li, const uint4* __restrict__ Es, int64_t gn, int m0, int rows,
    void* __restrict__ W, int N, int M) {
  typedef B3Cfg Cfg;
  const int nbi = (N + Cfg::BM - 1) / Cfg::BM, nbj = (rows + Cfg::BN - 1) / Cfg::BN;
  // as the FP32 product: each XCD runs column groups of 8 sample blocks over
  // every row block, longest K ranges first
  int r, bj;
  grouped_tile<8>(xcd_contiguous(blockIdx.x, nbi * nbj), nbi, nbj, &r, &bj);
  const int bi = nbi - 1 - r;
  LoadSP<Cfg, Cfg::BM> la;   // L^-1 rows n (zero above the diagonal and past N)
  la.p = Li;
  la.gpr = gn;
  la.o0 = bi * Cfg::BM;
  la.oend = N;
  LoadSP<Cfg, Cfg::BN> lb;   // conj(E) rows m of the slab
  lb.p = Es;
  lb.gpr = gn;
  lb.o0 = bj * Cfg::BN;
  lb.oend = rows;
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, min(N, (bi + 1) * Cfg::BM), acc, smem_base<Cfg>());
  // rows N .. Np of W^T's k range come out zero (their L^-1 rows load as zeros)
  acc_store_sp_t<Cfg>(acc, W, gn, bi * Cfg::BM, m0 + bj * Cfg::BN, (int)(gn * 8), M);
}

// ---------------------------------------------------------------------------
// R^T tiles: R^T[m][n] = sum_{n' >= n} W^T[m][n'] conj(Li[n'][n]), written SP
// as R with rows n and k = m
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(B3Cfg::NT, B3Cfg::MIN_BLOCKS) void k_trmm_r_sp(const uint4* __restrict__ W,
                                                   const uint4* __restrict__ Lh, int64_t gn,
                                                   void* __restrict__ R, int64_t gm, int N, int M) {
  typedef B3Cfg Cfg;
  const int nbm = (M + Cfg::BM - 1) / Cfg::BM, nbn = (N + Cfg::BN - 1) / Cfg::BN;
  // each XCD runs groups of 8 sample blocks over every unknown block (so the
  // XCDs' shares of the triangle are equal), the longest K ranges first, and
  // the contraction runs from n' = N down, so resident tiles read the same
  // W^T and L^-H chunks at the same time
  int bn, bm;
  grouped_tile<8>(xcd_contiguous(blockIdx.x, nbm * nbn), nbn, nbm, &bn, &bm);
  LoadSP<Cfg, Cfg::BM> la;   // W^T rows m
  la.p = W;
  la.gpr = gn;
  la.o0 = bm * Cfg::BM;
  la.oend = M;
  LoadSP<Cfg, Cfg::BN> lb;   // L^-H rows n: conj(Li[n'][n]), zero for n' < n
  lb.p = Lh;
  lb.gpr = gn;
  lb.o0 = bn * Cfg::BN;
  lb.oend = N;
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg, true, true>(la, lb, bn * Cfg::BN, N, acc, smem_base<Cfg>());
  // R's k range M .. Mp comes out zero (W^T rows past M load as zeros)
  acc_store_sp_t<Cfg>(acc, R, gm, bm * Cfg::BM, bn * Cfg::BN, (int)(gm * 8), N);
}

hipError_t launch_trmm_w_sp(const EncDev<float>& e, const void* Li, void* W, void* Es,
                            int64_t slab_rows, hipStream_t s) {
  typedef B3Cfg Cfg;
  const int N = e.N, M = e.M;
  if (N <= 0 || M <= 0) return hipSuccess;
  if (slab_rows <= 0 || slab_rows % Cfg::BN != 0) return hipErrorInvalidValue;
  static const hipError_t attr = allow_smem(k_trmm_w_sp, smem_bytes<Cfg>());
  if (attr != hipSuccess) return attr;
  const int64_t gn = sp_cols(N) / 8;
  const int nbc = (int)cdiv(gn * 8, 32 * kGenChunks);
  for (int64_t m0 = 0; m0 < M; m0 += slab_rows) {
    const int rows = (int)std::min<int64_t>(slab_rows, M - m0);
    hipError_t err = with_feat_al(enc_features(e), row_aligned(e, Cfg::BK), [&](auto fc, auto al) {
      hipLaunchKernelGGL((k_gen_e_sp<decltype(fc)::value, decltype(al)::value>),
                         dim3((unsigned)(cdiv(rows, 64) * nbc)), dim3(256), 0, s, e, (int)m0, rows, gn,
                         reinterpret_cast<uint4*>(Es));
      return hipGetLastError();
    });
    if (err != hipSuccess) return err;
    const int tiles = cdiv(N, Cfg::BM) * cdiv(rows, Cfg::BN);
    hipLaunchKernelGGL(k_trmm_w_sp, dim3(tiles), dim3(Cfg::NT), smem_bytes<Cfg>(), s,
                       reinterpret_cast<const uint4*>(Li), reinterpret_cast<const uint4*>(Es), gn,
                       (int)m0, rows, W, N, M);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_trmm_r_sp(const void* W, const void* Lh, void* R, int N, int M, hipStream_t s) {
  typedef B3Cfg Cfg;
  static const hipError_t attr = allow_smem(k_trmm_r_sp, smem_bytes<Cfg>());
  if (attr != hipSuccess) return attr;
  const int tiles = cdiv(N, Cfg::BN) * cdiv(M, Cfg::BM);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_trmm_r_sp, dim3(tiles), dim3(Cfg::NT), smem_bytes<Cfg>(), s,
                     reinterpret_cast<const uint4*>(W), reinterpret_cast<const uint4*>(Lh),
                     sp_cols(N) / 8, R, sp_cols(M) / 8, N, M);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A few frames: stream R's SP rows (HBM-bound), as the FP32 row apply
// ---------------------------------------------------------------------------
// Lane l takes columns 2s and 2s + 1 (s = l % 4) of 8-group l / 4 of each
// 16-group block, as the FP32 row apply takes two columns per lane: it reads
// dword s of each of the group's four planes (the hi and lo halves of both
// columns' real and imaginary parts; the wave's four loads together cover 1 KB
// of the row) and one 16-byte pair of data values per frame (1 KB per wave,
// contiguous).  R = hi + lo is exact in FP32, so the sums are those of the
// FP32 row apply on that R.  Past M, R is zero and the data are read clamped
// (a finite value times zero).  The contraction is sliced over the XCDs as in
// the FP32 row apply (nseg slices of seg_groups 8-groups, partials to
// X[slice][F][N] when nseg > 1).
template <int FM, int RW>
__global__ __launch_bounds__(256) void k_apply_rows_sp(const uint4* __restrict__ R, int64_t gpr,
                                                       const float* __restrict__ D,
                                                       float* __restrict__ X, int N, int M, int F,
                                                       int nseg, int seg_groups) {
  const int lane = threadIdx.x & 63;
  const int sl = lane & 3;
  const int seg = blockIdx.x % nseg;
  const int n0 = ((blockIdx.x / nseg) * 4 + (int)(threadIdx.x >> 6)) * RW;
  if (n0 >= N) return;   // the whole wavefront leaves; no barrier follows
  const int64_t g_lo = (int64_t)seg * seg_groups, g_hi = std::min<int64_t>(gpr, g_lo + seg_groups);
  const uint32_t* r[RW];
#pragma unroll
  for (int j = 0; j < RW; ++j)   // rows past N re-read row N-1 and are not written
    r[j] = reinterpret_cast<const uint32_t*>(R + (int64_t)min(n0 + j, N - 1) * gpr * 4);
  const cx<float>* d = reinterpret_cast<const cx<float>*>(D);
  float ar[RW][FM], ai[RW][FM];
#pragma unroll
  for (int j = 0; j < RW; ++j)
#pragma unroll
    for (int f = 0; f < FM; ++f) ar[j][f] = ai[j][f] = 0.f;
  for (int64_t g = g_lo + (lane >> 2); g < g_hi; g += 16) {
    float rr[RW][2], ri[RW][2];
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      const uint32_t* q = r[j] + g * 16 + sl;   // dword sl of planes 0..3
      const uint32_t h = q[0], l = q[4], ih = q[8], il = q[12];
      rr[j][0] = join2(h, l, 0);
      rr[j][1] = join2(h, l, 1);
      ri[j][0] = join2(ih, il, 0);
      ri[j][1] = join2(ih, il, 1);
    }
    const int64_t m0 = std::min<int64_t>(g * 8 + 2 * sl, M - 1), m1 = std::min<int64_t>(g * 8 + 2 * sl + 1, M - 1);
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      if (f >= F) break;
      const cx<float> d0 = d[(int64_t)f * M + m0], d1 = d[(int64_t)f * M + m1];
#pragma unroll
      for (int j = 0; j < RW; ++j) {
        ar[j][f] += d0.re * rr[j][0] - d0.im * ri[j][0];
        ai[j][f] += d0.re * ri[j][0] + d0.im * rr[j][0];
        ar[j][f] += d1.re * rr[j][1] - d1.im * ri[j][1];
        ai[j][f] += d1.re * ri[j][1] + d1.im * rr[j][1];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RW; ++j)
#pragma unroll
    for (int f = 0; f < FM; ++f) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        ar[j][f] += __shfl_xor(ar[j][f], off);
        ai[j][f] += __shfl_xor(ai[j][f], off);
      }
    }
  if (lane == 0) {
    cx<float>* x = reinterpret_cast<cx<float>*>(X) + (size_t)seg * F * N;
#pragma unroll
    for (int j = 0; j < RW; ++j)
#pragma unroll
      for (int f = 0; f < FM; ++f)
        if (f < F && n0 + j < N) x[(size_t)f * N + n0 + j] = cx<float>{ar[j][f], ai[j][f]};
  }
}

// X = sum_s P[s] over the slices, in slice order (n complex64 values each).
__global__ __launch_bounds__(256) void k_rows_reduce_sp(const float* __restrict__ P, int nseg,
                                                        int64_t n, float* __restrict__ X) {
  const cx<float>* p = reinterpret_cast<const cx<float>*>(P);
  cx<float>* x = reinterpret_cast<cx<float>*>(X);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float zr = p[i].re, zi = p[i].im;
    for (int s = 1; s < nseg; ++s) {
      zr += p[(int64_t)s * n + i].re;
      zi += p[(int64_t)s * n + i].im;
    }
    x[i] = cx<float>{zr, zi};
  }
}

hipError_t launch_apply_rows_sp(const void* R, const float* D, float* X, int N, int M, int F,
                                Scratch& sc, hipStream_t s) {
  if (F <= 0 || N <= 0) return hipSuccess;
  if (F > kRowApplyMaxF) return hipErrorInvalidValue;
  const uint4* r = reinterpret_cast<const uint4*>(R);
  const int64_t gpr = sp_cols(M) / 8;
  const int nseg = row_slices(M);
  // slice length: a multiple of one wave-wide pass (16 groups of 8)
  const int seg_groups = nseg > 1 ? cdiv(cdiv(gpr, nseg), 16) * 16 : (int)gpr;
  void* P = nullptr;
  if (nseg > 1) {
    const hipError_t e = sc.get(&P, apply_rows_scratch_bytes<float>(F, N, M), s);
    if (e != hipSuccess) return e;
  }
  float* out = nseg > 1 ? (float*)P : X;
  auto go = [&](auto fm, auto rw) {
    constexpr int FM = decltype(fm)::value, RW = decltype(rw)::value;
    hipLaunchKernelGGL((k_apply_rows_sp<FM, RW>), dim3(cdiv(N, 4 * RW) * nseg), dim3(256), 0, s, r,
                       gpr, D, out, N, M, F, nseg, seg_groups);
    return hipGetLastError();
  };
  using std::integral_constant;
  hipError_t e;
  if (F <= 1) e = go(integral_constant<int, 1>(), integral_constant<int, 1>());
  else if (F <= 2) e = go(integral_constant<int, 2>(), integral_constant<int, 4>());
  else if (F <= 4) e = go(integral_constant<int, 4>(), integral_constant<int, 4>());
  else e = go(integral_constant<int, 8>(), integral_constant<int, 4>());
  if (nseg > 1) {
    if (e == hipSuccess) {
      const int64_t n = (int64_t)F * N;
      hipLaunchKernelGGL(k_rows_reduce_sp, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 4096)),
                         dim3(256), 0, s, (const float*)P, nseg, n, X);
      e = hipGetLastError();
    }
    const hipError_t f = sc.put(P, s);
    if (e == hipSuccess) e = f;
  }
  return e;
}

template hipError_t launch_sp_pack<float>(const float*, int64_t, int, int, bool, bool, void*,
                                          hipStream_t);
template hipError_t launch_sp_pack<double>(const double*, int64_t, int, int, bool, bool, void*,
                                           hipStream_t);

}  // namespace pinv
