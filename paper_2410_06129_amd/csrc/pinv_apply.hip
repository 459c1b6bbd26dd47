// Apply image = R data for every frame (Eq. 3), grouped over plans, and the
// row-streaming apply for a few frames.
#include <type_traits>

#include "pinv_internal.h"

namespace pinv {

// ---------------------------------------------------------------------------
// Apply (grouped): for each item, X[f][n] = sum_m D[f][m] R[n][m]
// ---------------------------------------------------------------------------
// An item whose tile grid alone would leave the GPU partly idle is split over
// M (the split depends only on the item's F, N and M, so a result is the same
// alone and in any group); its splits write partial tiles to item.work and
// k_apply_reduce adds them in split order.
//
// Tiles run frame-tile fastest and each XCD takes a contiguous range of them,
// so the F/BM tiles that read one BN-row panel of R are resident together on
// one XCD and share its L2.
//
// SEG: the contraction runs in segments of kApplySegRows rows; each segment's
// accumulators are folded into a second FP32 accumulator set.  A running FP32
// sum over L terms carries a relative rounding error growing like sqrt(L), so
// over M = 262144 rows (32768 k-steps) an R exact to its FP32 rounding gave
// 1.5e-5; segments of 4096 rows keep each running sum 8 times shorter.
constexpr int kApplySegRows = 4096;

template <class Cfg> struct ApplyMinBlocks { static constexpr int value = 1; };
template <int BM, int BN, int WGM, int WGN, int ST>
struct ApplyMinBlocks<TileCfgB3<BM, BN, WGM, WGN, ST>> { static constexpr int value = TileCfgB3<BM, BN, WGM, WGN, ST>::MIN_BLOCKS; };

template <class Cfg, bool SEG = false>
__global__ __launch_bounds__(Cfg::NT, ApplyMinBlocks<Cfg>::value) void k_apply(const ApplyBatch batch) {
  typedef typename Cfg::T T;
  // locate the item owning this tile (items carry exclusive tile prefix sums)
  int lo = 0, hi = batch.n - 1;
  const int t = xcd_contiguous(blockIdx.x, gridDim.x);
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (batch.it[mid].tile0 <= t) lo = mid; else hi = mid - 1;
  }
  const ApplyItemDev it = batch.it[lo];
  const int u0 = t - it.tile0;
  const int split = u0 / it.ntile;
  const int u = u0 - split * it.ntile;
  const int nbi = (it.F + Cfg::BM - 1) / Cfg::BM;
  const int bi = u % nbi, bj = u / nbi;
  const int k0 = split * it.kchunk, k1 = min(it.M, k0 + it.kchunk);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  if constexpr (IsB3<Cfg>::value) {
    // split-precision items: D and R split-packed, it.M their padded row length
    cx<T>* O = it.splits > 1
                   ? reinterpret_cast<cx<T>*>(it.work) + (size_t)split * it.F * it.N
                   : reinterpret_cast<cx<T>*>(it.X);
    LoadSP<Cfg, Cfg::BM> la;   // D rows f
    la.p = reinterpret_cast<const uint4*>(it.D);
    la.gpr = it.M / 8;
    la.o0 = r0;
    la.oend = it.F;
    LoadSP<Cfg, Cfg::BN> lb;   // R rows n
    lb.p = reinterpret_cast<const uint4*>(it.R);
    lb.gpr = it.M / 8;
    lb.o0 = c0;
    lb.oend = it.N;
    AccTile<Cfg> acc;
    acc.zero();
    mainloop<Cfg>(la, lb, k0, k1, acc, smem_base<Cfg>());
    acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
      const int row = r0 + r, col = c0 + c;
      if (row < it.F && col < it.N) O[(size_t)row * it.N + col] = cx<T>{re, im};
    });
    return;
  } else {
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;   // D[f][m]
  la.p = reinterpret_cast<const cx<T>*>(it.D);
  la.ld = it.M;
  la.o0 = bi * Cfg::BM;
  la.oend = it.F;
  LoadDenseKC<Cfg, Cfg::BN, Cfg::LDB, T, false> lb;   // R[n][m]
  lb.p = reinterpret_cast<const cx<T>*>(it.R);
  lb.ld = it.M;
  lb.o0 = bj * Cfg::BN;
  lb.oend = it.N;
  AccTile<Cfg> acc;
  cx<T>* O = it.splits > 1
                 ? reinterpret_cast<cx<T>*>(it.work) + (size_t)split * it.F * it.N
                 : reinterpret_cast<cx<T>*>(it.X);
  if constexpr (SEG) {
    typename Acc<T>::type ore[Cfg::MB][Cfg::NB], oim[Cfg::MB][Cfg::NB];
#pragma unroll
    for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
      for (int b = 0; b < Cfg::NB; ++b) ore[a][b] = oim[a][b] = typename Acc<T>::type{0, 0, 0, 0};
    int ks = k0;
    do {
      const int ke = min(k1, ks + kApplySegRows);
      acc.zero();
      mainloop<Cfg>(la, lb, ks, ke, acc, smem_base<Cfg>());
      acc_fold<Cfg>(acc, ore, oim);
      ks = ke;
    } while (ks < k1);
    acc_foreach_outer<Cfg>(ore, oim, [&](int r, int c, T re, T im) {
      const int row = r0 + r, col = c0 + c;
      if (row < it.F && col < it.N) O[(size_t)row * it.N + col] = cx<T>{re, im};
    });
    return;
  }
  acc.zero();
  mainloop<Cfg>(la, lb, k0, k1, acc, smem_base<Cfg>());
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < it.F && col < it.N) O[(size_t)row * it.N + col] = cx<T>{re, im};
  });
  }
}

// X = sum_s work[s] in split order, for the split items of a grouped apply
// (blockIdx.y = item).
template <typename T>
__global__ __launch_bounds__(256) void k_apply_reduce(const ApplyBatch batch) {
  const ApplyItemDev& it = batch.it[blockIdx.y];
  if (it.splits <= 1) return;
  const int64_t n = (int64_t)it.F * it.N;
  const cx<T>* W = reinterpret_cast<const cx<T>*>(it.work);
  cx<T>* X = reinterpret_cast<cx<T>*>(it.X);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double zr = W[i].re, zi = W[i].im;   // partials added in FP64, rounded once
    for (int s = 1; s < it.splits; ++s) {
      zr += W[(int64_t)s * n + i].re;
      zi += W[(int64_t)s * n + i].im;
    }
    X[i] = cx<T>{T(zr), T(zi)};
  }
}


// streaming RW rows of R.  At small F each element of R feeds only F
// multiply-adds, so the apply is bound by memory bandwidth, not by MFMA: rows
// stream through wide coalesced loads (two complex64 per lane and load when
// VEC = 2), and each data element loaded serves RW rows.  Every wave reduces
// its lane partial sums in a fixed butterfly order, so a result depends only
// on its own row and frame.
//
// The contraction over M is cut into `nseg` slices (kRowSlices = one per XCD
// for long rows): workgroup b takes slice b % nseg, and the dispatcher deals
// workgroups round-robin over the XCDs, so every XCD streams one slice of
// every row of R and its L2 holds that slice of the data, which the waves on
// the XCD re-read for their rows.  With nseg > 1 each slice writes its partial
// images to P[slice][F][N] and k_rows_reduce adds them in slice order.
template <typename T, int FM, int RW, int VEC>
__global__ __launch_bounds__(256) void k_apply_rows(const T* __restrict__ R, const T* __restrict__ D,
                                                    T* __restrict__ X, int N, int M, int F, int nseg,
                                                    int seg_len) {
  const int lane = threadIdx.x & 63;
  const int seg = blockIdx.x % nseg;
  const int n0 = ((blockIdx.x / nseg) * 4 + (int)(threadIdx.x >> 6)) * RW;
  if (n0 >= N) return;   // the whole wavefront leaves; no barrier follows
  const int m_lo = seg * seg_len, m_hi = min(M, m_lo + seg_len);
  const cx<T>* r[RW];
#pragma unroll
  for (int j = 0; j < RW; ++j)   // rows past N re-read row N-1 and are not written
    r[j] = reinterpret_cast<const cx<T>*>(R) + (size_t)min(n0 + j, N - 1) * M;
  const cx<T>* d = reinterpret_cast<const cx<T>*>(D);
  T ar[RW][FM], ai[RW][FM];
#pragma unroll
  for (int j = 0; j < RW; ++j)
#pragma unroll
    for (int f = 0; f < FM; ++f) ar[j][f] = ai[j][f] = T(0);
  for (int m0 = m_lo + lane * VEC; m0 < m_hi; m0 += 64 * VEC) {
    cx<T> rv[RW][VEC];
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      if constexpr (VEC == 2) {
        // M even, slices of even length and 16-byte aligned rows (checked by
        // the launcher): m0 + 1 < m_hi
        const float4 q = *reinterpret_cast<const float4*>(r[j] + m0);
        rv[j][0] = cx<T>{q.x, q.y};
        rv[j][1] = cx<T>{q.z, q.w};
      } else {
        rv[j][0] = r[j][m0];
      }
    }
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      if (f >= F) break;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const cx<T> dv = d[(size_t)f * M + m0 + v];
#pragma unroll
        for (int j = 0; j < RW; ++j) {
          ar[j][f] += dv.re * rv[j][v].re - dv.im * rv[j][v].im;
          ai[j][f] += dv.re * rv[j][v].im + dv.im * rv[j][v].re;
        }
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
    cx<T>* x = reinterpret_cast<cx<T>*>(X) + (size_t)seg * F * N;
#pragma unroll
    for (int j = 0; j < RW; ++j)
#pragma unroll
      for (int f = 0; f < FM; ++f)
        if (f < F && n0 + j < N) x[(size_t)f * N + n0 + j] = cx<T>{ar[j][f], ai[j][f]};
  }
}

// X = sum_s P[s] over the slices, in slice order (n complex values each).
template <typename T>
__global__ __launch_bounds__(256) void k_rows_reduce(const T* __restrict__ P, int nseg, int64_t n,
                                                     T* __restrict__ X) {
  const cx<T>* p = reinterpret_cast<const cx<T>*>(P);
  cx<T>* x = reinterpret_cast<cx<T>*>(X);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T zr = p[i].re, zi = p[i].im;
    for (int s = 1; s < nseg; ++s) {
      zr += p[(int64_t)s * n + i].re;
      zi += p[(int64_t)s * n + i].im;
    }
    x[i] = cx<T>{zr, zi};
  }
}


// ---------------------------------------------------------------------------
// 5 to 32 frames: R streamed into the matrix cores through transposing LDS
// tiles
// ---------------------------------------------------------------------------
// Between a few and 32 frames an apply still reads R once (8NM bytes) but
// does up to 32 complex multiply-adds per element read, more than the VALU
// row kernel keeps up with.  Each wave takes 16 NB rows of R; on
// v_mfma_f32_16x16x4f32 an image block is X^T (16 frames x 16 rows of R),
// A = D (frames x k), B = R^T (k x rows), and lane (j = l % 16, q = l / 16)
// supplies k-slot q of row (or frame) j.  The operand layout puts 16 rows in
// every wave-wide access, and loads of that shape (64 bytes from each of 16
// rows) stream at 0.59 of HBM where loads of four rows x 256 bytes stream at
// 0.77 (pure reads at N = 16384, M = 262144).  So R is loaded in the second
// shape, 32 columns (256 bytes) per row and chunk, stored to a wave-private
// LDS tile (rows of 256 bytes plus 16 of padding, so the 16 rows a fragment
// read touches fall in distinct banks) and read back in the operand layout:
// lane (j, q) reads columns 8q .. 8q + 7 of row j, and MFMA step u pairs
// slot q with column 8q + u.  A wave's own LDS operations run in order, so
// its R tile needs no barrier.  The data chunk (16 FB frames x 32 columns) is
// the same for the workgroup's four waves: each loads a quarter of it into a
// shared, double-buffered LDS tile, with one barrier per chunk.  Two chunks
// of R are in flight while one computes.  Frames past F and rows past N
// re-read frame F-1 and row N-1 and are not written (waves past N still
// load their share of the data and take the barriers); columns past a
// slice's end count as zero.  VEC: complex values per load (2 when M is even
// and the rows 16-byte aligned, else 1).  FORM: the plan's complex-product
// form on FP32 operands (kForm4M, kForm3M), or kFormB3 for split-packed R and
// data (BF16X3 plans): there each 64-byte group of a row holds the bf16
// planes re_hi, re_lo, im_hi, im_lo of 8 columns, so the same 256-byte row
// pieces and the same fragment reads give a lane the four planes of its
// 8-group q, one v_mfma_f32_16x16x32_bf16 step per chunk and plane pair
// (hi*hi + hi*lo + lo*hi per real product).  Split-packed rows are padded to
// whole chunks (zeros past M), so those slices have no partial chunk.
//
// Slices: the contraction is cut into nseg slices of at most
// kStreamSliceCols columns (nseg a multiple of 8, or 1 for short rows).
// Workgroup b runs on XCD b % 8 and takes row block (b / 8) % nrb of slice
// 8 (b / (8 nrb)) + b % 8, so each XCD works through its slices one after
// another with all row blocks of a slice together, and its L2 holds that
// slice of the data (at most 32 frames x 4096 columns, 1 MB).  Slice partials
// go to P[slice][F][N] and k_rows_reduce adds them in slice order; a running
// FP32 sum so covers at most 4096 columns, as in the segmented tiles.
constexpr int kStreamSliceCols = 4096;
constexpr int kForm4M = 0, kForm3M = 1, kFormB3 = 2;

typedef float f32x4v __attribute__((ext_vector_type(4)));

template <int FB, int NB, int VEC, int FORM>
__global__ __launch_bounds__(256) void k_apply_stream(const float* __restrict__ R,
                                                      const float* __restrict__ D,
                                                      float* __restrict__ X, int N, int M, int F,
                                                      int nseg, int seg_len, int nrb) {
  constexpr int L = 32;                 // columns per chunk
  constexpr int ROWB = 272;             // LDS bytes per row
  constexpr int RPI = 2 * VEC;          // rows per wave-wide load
  constexpr int LPR = 32 / VEC;         // lanes per row in a load
  constexpr int GI = 16 / RPI;          // loads per 16-row block of R
  constexpr int DI = 4 * FB / RPI;      // data loads per wave (its 4 FB frames)
  typedef typename std::conditional<VEC == 2, f32x4v, f32x2v>::type VT;
  __shared__ __attribute__((aligned(16))) char rtiles[4][16 * NB * ROWB];
  __shared__ __attribute__((aligned(16))) char dtile[2][16 * FB * ROWB];
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
  const int j = lane & 15, q = lane >> 4;
  int seg = 0, rb = blockIdx.x;
  if (nseg > 1) {
    const int t = blockIdx.x / kXcds;
    seg = (t / nrb) * kXcds + (int)(blockIdx.x % kXcds);
    rb = t % nrb;
  }
  const int n0 = (rb * 4 + w) * 16 * NB;
  const int m_lo = seg * seg_len;
  const int m_hi = min(M, m_lo + seg_len);
  char* const tile = rtiles[w];
  // load lanes: row RPI i + l / LPR, chunk columns VEC (l % LPR) ..
  const int lrow = lane / LPR, lcol = VEC * (lane % LPR);
  const cx<float>* grow[NB][GI];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < GI; ++i)
      grow[b][i] = reinterpret_cast<const cx<float>*>(R) +
                   (size_t)min(n0 + 16 * b + RPI * i + lrow, N - 1) * M + lcol;
  const cx<float>* dsrc[DI];
#pragma unroll
  for (int i = 0; i < DI; ++i)
    dsrc[i] = reinterpret_cast<const cx<float>*>(D) +
              (size_t)min(4 * FB * w + RPI * i + lrow, F - 1) * M + lcol;

  struct Raw { VT v[NB][GI]; };        // R as loaded
  struct DRaw { VT v[DI]; };           // the wave's quarter of the data
  struct Frag { f32x4v v[NB][4]; };    // R, operand layout
  struct DFrag { f32x4v v[FB][4]; };   // data, operand layout
  // TAIL: the slice's last, partial chunk (columns at or past m_hi read
  // column m_hi - VEC, a whole load, and count as zero)
  auto gload = [&](Raw& g, int m0, auto tail) __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < GI; ++i) {
        if constexpr (decltype(tail)::value) {
          const bool in = m0 + lcol < m_hi;
          const VT v = *reinterpret_cast<const VT*>(grow[b][i] + (in ? m0 : m_hi - VEC - lcol));
          g.v[b][i] = in ? v : VT{};
        } else {
          g.v[b][i] = *reinterpret_cast<const VT*>(grow[b][i] + m0);
        }
      }
  };
  auto dload = [&](DRaw& d, int m0, auto tail) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < DI; ++i) {
      if constexpr (decltype(tail)::value) {
        const bool in = m0 + lcol < m_hi;
        const VT v = *reinterpret_cast<const VT*>(dsrc[i] + (in ? m0 : m_hi - VEC - lcol));
        d.v[i] = in ? v : VT{};
      } else {
        d.v[i] = *reinterpret_cast<const VT*>(dsrc[i] + m0);
      }
    }
  };
  auto lwrite = [&](const Raw& g) __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < GI; ++i)
        *reinterpret_cast<VT*>(tile + (16 * b + RPI * i + lrow) * ROWB + 8 * lcol) = g.v[b][i];
  };
  auto lread = [&](Frag& r) __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        r.v[b][p] = *reinterpret_cast<const f32x4v*>(tile + (16 * b + j) * ROWB + 64 * q + 16 * p);
  };
  auto dwrite = [&](const DRaw& d, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < DI; ++i)
      *reinterpret_cast<VT*>(dtile[buf] + (4 * FB * w + RPI * i + lrow) * ROWB + 8 * lcol) = d.v[i];
  };
  auto dread = [&](DFrag& df, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        df.v[a][p] = *reinterpret_cast<const f32x4v*>(dtile[buf] + (16 * a + j) * ROWB + 64 * q + 16 * p);
  };
  // 4M: re = dr rr - di ri, im = dr ri + di rr.  3M: t1 = dr rr, t2 = di ri,
  // t3 = (dr + di)(rr + ri); re = t1 - t2, im = t3 - t1 - t2.  B3: as 4M,
  // each real product split.
  f32x4 acc[FORM == kForm3M ? 3 : 2][FB][NB];
#pragma unroll
  for (int t = 0; t < (FORM == kForm3M ? 3 : 2); ++t)
#pragma unroll
    for (int a = 0; a < FB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[t][a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  auto compute = [&](const Frag& r, const DFrag& d) __attribute__((always_inline)) {
    if constexpr (FORM == kFormB3) {
#pragma unroll
      for (int a = 0; a < FB; ++a) {
        const bf16x8 arh = __builtin_bit_cast(bf16x8, d.v[a][0]);
        const bf16x8 arl = __builtin_bit_cast(bf16x8, d.v[a][1]);
        const bf16x8 aih = __builtin_bit_cast(bf16x8, d.v[a][2]);
        const bf16x8 ail = __builtin_bit_cast(bf16x8, d.v[a][3]);
        const bf16x8 naih = neg_b16(aih), nail = neg_b16(ail);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const bf16x8 brh = __builtin_bit_cast(bf16x8, r.v[b][0]);
          const bf16x8 brl = __builtin_bit_cast(bf16x8, r.v[b][1]);
          const bf16x8 bih = __builtin_bit_cast(bf16x8, r.v[b][2]);
          const bf16x8 bil = __builtin_bit_cast(bf16x8, r.v[b][3]);
          f32x4 cr = acc[0][a][b], ci = acc[1][a][b];
          cr = mfma_b16(arh, brh, cr);
          cr = mfma_b16(arh, brl, cr);
          cr = mfma_b16(arl, brh, cr);
          cr = mfma_b16(naih, bih, cr);
          cr = mfma_b16(naih, bil, cr);
          cr = mfma_b16(nail, bih, cr);
          ci = mfma_b16(arh, bih, ci);
          ci = mfma_b16(arh, bil, ci);
          ci = mfma_b16(arl, bih, ci);
          ci = mfma_b16(aih, brh, ci);
          ci = mfma_b16(aih, brl, ci);
          ci = mfma_b16(ail, brh, ci);
          acc[0][a][b] = cr;
          acc[1][a][b] = ci;
        }
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int a = 0; a < FB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const float rr = r.v[b][u / 2][2 * (u % 2)], ri = r.v[b][u / 2][2 * (u % 2) + 1];
          const float dr = d.v[a][u / 2][2 * (u % 2)], di = d.v[a][u / 2][2 * (u % 2) + 1];
          if constexpr (FORM == kForm3M) {
            acc[0][a][b] = mfma4(dr, rr, acc[0][a][b]);
            acc[1][a][b] = mfma4(di, ri, acc[1][a][b]);
            acc[2][a][b] = mfma4(dr + di, rr + ri, acc[2][a][b]);
          } else {
            acc[0][a][b] = mfma4(dr, rr, acc[0][a][b]);
            acc[0][a][b] = mfma4(-di, ri, acc[0][a][b]);
            acc[1][a][b] = mfma4(dr, ri, acc[1][a][b]);
            acc[1][a][b] = mfma4(di, rr, acc[1][a][b]);
          }
        }
  };
  typedef std::false_type Full;
  typedef std::true_type Tail;
  // every wave of the workgroup has the same slice, so the same chunk count
  // and the same barriers
  const int nfull = m_hi > m_lo ? (m_hi - m_lo) / L : 0;
  auto at = [&](int k) { return m_lo + min(k, nfull - 1) * L; };
  Frag rf;
  DFrag df;
  if (nfull > 0) {
    Raw ga, gb;
    DRaw xa, xb;
    gload(ga, at(0), Full());
    dload(xa, at(0), Full());
    gload(gb, at(1), Full());
    dload(xb, at(1), Full());
    dwrite(xa, 0);
    __syncthreads();
    dload(xa, at(2), Full());
    // Two chunks per pass; chunk k computes from R in ga (gb) and data in
    // buffer k % 2 while chunk k + 1's data goes to the other buffer.  Each
    // barrier publishes that write and retires every wave's reads of the
    // buffer the next half overwrites.  The loop's only exit is at the
    // bottom (an exit between a load and its use let the compiler sink the
    // load past it); the scheduling barriers keep each chunk's loads ahead
    // of the previous chunk's products.  The last passes re-load the final
    // chunk, unused.
    int k = 0;
    for (; k + 2 <= nfull; k += 2) {
      lwrite(ga);
      lread(rf);
      dread(df, 0);
      dwrite(xb, 1);
      gload(ga, at(k + 2), Full());
      dload(xb, at(k + 3), Full());
      __syncthreads();
      compute(rf, df);
      lwrite(gb);
      lread(rf);
      dread(df, 1);
      dwrite(xa, 0);
      gload(gb, at(k + 3), Full());
      dload(xa, at(k + 4), Full());
      __syncthreads();
      compute(rf, df);
    }
    if (k < nfull) {   // odd count: the last chunk's R is in ga, its data in buffer 0
      lwrite(ga);
      lread(rf);
      dread(df, 0);
      compute(rf, df);
    }
  }
  const int mt = m_lo + nfull * L;
  if (mt < m_hi) {
    Raw g;
    DRaw x;
    gload(g, mt, Tail());
    dload(x, mt, Tail());
    __syncthreads();   // every wave's reads of the data buffers are done
    dwrite(x, 0);
    lwrite(g);
    __syncthreads();
    lread(rf);
    dread(df, 0);
    compute(rf, df);
  }
  cx<float>* out = reinterpret_cast<cx<float>*>(X) + (size_t)seg * F * N;
#pragma unroll
  for (int a = 0; a < FB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = 16 * a + 4 * q + r, n = n0 + 16 * b + j;
        float re, im;
        if constexpr (FORM == kForm3M) {
          re = acc[0][a][b][r] - acc[1][a][b][r];
          im = acc[2][a][b][r] - acc[0][a][b][r] - acc[1][a][b][r];
        } else {
          re = acc[0][a][b][r];
          im = acc[1][a][b][r];
        }
        if (f < F && n < N) out[(size_t)f * N + n] = cx<float>{re, im};
      }
}

// host launchers
// The apply uses the same 128x64 3M tiles as the triangular products: with
// the raised wave priority over the matrix products, their occupancy of two
// workgroups per CU beats 128x128 at one (7.76 against 8.04 ms at 1000
// frames, N = 4096, M = 32768; without the priority raise 128x128 had been
// ahead, 8.1 against 8.3 ms).
// Tile shapes by element type and complex-product form (FP32 applies of at
// most 32 frames stream instead, k_apply_stream).
template <typename T, bool M3> struct ApplyCfgOf;
template <> struct ApplyCfgOf<float, true> { typedef F32Cfg many; };
template <> struct ApplyCfgOf<float, false> { typedef F32Cfg4 many; };
template <> struct ApplyCfgOf<double, true> { typedef F64Cfg3 many; };
template <> struct ApplyCfgOf<double, false> { typedef F64Cfg many; };
// A grouped apply of few frames has few tiles, so its contraction may be split
// up to 16 ways (the other split launches stop at 4).
constexpr int kApplyMaxSplit = 16;

// An item's tiles, contraction split and split length: a function of its own
// F, N and M (and the tile kernel's occupancy) only, so a result is the same
// alone and in any group.
template <class Cfg> static void plan_item(ApplyItemDev& it, int slots) {
  const int nchunks = cdiv(it.M, Cfg::BK);
  it.ntile = cdiv(it.F, Cfg::BM) * cdiv(it.N, Cfg::BN);
  it.splits = pick_split(it.ntile, slots, nchunks, kApplyMaxSplit);
  it.kchunk = cdiv(nchunks, it.splits) * Cfg::BK;
}

template <class Cfg, bool SEG> static int apply_slots() {
  static const hipError_t attr = allow_smem(k_apply<Cfg, SEG>, smem_bytes<Cfg>());
  (void)attr;
  return resident_blocks(k_apply<Cfg, SEG>, Cfg::NT, smem_bytes<Cfg>());
}

template <class Cfg, bool SEG> static size_t item_work_bytes(int F, int N, int M) {
  ApplyItemDev it{};
  it.F = F;
  it.N = N;
  it.M = M;
  plan_item<Cfg>(it, apply_slots<Cfg, SEG>());
  return it.splits > 1 ? (size_t)it.splits * F * N * 2 * sizeof(typename Cfg::T) : 0;
}

// Grouped apply with per-item contraction splits: sets each item's split,
// tile range and partial-sum workspace, runs the tiles, then the reduction.
template <class Cfg, bool SEG = false>
static hipError_t run_apply(ApplyBatch b, Scratch& sc, hipStream_t s) {
  typedef typename Cfg::T T;
  const int slots = apply_slots<Cfg, SEG>();
  int tiles = 0, nsplit = 0;
  size_t work_elems = 0;
  for (int i = 0; i < b.n; ++i) {
    ApplyItemDev& it = b.it[i];
    plan_item<Cfg>(it, slots);
    it.tile0 = tiles;
    it.work = nullptr;
    tiles += it.ntile * it.splits;
    if (it.splits > 1) {
      work_elems += (size_t)it.splits * it.F * it.N;
      ++nsplit;
    }
  }
  if (tiles <= 0) return hipSuccess;
  void* work = nullptr;
  if (nsplit) {
    hipError_t err = sc.get(&work, work_elems * 2 * sizeof(T), s);
    if (err != hipSuccess) return err;
    size_t off = 0;
    for (int i = 0; i < b.n; ++i)
      if (b.it[i].splits > 1) {
        b.it[i].work = (cx<T>*)work + off;
        off += (size_t)b.it[i].splits * b.it[i].F * b.it[i].N;
      }
  }
  hipLaunchKernelGGL((k_apply<Cfg, SEG>), dim3(tiles), dim3(Cfg::NT), smem_bytes<Cfg>(), s, b);
  hipError_t err = hipGetLastError();
  if (nsplit) {
    if (err == hipSuccess) {
      hipLaunchKernelGGL(k_apply_reduce<T>, dim3(1024, b.n), dim3(256), 0, s, b);
      err = hipGetLastError();
    }
    const hipError_t ferr = sc.put(work, s);
    if (err == hipSuccess) err = ferr;
  }
  return err;
}

template <typename T, bool M3, bool SEG>
static hipError_t apply_form(const ApplyBatch& b, Scratch& sc, hipStream_t s) {
  typedef ApplyCfgOf<T, M3> C;
  if constexpr (std::is_same<T, float>::value) {
    // items go to the tile shape their own frame count selects, so an item's
    // result does not depend on the other items of the group
    ApplyBatch many;
    many.n = 0;
    for (int i = 0; i < b.n; ++i) {
      const ApplyItemDev& it = b.it[i];
      if (it.F <= kStreamMaxF) {
        const hipError_t err = launch_apply_stream((const float*)it.R, (const float*)it.D,
                                                   (float*)it.X, it.N, it.M, it.F, M3, sc, s);
        if (err != hipSuccess) return err;
      } else {
        many.it[many.n++] = it;
      }
    }
    return many.n ? run_apply<typename C::many, SEG>(many, sc, s) : hipSuccess;
  } else {
    return run_apply<typename C::many, SEG>(b, sc, s);
  }
}

template <typename T>
hipError_t launch_apply(const ApplyBatch& b, bool m3, bool seg, Scratch& sc, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (seg) return m3 ? apply_form<T, true, true>(b, sc, s) : apply_form<T, false, true>(b, sc, s);
  }
  return m3 ? apply_form<T, true, false>(b, sc, s) : apply_form<T, false, false>(b, sc, s);
}

template <typename T>
size_t apply_scratch_bytes(int F, int N, int M, bool m3, bool seg) {
  auto go = [&](auto form, auto sg) -> size_t {
    typedef ApplyCfgOf<T, decltype(form)::value> C;
    constexpr bool S = std::is_same<T, float>::value && decltype(sg)::value;
    if (std::is_same<T, float>::value && F <= kStreamMaxF) return apply_stream_scratch_bytes(F, N, M);
    return item_work_bytes<typename C::many, S>(F, N, M);
  };
  if (seg)
    return m3 ? go(std::true_type{}, std::true_type{}) : go(std::false_type{}, std::true_type{});
  return m3 ? go(std::true_type{}, std::false_type{}) : go(std::false_type{}, std::false_type{});
}

// Slices of the row apply's contraction: one per XCD when rows are long
// enough that a slice still spans several wave-wide passes, else one.
int row_slices(int M) { return M >= kRowSliceMinM ? kXcds : 1; }

template <typename T>
size_t apply_rows_scratch_bytes(int F, int N, int M) {
  const int nseg = row_slices(M);
  return nseg > 1 ? (size_t)nseg * F * N * 2 * sizeof(T) : 0;
}

template <typename T>
hipError_t launch_apply_rows(const T* R, const T* D, T* X, int N, int M, int F, Scratch& sc,
                             hipStream_t s) {
  if (F <= 0 || N <= 0) return hipSuccess;
  if (F > kRowApplyMaxF) return hipErrorInvalidValue;
  const bool vec = M % 2 == 0 && ((uintptr_t)R % 16) == 0 && ((uintptr_t)D % 16) == 0;
  const int nseg = row_slices(M);
  // slice length: a multiple of one wave-wide pass (128 complex values)
  const int seg_len = nseg > 1 ? cdiv(cdiv(M, nseg), 128) * 128 : M;
  void* P = nullptr;
  if (nseg > 1) {
    const hipError_t e = sc.get(&P, apply_rows_scratch_bytes<T>(F, N, M), s);
    if (e != hipSuccess) return e;
  }
  T* out = nseg > 1 ? (T*)P : X;
  auto go = [&](auto fm, auto rw) {
    constexpr int FM = decltype(fm)::value, RW = decltype(rw)::value;
    const dim3 grid(cdiv(N, 4 * RW) * nseg), block(256);
    if constexpr (sizeof(T) == 4) {
      if (vec) {
        hipLaunchKernelGGL((k_apply_rows<T, FM, RW, 2>), grid, block, 0, s, R, D, out, N, M, F, nseg,
                           seg_len);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_apply_rows<T, FM, RW, 1>), grid, block, 0, s, R, D, out, N, M, F, nseg,
                       seg_len);
    return hipGetLastError();
  };
  // rows per wave: as many as keep the accumulators (2 FM RW values) within
  // 64 registers
  using std::integral_constant;
  constexpr int W = sizeof(T) == 4 ? 4 : 2;
  hipError_t e;
  if (F <= 1) e = go(integral_constant<int, 1>(), integral_constant<int, 1>());
  else if (F <= 2) e = go(integral_constant<int, 2>(), integral_constant<int, W>());
  else if (F <= 4) e = go(integral_constant<int, 4>(), integral_constant<int, W>());
  else e = go(integral_constant<int, 8>(), integral_constant<int, W>());
  if (nseg > 1) {
    if (e == hipSuccess) {
      const int64_t n = (int64_t)F * N;
      hipLaunchKernelGGL(k_rows_reduce<T>, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 4096)),
                         dim3(256), 0, s, (const T*)P, nseg, n, X);
      e = hipGetLastError();
    }
    const hipError_t f = sc.put(P, s);
    if (e == hipSuccess) e = f;
  }
  return e;
}

// Slices of the streamed apply's contraction (see k_apply_stream).
static int stream_slices(int M) {
  if (M < kRowSliceMinM) return 1;
  return kXcds * cdiv(M, kXcds * kStreamSliceCols);
}

size_t apply_stream_scratch_bytes(int F, int N, int M) {
  const int nseg = stream_slices(M);
  return nseg > 1 ? (size_t)nseg * F * N * 2 * sizeof(float) : 0;
}

// The streamed apply of F frames (form: kForm4M, kForm3M on complex64 R and
// data; kFormB3 on split-packed R and data, M then their padded row length).
static hipError_t stream_apply(const void* R, const void* D, float* X, int N, int M, int F, int form,
                               Scratch& sc, hipStream_t s) {
  if (F <= 0 || N <= 0) return hipSuccess;
  if (F < kStreamMinF || F > kStreamMaxF) return hipErrorInvalidValue;
  if (form == kFormB3 && M % 32 != 0) return hipErrorInvalidValue;
  const bool vec = M % 2 == 0 && ((uintptr_t)R % 16) == 0 && ((uintptr_t)D % 16) == 0;
  if (form == kFormB3 && !vec) return hipErrorInvalidValue;
  const int nseg = stream_slices(M);
  // slice length: whole 32-column chunks, so only the last slice has a
  // partial chunk
  const int seg_len = nseg > 1 ? cdiv(cdiv(M, nseg), 32) * 32 : M;
  void* P = nullptr;
  if (nseg > 1) {
    const hipError_t e = sc.get(&P, apply_stream_scratch_bytes(F, N, M), s);
    if (e != hipSuccess) return e;
  }
  float* out = nseg > 1 ? (float*)P : X;
  const float* Rf = (const float*)R;
  const float* Df = (const float*)D;
  auto go = [&](auto fb, auto fm) {
    constexpr int FB = decltype(fb)::value, NB = 2, FORM = decltype(fm)::value;
    const int nrb = cdiv(N, 64 * NB);
    const dim3 grid((unsigned)(nrb * nseg)), block(256);
    if (vec)
      hipLaunchKernelGGL((k_apply_stream<FB, NB, 2, FORM>), grid, block, 0, s, Rf, Df, out, N, M, F,
                         nseg, seg_len, nrb);
    else if constexpr (FORM != kFormB3)
      hipLaunchKernelGGL((k_apply_stream<FB, NB, 1, FORM>), grid, block, 0, s, Rf, Df, out, N, M, F,
                         nseg, seg_len, nrb);
    return hipGetLastError();
  };
  using std::integral_constant;
  auto by_form = [&](auto fb) {
    if (form == kFormB3) return go(fb, integral_constant<int, kFormB3>());
    if (form == kForm3M) return go(fb, integral_constant<int, kForm3M>());
    return go(fb, integral_constant<int, kForm4M>());
  };
  hipError_t e = F <= 16 ? by_form(integral_constant<int, 1>()) : by_form(integral_constant<int, 2>());
  if (nseg > 1) {
    if (e == hipSuccess) {
      const int64_t n = (int64_t)F * N;
      hipLaunchKernelGGL(k_rows_reduce<float>, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 4096)),
                         dim3(256), 0, s, (const float*)P, nseg, n, X);
      e = hipGetLastError();
    }
    const hipError_t f = sc.put(P, s);
    if (e == hipSuccess) e = f;
  }
  return e;
}

hipError_t launch_apply_stream(const float* R, const float* D, float* X, int N, int M, int F,
                               bool m3, Scratch& sc, hipStream_t s) {
  return stream_apply(R, D, X, N, M, F, m3 ? kForm3M : kForm4M, sc, s);
}

hipError_t launch_apply_stream_sp(const void* R, const void* D, float* X, int N, int Mp, int F,
                                  Scratch& sc, hipStream_t s) {
  return stream_apply(R, D, X, N, Mp, F, kFormB3, sc, s);
}

hipError_t launch_apply_b3(const ApplyBatch& b, Scratch& sc, hipStream_t s) {
  return run_apply<B3Cfg>(b, sc, s);
}

size_t apply_scratch_bytes_b3(int F, int N, int Mp) { return item_work_bytes<B3Cfg, false>(F, N, Mp); }

// explicit instantiations
template hipError_t launch_apply<float>(const ApplyBatch&, bool, bool, Scratch&, hipStream_t);
template hipError_t launch_apply<double>(const ApplyBatch&, bool, bool, Scratch&, hipStream_t);
template size_t apply_scratch_bytes<float>(int, int, int, bool, bool);
template size_t apply_scratch_bytes<double>(int, int, int, bool, bool);
template hipError_t launch_apply_rows<float>(const float*, const float*, float*, int, int, int,
                                             Scratch&, hipStream_t);
template hipError_t launch_apply_rows<double>(const double*, const double*, double*, int, int, int,
                                              Scratch&, hipStream_t);
template size_t apply_rows_scratch_bytes<float>(int, int, int);
template size_t apply_rows_scratch_bytes<double>(int, int, int);

}  // namespace pinv
