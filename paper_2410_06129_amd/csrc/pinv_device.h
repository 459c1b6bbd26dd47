// Device-side building blocks for the Pinv-Recon hot path on gfx950.
//
// Everything here is a template over the arithmetic type T (float or double).
// Complex matrices live in HBM as interleaved (re, im) pairs, row-major.
//
//  * EncDev / egen: one element of the encoding matrix E from separable tables
//    (paper Eq. 2 and the product form of Sec. 3.3):
//        E[(c,i),(s,v)] = C_c(v) * Px[i,ix] * Py[i,iy] * Q[i,s] * exp(-i 2 pi B0(v) t_i)
//    with Px[i,ix] = exp(-i 2 pi kx_i x_ix), Py[i,iy] = exp(-i 2 pi ky_i y_iy),
//    Q[i,s] = exp(-i 2 pi f_s t_i), rows m = c*K + i, columns n = s*V + iy*nx + ix.
//  * Tile: a block tile of C = op(A) op(B) on MFMA 16x16x4 (f32 or f64), four
//    real products per complex product ("4M"), operands staged in LDS as split
//    real/imaginary planes laid out [k][outer].
//  * Loaders fill one BK-deep chunk of an operand into registers (fetch) and then
//    into LDS (store); the mainloop double-buffers LDS so the next chunk's global
//    loads or E generation overlap the current chunk's MFMAs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pinv {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<float> { typedef f32x4 type; };
template <> struct Acc<double> { typedef f64x4 type; };

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> struct cx { T re, im; };

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ __forceinline__ void sincospi_t(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_t(double x, double* s, double* c) { sincospi(x, s, c); }

// ---------------------------------------------------------------------------
// Encoding tables on the device
// ---------------------------------------------------------------------------
template <typename T> struct EncDev {
  const T* px;    // [K][nx] complex
  const T* py;    // [K][ny] complex
  const T* q;     // [K][S] complex, or null when S == 1 and f_0 == 0
  const T* coil;  // [C][V] complex (unknown voxels only), or null for one unit coil
  const T* b0;    // [V] Hz (unknown voxels only), or null
  const T* t;     // [K] s, or null
  const int* vxy; // [V] grid position (iy << 16) | ix of unknown voxel v when a voxel
                  // mask restricts the unknowns; null when v = iy*nx + ix covers the grid
  int nx, ny, S, C, K, V;
  int M, N;       // M = C*K rows, N = S*V columns
};

// Grid position of unknown voxel v.
template <typename T>
__device__ __forceinline__ void voxel_xy(const EncDev<T>& e, int v, int* ix, int* iy) {
  if (e.vxy) {
    const int p = e.vxy[v];
    *iy = p >> 16;
    *ix = p & 0xffff;
  } else {
    *iy = v / e.nx;
    *ix = v - *iy * e.nx;
  }
}

// Which optional factors an encoding has; generated-operand kernels are
// specialised on this so that absent factors cost neither loads nor registers.
enum { FEAT_Q = 1, FEAT_B0 = 2, FEAT_COIL = 4 };
template <typename T> inline int enc_features(const EncDev<T>& e) {
  return (e.q ? FEAT_Q : 0) | (e.b0 ? FEAT_B0 : 0) | (e.coil ? FEAT_COIL : 0);
}

// ---------------------------------------------------------------------------
// Tile configuration
// ---------------------------------------------------------------------------
// M3: complex products with three real products (Gauss):
//   t1 = ar br, t2 = ai bi, t3 = (ar + ai)(br + bi);  re = t1 - t2, im = t3 - t1 - t2
// (a third LDS plane holds re + im of each operand value); otherwise four
// real products (4M).
// Four wavefronts in a WGM_ x (4 / WGM_) grid (2 x 2 by default; 1 x 4 for
// tiles of only 16 rows).
template <typename T_, int BM_, int BN_, int BK_, bool M3_ = false, int WGM_ = 2> struct TileCfg {
  typedef T_ T;
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr bool M3 = M3_;
  static constexpr int PLANES = M3 ? 3 : 2;
  static constexpr int NT = 256;
  static constexpr int WGN = 4 / WGM_;           // wavefronts along N
  static constexpr int WTM = BM / WGM_, WTN = BN / WGN;
  static constexpr int MB = WTM / 16, NB = WTN / 16;
  // FP64 3M tiles pad rows by 4 doubles: two stages then take 51 KB of LDS,
  // so three workgroups fit in a CU's 160 KB
  static constexpr int PAD = sizeof(T) == 4 ? 16 : (M3_ ? 4 : 8);
  static constexpr int LDA = BM + PAD, LDB = BN + PAD;
  static constexpr int A_PLANE = BK * LDA, B_PLANE = BK * LDB;
  static constexpr int STAGE = PLANES * A_PLANE + PLANES * B_PLANE;   // elements of T
  static constexpr int SMEM_ELEMS = 2 * STAGE;
  static_assert(WTM % 16 == 0 && WTN % 16 == 0 && BK % 4 == 0, "tile shape");
};

template <class Cfg, class = void> struct IsM3 { static constexpr bool value = false; };
template <class Cfg> struct IsM3<Cfg, decltype((void)Cfg::M3)> { static constexpr bool value = Cfg::M3; };

// 4M tiles accumulate re and im directly; M3 tiles accumulate t1 in `re`,
// t3 in `im` and t2 in `t2`, and acc_foreach forms re = t1 - t2 and
// im = t3 - t1 - t2 element by element (no second copy of the tile).
template <class Cfg> struct AccTile {
  typename Acc<typename Cfg::T>::type re[Cfg::MB][Cfg::NB];
  typename Acc<typename Cfg::T>::type im[Cfg::MB][Cfg::NB];
  typename Acc<typename Cfg::T>::type t2[Cfg::MB][Cfg::NB];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
      for (int b = 0; b < Cfg::NB; ++b) {
        re[a][b] = typename Acc<typename Cfg::T>::type{0, 0, 0, 0};
        im[a][b] = typename Acc<typename Cfg::T>::type{0, 0, 0, 0};
        if constexpr (IsM3<Cfg>::value) t2[a][b] = typename Acc<typename Cfg::T>::type{0, 0, 0, 0};
      }
  }
};


// One BK chunk of MFMAs from LDS.  sA = [re plane | im plane] of op(A) as
// [k][m], sB likewise [k][n].  Lane l supplies A[m = l%16][k = l/16] and
// B[k = l/16][n = l%16] for each 16x16x4 product.  After the MFMAs of k-step
// kk the hook `between(kk)` runs, so the loaders' element math for the next
// chunk is interleaved with this chunk's matrix products.
template <class Cfg, class Hook>
__device__ __forceinline__ void tile_compute(const typename Cfg::T* __restrict__ sA,
                                             const typename Cfg::T* __restrict__ sB,
                                             AccTile<Cfg>& acc, Hook&& between) {
  typedef typename Cfg::T T;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int wr = wid / Cfg::WGN, wc = wid % Cfg::WGN;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < Cfg::BK / 4; ++kk) {
    const int krow = kk * 4 + lk;
    if constexpr (IsM3<Cfg>::value) {
      T ar[Cfg::MB], ai[Cfg::MB], as[Cfg::MB], br[Cfg::NB], bi[Cfg::NB], bs[Cfg::NB];
#pragma unroll
      for (int a = 0; a < Cfg::MB; ++a) {
        const int off = krow * Cfg::LDA + wr * Cfg::WTM + a * 16 + lr;
        ar[a] = sA[off];
        ai[a] = sA[Cfg::A_PLANE + off];
        as[a] = sA[2 * Cfg::A_PLANE + off];
      }
#pragma unroll
      for (int b = 0; b < Cfg::NB; ++b) {
        const int off = krow * Cfg::LDB + wc * Cfg::WTN + b * 16 + lr;
        br[b] = sB[off];
        bi[b] = sB[Cfg::B_PLANE + off];
        bs[b] = sB[2 * Cfg::B_PLANE + off];
      }
#pragma unroll
      for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
        for (int b = 0; b < Cfg::NB; ++b) {
          acc.re[a][b] = mfma4(ar[a], br[b], acc.re[a][b]);
          acc.t2[a][b] = mfma4(ai[a], bi[b], acc.t2[a][b]);
          acc.im[a][b] = mfma4(as[a], bs[b], acc.im[a][b]);
        }
      between(kk);
      continue;
    }
    T ar[Cfg::MB], ai[Cfg::MB], nai[Cfg::MB], br[Cfg::NB], bi[Cfg::NB];
#pragma unroll
    for (int a = 0; a < Cfg::MB; ++a) {
      const int off = krow * Cfg::LDA + wr * Cfg::WTM + a * 16 + lr;
      ar[a] = sA[off];
      ai[a] = sA[Cfg::A_PLANE + off];
      nai[a] = -ai[a];
    }
#pragma unroll
    for (int b = 0; b < Cfg::NB; ++b) {
      const int off = krow * Cfg::LDB + wc * Cfg::WTN + b * 16 + lr;
      br[b] = sB[off];
      bi[b] = sB[Cfg::B_PLANE + off];
    }
#pragma unroll
    for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
      for (int b = 0; b < Cfg::NB; ++b) {
        acc.re[a][b] = mfma4(ar[a], br[b], acc.re[a][b]);
        acc.re[a][b] = mfma4(nai[a], bi[b], acc.re[a][b]);
        acc.im[a][b] = mfma4(ar[a], bi[b], acc.im[a][b]);
        acc.im[a][b] = mfma4(ai[a], br[b], acc.im[a][b]);
      }
    between(kk);
  }
}

// Double-buffered mainloop over k in [kbeg, kend).  Loaders zero-fill k >= kend.
// Loader protocol: fetch(k0, kend) issues the global loads of a chunk,
// finish<STEP, STEPS>() turns loaded values into operand values (the E
// element products for generated operands), store(s) writes them to LDS.
template <class Cfg, bool DOWN, class LA, class LB>
__device__ __forceinline__ void mainloop_b3(LA& la, LB& lb, int kbeg, int kend, AccTile<Cfg>& acc,
                                            float* smem_f);
template <class Cfg, class = void> struct IsB3;

// PRIO: raise the wave's issue priority over the chunk's matrix products, so
// the MFMAs of a wave that has its operands in LDS are not held back by the
// address and element math of the other waves on the SIMD (measured: W 17.35
// -> 16.78 ms, R 16.34 -> 16.06 ms at N = 4096, M = 32768).  The Cholesky's
// short panel and trailing launches keep the default: raised, they delayed
// the diagonal-block kernel beside them (7.48 -> 7.84 ms).
// DOWN: visit the chunks from the top of [kbeg, kend) down (chunk starts
// kbeg + (nch-1)*BK, ..., kbeg; the loaders still zero-fill k >= kend), so
// tiles whose ranges share their upper end read the same rows at the same time.
template <class Cfg, bool PRIO = true, bool DOWN = false, class LA, class LB>
__device__ __forceinline__ void mainloop(LA& la, LB& lb, int kbeg, int kend, AccTile<Cfg>& acc,
                                         typename Cfg::T* smem) {
  if constexpr (IsB3<Cfg>::value) {
    mainloop_b3<Cfg, DOWN>(la, lb, kbeg, kend, acc, smem);
    return;
  } else {
  typedef typename Cfg::T T;
  constexpr int STEPS = Cfg::BK / 4;
  T* stage0 = smem;
  T* stage1 = smem + Cfg::STAGE;
  // FP32 tiles run at least one chunk (an empty range loads zeros): with no
  // path around the MFMAs the compiler keeps the accumulators in AGPRs only,
  // where an early return made it hold a zeroed VGPR copy and halved the
  // occupancy.  FP64 tiles allocate better with the early return.
  if constexpr (sizeof(T) == 8) {
    if (kend <= kbeg) return;
  }
  const int nch = max(1, (kend - kbeg + Cfg::BK - 1) / Cfg::BK);
  auto chunk = [&](int c) { return DOWN ? kbeg + (nch - 1 - c) * Cfg::BK : kbeg + c * Cfg::BK; };
  la.fetch(chunk(0), kend);
  lb.fetch(chunk(0), kend);
#pragma unroll
  for (int q = 0; q < STEPS; ++q) {
    la.finish(q, STEPS);
    lb.finish(q, STEPS);
  }
  la.store(stage0);
  lb.store(stage0 + Cfg::PLANES * Cfg::A_PLANE);
  __syncthreads();
  int c = 0;
  do {
    T* cur = (c & 1) ? stage1 : stage0;
    T* nxt = (c & 1) ? stage0 : stage1;
    const bool more = c + 1 < nch;
    if (more) {
      la.fetch(chunk(c + 1), kend);
      lb.fetch(chunk(c + 1), kend);
    }
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
    tile_compute<Cfg>(cur, cur + Cfg::PLANES * Cfg::A_PLANE, acc, [&](int kk) {
      la.finish(kk, STEPS);
      lb.finish(kk, STEPS);
    });
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    if (more) {
      la.store(nxt);
      lb.store(nxt + Cfg::PLANES * Cfg::A_PLANE);
    }
    __syncthreads();
  } while (++c < nch);
  }
}

// ---------------------------------------------------------------------------
// BF16x3 ("BF16 split") products.  Each FP32 operand value x is split into
// hi = bf16(x) and lo = bf16(x - hi); a real product is hi*hi + hi*lo + lo*hi
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (relative error ~2^-16
// per product, the lo*lo term dropped).
//
// The operands are split once, where they are produced, into "split-packed"
// (SP) storage: a complex matrix with k contiguous, rows of Kp = 32 *
// ceil(K / 32) columns (zero beyond K), each group of 8 consecutive k of a row
// stored as 64 bytes: re_hi[8], re_lo[8], im_hi[8], im_lo[8] (bf16).  That is
// eight bytes per complex value, as for complex64; a tile moves SP chunks into
// LDS with 16-byte loads and stores and no arithmetic.
//
// In LDS an operand row holds its chunk as SP memory does: the chunk's four
// 8-groups, each as its four planes (re_hi, re_lo, im_hi, im_lo), 256 bytes,
// plus 16 bytes of padding (ROW = 136 bf16).  An SP chunk row is then copied
// with 16-byte stores to consecutive addresses (conflict-free), and the
// 16-byte reads of 16 consecutive rows, 68 dwords apart, fall in distinct
// banks; a lane reads its eight consecutive k values of one plane with one
// load.  (Four separate plane arrays, each starting on bank 0, made the 16
// stores of a row segment collide four ways: bank conflicts were 24% of the
// R product's cycles.)  One chunk is BK = 32, a single MFMA k-step.  Two LDS
// stages: the next chunk is written to one while the other's MFMAs run.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_b16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 neg_b16(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}
// hi and lo parts of x0 and x1, each pair packed in a 32-bit word (x0 in the
// low half).  x - float(hi) is exact in FP32.
__device__ __forceinline__ void split2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2v{x0, x1}, bf16x2));
  const float h0 = __builtin_bit_cast(float, h << 16);
  const float h1 = __builtin_bit_cast(float, h & 0xffff0000u);
  hi = h;
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2v{x0 - h0, x1 - h1}, bf16x2));
}
// The value a packed hi/lo word pair holds in element e (0 low, 1 high).
__device__ __forceinline__ float join2(uint32_t hi, uint32_t lo, int e) {
  const uint32_t sh = e ? 0u : 16u;
  return __builtin_bit_cast(float, (hi << sh) & 0xffff0000u) +
         __builtin_bit_cast(float, (lo << sh) & 0xffff0000u);
}
// One SP group (64 bytes) from eight complex values.
__device__ __forceinline__ void sp_group(const float (&re)[8], const float (&im)[8], uint4 (&g)[4]) {
  uint32_t rh[4], rl[4], ih[4], il[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    split2(re[2 * j], re[2 * j + 1], rh[j], rl[j]);
    split2(im[2 * j], im[2 * j + 1], ih[j], il[j]);
  }
  g[0] = uint4{rh[0], rh[1], rh[2], rh[3]};
  g[1] = uint4{rl[0], rl[1], rl[2], rl[3]};
  g[2] = uint4{ih[0], ih[1], ih[2], ih[3]};
  g[3] = uint4{il[0], il[1], il[2], il[3]};
}

// WGM x WGN wavefronts, each with a WTM x WTN part of the tile; STAGES LDS
// stages (2: the next chunk is stored while this one computes, one barrier
// per chunk; 1: store, barrier, compute, barrier, with other workgroups on
// the CU filling the gaps).
template <int BM_, int BN_, int WGM_ = 2, int WGN_ = 2, int STAGES_ = 2> struct TileCfgB3 {
  typedef float T;
  static constexpr bool B3 = true;
  static constexpr int BM = BM_, BN = BN_, BK = 32;
  static constexpr int STAGES = STAGES_;
  // single-stage tiles are meant to share a CU with another workgroup
  static constexpr int MIN_BLOCKS = STAGES_ == 1 ? 2 : 1;
  static constexpr int WGN = WGN_;
  static constexpr int NT = 64 * WGM_ * WGN_;
  static constexpr int WTM = BM / WGM_, WTN = BN / WGN_;
  static constexpr int MB = WTM / 16, NB = WTN / 16;
  static constexpr int ROW = 4 * BK + 8;           // bf16 per LDS row (272 bytes)
  static constexpr int LDA = 0, LDB = 0;            // FP32 layouts unused
  static constexpr int A_OPER = BM * ROW, B_OPER = BN * ROW;   // bf16 elements
  static constexpr int STAGE = A_OPER + B_OPER;                  // bf16 elements
  static constexpr int SMEM_BYTES = STAGES * STAGE * 2;
  static constexpr int SMEM_ELEMS = SMEM_BYTES / 4;
};

template <class Cfg, class> struct IsB3 { static constexpr bool value = false; };
template <class Cfg> struct IsB3<Cfg, decltype((void)Cfg::B3)> { static constexpr bool value = Cfg::B3; };

template <class Cfg, class Hook>
__device__ __forceinline__ void tile_compute_b3(const __bf16* __restrict__ sA,
                                                const __bf16* __restrict__ sB, AccTile<Cfg>& acc,
                                                Hook&& between) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int wr = wid / Cfg::WGN, wc = wid % Cfg::WGN;
  const int lr = lane & 15, kb = 32 * (lane >> 4);   // the lane's 8-group within the row
  bf16x8 b[Cfg::NB][4];
#pragma unroll
  for (int j = 0; j < Cfg::NB; ++j) {
    const int off = (wc * Cfg::WTN + j * 16 + lr) * Cfg::ROW + kb;
#pragma unroll
    for (int p = 0; p < 4; ++p) b[j][p] = *reinterpret_cast<const bf16x8*>(sB + off + 8 * p);
  }
#pragma unroll
  for (int i = 0; i < Cfg::MB; ++i) {
    const int off = (wr * Cfg::WTM + i * 16 + lr) * Cfg::ROW + kb;
    const bf16x8 arh = *reinterpret_cast<const bf16x8*>(sA + off);
    const bf16x8 arl = *reinterpret_cast<const bf16x8*>(sA + off + 8);
    const bf16x8 aih = *reinterpret_cast<const bf16x8*>(sA + off + 16);
    const bf16x8 ail = *reinterpret_cast<const bf16x8*>(sA + off + 24);
    const bf16x8 naih = neg_b16(aih), nail = neg_b16(ail);
#pragma unroll
    for (int j = 0; j < Cfg::NB; ++j) {
      f32x4 cr = acc.re[i][j], ci = acc.im[i][j];
      cr = mfma_b16(arh, b[j][0], cr);
      cr = mfma_b16(arh, b[j][1], cr);
      cr = mfma_b16(arl, b[j][0], cr);
      cr = mfma_b16(naih, b[j][2], cr);
      cr = mfma_b16(naih, b[j][3], cr);
      cr = mfma_b16(nail, b[j][2], cr);
      ci = mfma_b16(arh, b[j][2], ci);
      ci = mfma_b16(arh, b[j][3], ci);
      ci = mfma_b16(arl, b[j][2], ci);
      ci = mfma_b16(aih, b[j][0], ci);
      ci = mfma_b16(aih, b[j][1], ci);
      ci = mfma_b16(ail, b[j][0], ci);
      acc.re[i][j] = cr;
      acc.im[i][j] = ci;
    }
    between(i);
  }
}

// Loader protocol as for the FP32 tiles, with store_b3<ROW>(s) writing the
// chunk's rows in the layout above.  DOWN as for mainloop.
template <class Cfg, bool DOWN, class LA, class LB>
__device__ __forceinline__ void mainloop_b3(LA& la, LB& lb, int kbeg, int kend, AccTile<Cfg>& acc,
                                            float* smem_f) {
  // at least one chunk (an empty range loads zeros): a path around the MFMAs
  // made the compiler keep a copy of the accumulators outside the AGPRs
  __bf16* const stage0 = reinterpret_cast<__bf16*>(smem_f);
  __bf16* const stage1 = stage0 + Cfg::STAGE;
  const int nch = max(1, (kend - kbeg + Cfg::BK - 1) / Cfg::BK);
  auto chunk = [&](int c) { return DOWN ? kbeg + (nch - 1 - c) * Cfg::BK : kbeg + c * Cfg::BK; };
  la.fetch(chunk(0), kend);
  lb.fetch(chunk(0), kend);
#pragma unroll
  for (int q = 0; q < Cfg::MB; ++q) {
    la.finish(q, Cfg::MB);
    lb.finish(q, Cfg::MB);
  }
  if constexpr (Cfg::STAGES == 1) {
    for (int c = 0; c < nch; ++c) {
      const bool more = c + 1 < nch;
      la.template store_b3<Cfg::ROW>(stage0);
      lb.template store_b3<Cfg::ROW>(stage0 + Cfg::A_OPER);
      __syncthreads();
      if (more) {
        la.fetch(chunk(c + 1), kend);
        lb.fetch(chunk(c + 1), kend);
      }
      // raised issue priority over the matrix products, as in the FP32 loop:
      // the other workgroup's stores and address math on the SIMD wait
      __builtin_amdgcn_s_setprio(1);
      tile_compute_b3<Cfg>(stage0, stage0 + Cfg::A_OPER, acc, [&](int i) {
        if (more) {
          la.finish(i, Cfg::MB);
          lb.finish(i, Cfg::MB);
        }
      });
      __builtin_amdgcn_s_setprio(0);
      __syncthreads();
    }
    return;
  }
  la.template store_b3<Cfg::ROW>(stage0);
  lb.template store_b3<Cfg::ROW>(stage0 + Cfg::A_OPER);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    __bf16* cur = (c & 1) ? stage1 : stage0;
    __bf16* nxt = (c & 1) ? stage0 : stage1;
    const bool more = c + 1 < nch;
    if (more) {
      la.fetch(chunk(c + 1), kend);
      lb.fetch(chunk(c + 1), kend);
    }
    tile_compute_b3<Cfg>(cur, cur + Cfg::A_OPER, acc, [&](int i) {
      if (more) {
        la.finish(i, Cfg::MB);
        lb.finish(i, Cfg::MB);
      }
    });
    if (more) {
      la.template store_b3<Cfg::ROW>(nxt);
      lb.template store_b3<Cfg::ROW>(nxt + Cfg::A_OPER);
    }
    __syncthreads();
  }
}

// Tile-local coordinates of accumulator (a, b, r) for this lane.
template <class Cfg>
__device__ __forceinline__ void acc_coord(int a, int b, int r, int* row, int* col) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int wr = wid / Cfg::WGN, wc = wid % Cfg::WGN;
  constexpr bool f64 = sizeof(typename Cfg::T) == 8;
  *row = wr * Cfg::WTM + a * 16 + (f64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
  *col = wc * Cfg::WTN + b * 16 + (lane & 15);
}

// Visit every accumulator element: f(row, col, re, im) with tile-local row/col.
// Output layout of the 16x16 result: column = lane % 16 for both types; the
// row of accumulator register r is 4*(lane/16) + r for the f32 instruction and
// lane/16 + 4*r for the f64 one.
template <class Cfg, class F>
__device__ __forceinline__ void acc_foreach(const AccTile<Cfg>& acc, F&& f) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int wr = wid / Cfg::WGN, wc = wid % Cfg::WGN;
  constexpr bool f64 = sizeof(typename Cfg::T) == 8;
#pragma unroll
  for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
    for (int b = 0; b < Cfg::NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr * Cfg::WTM + a * 16 + (f64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        const int col = wc * Cfg::WTN + b * 16 + (lane & 15);
        if constexpr (IsM3<Cfg>::value) {
          const typename Cfg::T t1 = acc.re[a][b][r], t3 = acc.im[a][b][r], t2 = acc.t2[a][b][r];
          f(row, col, t1 - t2, t3 - t1 - t2);
          // keep the scheduler from hoisting every accumulator read ahead of the
          // stores (that would need a VGPR copy of the whole tile)
          __builtin_amdgcn_sched_barrier(0);
        } else {
          f(row, col, acc.re[a][b][r], acc.im[a][b][r]);
        }
      }
}

// Fold a tile's accumulators into an outer accumulator pair (re, im), for
// contractions run in segments.
template <class Cfg>
__device__ __forceinline__ void acc_fold(const AccTile<Cfg>& acc,
                                         typename Acc<typename Cfg::T>::type (&ore)[Cfg::MB][Cfg::NB],
                                         typename Acc<typename Cfg::T>::type (&oim)[Cfg::MB][Cfg::NB]) {
#pragma unroll
  for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
    for (int b = 0; b < Cfg::NB; ++b) {
      if constexpr (IsM3<Cfg>::value) {
        ore[a][b] += acc.re[a][b] - acc.t2[a][b];
        oim[a][b] += acc.im[a][b] - acc.re[a][b] - acc.t2[a][b];
      } else {
        ore[a][b] += acc.re[a][b];
        oim[a][b] += acc.im[a][b];
      }
    }
}

// Visit the elements of an outer accumulator pair: f(row, col, re, im).
template <class Cfg, class F>
__device__ __forceinline__ void acc_foreach_outer(
    const typename Acc<typename Cfg::T>::type (&ore)[Cfg::MB][Cfg::NB],
    const typename Acc<typename Cfg::T>::type (&oim)[Cfg::MB][Cfg::NB], F&& f) {
  int row, col;
#pragma unroll
  for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
    for (int b = 0; b < Cfg::NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc_coord<Cfg>(a, b, r, &row, &col);
        f(row, col, ore[a][b][r], oim[a][b][r]);
      }
}

// The same walk with writable accumulator entries (used to start a tile from
// existing output values).
template <class Cfg, class F>
__device__ __forceinline__ void acc_foreach_mut(AccTile<Cfg>& acc, F&& f) {
  static_assert(!IsM3<Cfg>::value, "4M tiles only: the walk reads and writes re and im directly");
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int wr = wid / Cfg::WGN, wc = wid % Cfg::WGN;
  constexpr bool f64 = sizeof(typename Cfg::T) == 8;
#pragma unroll
  for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
    for (int b = 0; b < Cfg::NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr * Cfg::WTM + a * 16 + (f64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        const int col = wc * Cfg::WTN + b * 16 + (lane & 15);
        typename Cfg::T re = acc.re[a][b][r], im = acc.im[a][b][r];
        f(row, col, re, im);
        acc.re[a][b][r] = re;
        acc.im[a][b][r] = im;
      }
}

// ---------------------------------------------------------------------------
// Loaders.  OUTER = BM (A operand) or BN (B operand).  Each writes its chunk to
// LDS planes s[0 .. BK*LD) (real) and s[BK*LD .. 2*BK*LD) (imaginary), at
// s[k*LD + o].
// ---------------------------------------------------------------------------

// Dense loaders.  fetch() issues one load per pass from a clamped, always
// in-bounds address and records which passes are in range; the range mask and
// the optional conjugation are applied when the values are written to LDS, so
// no instruction between fetch() and store() waits on the loads and the next
// chunk's loads stay in flight under the current chunk's MFMAs.
template <typename T, typename S, bool CONJ>
__device__ __forceinline__ void dense_value(const cx<S>& v, bool ok, T& re, T& im) {
  re = ok ? T(v.re) : T(0);
  im = ok ? (CONJ ? -T(v.im) : T(v.im)) : T(0);
}

// Dense complex storage with k contiguous: element (o, k) at p[o*ld + k].
template <class Cfg, int OUTER, int LD, typename S, bool CONJ>
struct LoadDenseKC {
  typedef typename Cfg::T T;
  static constexpr int TPR = Cfg::BK;                // one complex per thread per row
  static constexpr int RPP = Cfg::NT / TPR;          // rows per pass
  static constexpr int PASSES = OUTER / RPP;
  static_assert(OUTER % RPP == 0, "loader shape");
  const cx<S>* p;
  int64_t ld;
  int o0, oend;
  cx<S> v[PASSES];
  bool ok[PASSES];
  __device__ __forceinline__ void fetch(int k0, int kend) {
    const int k = k0 + (int)(threadIdx.x % TPR);
    const int kc = max(0, min(k, kend - 1));
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int o = o0 + (int)(threadIdx.x / TPR) + j * RPP;
      ok[j] = o < oend && k < kend;
      const int oc = max(0, min(o, oend - 1));
      v[j] = p[(int64_t)oc * ld + kc];
    }
  }
  __device__ __forceinline__ void finish(int, int) {}
  __device__ __forceinline__ void store(T* s) {
    const int kk = threadIdx.x % TPR;
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int o = threadIdx.x / TPR + j * RPP;
      T re, im;
      dense_value<T, S, CONJ>(v[j], ok[j], re, im);
      s[kk * LD + o] = re;
      s[Cfg::BK * LD + kk * LD + o] = im;
      if constexpr (IsM3<Cfg>::value) s[2 * Cfg::BK * LD + kk * LD + o] = re + im;
    }
  }
};

// Dense complex storage with the outer index contiguous: element (o, k) at p[k*ld + o].
template <class Cfg, int OUTER, int LD, typename S, bool CONJ>
struct LoadDenseOC {
  typedef typename Cfg::T T;
  static constexpr int KPP = Cfg::NT / OUTER;        // k rows per pass
  static constexpr int PASSES = Cfg::BK / KPP;
  static_assert(Cfg::NT % OUTER == 0 && Cfg::BK % KPP == 0, "loader shape");
  const cx<S>* p;
  int64_t ld;
  int o0, oend;
  cx<S> v[PASSES];
  bool ok[PASSES];
  __device__ __forceinline__ void fetch(int k0, int kend) {
    const int o = o0 + (int)(threadIdx.x % OUTER);
    const int oc = max(0, min(o, oend - 1));
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int k = k0 + (int)(threadIdx.x / OUTER) + j * KPP;
      ok[j] = o < oend && k < kend;
      const int kc = max(0, min(k, kend - 1));
      v[j] = p[(int64_t)kc * ld + oc];
    }
  }
  __device__ __forceinline__ void finish(int, int) {}
  __device__ __forceinline__ void store(T* s) {
    const int o = threadIdx.x % OUTER;
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int kk = threadIdx.x / OUTER + j * KPP;
      T re, im;
      dense_value<T, S, CONJ>(v[j], ok[j], re, im);
      s[kk * LD + o] = re;
      s[Cfg::BK * LD + kk * LD + o] = im;
      if constexpr (IsM3<Cfg>::value) s[2 * Cfg::BK * LD + kk * LD + o] = re + im;
    }
  }
};

// Raw factors of one generated element, loaded in fetch() and multiplied in
// finish(): E = Px * Py [* Q] [* exp(-i 2 pi B0 t)] [* coil].
template <typename T> struct GenRaw {
  cx<T> px, py, q, coil;
  T b0t;
};

template <int FEAT, typename T>
__device__ __forceinline__ void gen_load(const EncDev<T>& e, int i, int s, int v, int ix, int iy,
                                         int c, GenRaw<T>& r) {
  const cx<T>* px = reinterpret_cast<const cx<T>*>(e.px);
  const cx<T>* py = reinterpret_cast<const cx<T>*>(e.py);
  r.px = px[(size_t)i * e.nx + ix];
  r.py = py[(size_t)i * e.ny + iy];
  if constexpr ((FEAT & FEAT_Q) != 0) r.q = reinterpret_cast<const cx<T>*>(e.q)[(size_t)i * e.S + s];
  if constexpr ((FEAT & FEAT_B0) != 0) r.b0t = e.b0[v] * e.t[i];
  if constexpr ((FEAT & FEAT_COIL) != 0)
    r.coil = reinterpret_cast<const cx<T>*>(e.coil)[(size_t)c * e.V + v];
}

template <int FEAT, typename T>
__device__ __forceinline__ cx<T> gen_product(const GenRaw<T>& r) {
  cx<T> p = cmul(r.px, r.py);
  if constexpr ((FEAT & FEAT_Q) != 0) p = cmul(p, r.q);
  if constexpr ((FEAT & FEAT_B0) != 0) {
    T sn, cs;
    sincospi_t(T(-2) * r.b0t, &sn, &cs);
    p = cmul(p, cx<T>{cs, sn});
  }
  if constexpr ((FEAT & FEAT_COIL) != 0) p = cmul(p, r.coil);
  return p;
}

// Generated operand, outer index = column n of E, k = row m of E:
// element (o, k) = E[k, o] (or its conjugate).  Each thread keeps one column.
// ALIGNED (K a multiple of BK, chunks starting at multiples of BK): every row
// of a chunk lies in one coil, so the coil and off-resonance factors are
// loaded once per chunk or per tile and the per-sample tables advance by a
// constant stride instead of being re-indexed element by element.
template <class Cfg, int OUTER, int LD, bool CONJ, int FEAT, bool ALIGNED = false>
struct LoadGenCol {
  typedef typename Cfg::T T;
  static constexpr int KPP = Cfg::NT / OUTER;
  static constexpr int PASSES = Cfg::BK / KPP;
  static_assert(Cfg::NT % OUTER == 0 && Cfg::BK % KPP == 0, "loader shape");
  EncDev<T> e;
  bool valid;
  int s, v, ix, iy;
  T b0v;
  bool ok[PASSES];
  GenRaw<T> raw[PASSES];
  T re[PASSES], im[PASSES];
  __device__ __forceinline__ void init(const EncDev<T>& enc, int o0) {
    e = enc;
    const int n = o0 + threadIdx.x % OUTER;
    valid = n < e.N;
    const int nn = valid ? n : 0;
    s = nn / e.V;
    v = nn - s * e.V;
    voxel_xy(e, v, &ix, &iy);
    if constexpr (ALIGNED && (FEAT & FEAT_B0) != 0) b0v = e.b0[v];
  }
  __device__ __forceinline__ void fetch(int k0, int kend) {
    if constexpr (ALIGNED) {
      // k0 is a multiple of BK, so the chunk's rows share one coil and the
      // sample index stays below K; the coil index is clamped for chunks past M
      const int c = k0 / e.K;
      const int i0 = k0 - c * e.K + (int)(threadIdx.x / OUTER);
      const cx<T>* px = reinterpret_cast<const cx<T>*>(e.px) + (size_t)i0 * e.nx + ix;
      const cx<T>* py = reinterpret_cast<const cx<T>*>(e.py) + (size_t)i0 * e.ny + iy;
      cx<T> coil{T(1), T(0)};
      if constexpr ((FEAT & FEAT_COIL) != 0)
        coil = reinterpret_cast<const cx<T>*>(e.coil)[(size_t)min(c, e.C - 1) * e.V + v];
#pragma unroll
      for (int j = 0; j < PASSES; ++j) {
        ok[j] = valid && k0 + (int)(threadIdx.x / OUTER) + j * KPP < kend;
        raw[j].px = px[(size_t)j * KPP * e.nx];
        raw[j].py = py[(size_t)j * KPP * e.ny];
        if constexpr ((FEAT & FEAT_Q) != 0)
          raw[j].q = reinterpret_cast<const cx<T>*>(e.q)[(size_t)(i0 + j * KPP) * e.S + s];
        if constexpr ((FEAT & FEAT_B0) != 0) raw[j].b0t = b0v * e.t[i0 + j * KPP];
        if constexpr ((FEAT & FEAT_COIL) != 0) raw[j].coil = coil;
      }
      return;
    }
    int m = k0 + threadIdx.x / OUTER;
    int c = m / e.K;
    int i = m - c * e.K;
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      ok[j] = valid && m < kend;
      gen_load<FEAT>(e, ok[j] ? i : 0, s, v, ix, iy, ok[j] ? c : 0, raw[j]);
      m += KPP;
      i += KPP;
#pragma unroll
      for (int q = 0; q < KPP; ++q)
        if (i >= e.K) {
          i -= e.K;
          ++c;
        }
    }
  }
  __device__ __forceinline__ void finish(int step, int steps) {
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      if ((j * steps) / PASSES != step) continue;
      const cx<T> el = gen_product<FEAT>(raw[j]);
      re[j] = ok[j] ? el.re : T(0);
      im[j] = ok[j] ? (CONJ ? -el.im : el.im) : T(0);
    }
  }
  __device__ __forceinline__ void store(T* s_) {
    const int o = threadIdx.x % OUTER;
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int kk = threadIdx.x / OUTER + j * KPP;
      s_[kk * LD + o] = re[j];
      s_[Cfg::BK * LD + kk * LD + o] = im[j];
      if constexpr (IsM3<Cfg>::value) s_[2 * Cfg::BK * LD + kk * LD + o] = re[j] + im[j];
    }
  }
};

// Generated operand, outer index = row m of E, k = column n of E:
// element (o, k) = E[o, k] (or its conjugate).  Each thread keeps one row.
// ALIGNED (nx a multiple of BK, no voxel mask, chunks starting at multiples of
// BK): every column of a chunk lies in one image row of one species, so Py, Q
// and the sample's time are loaded once per chunk or per tile, and Px and the
// coil map advance by a constant stride.
template <class Cfg, int OUTER, int LD, bool CONJ, int FEAT, bool ALIGNED = false>
struct LoadGenRow {
  typedef typename Cfg::T T;
  static constexpr int KPP = Cfg::NT / OUTER;
  static constexpr int PASSES = Cfg::BK / KPP;
  static_assert(Cfg::NT % OUTER == 0 && Cfg::BK % KPP == 0, "loader shape");
  EncDev<T> e;
  bool valid;
  int c, i;
  T ti;
  bool ok[PASSES];
  GenRaw<T> raw[PASSES];
  T re[PASSES], im[PASSES];
  __device__ __forceinline__ void init(const EncDev<T>& enc, int o0) {
    e = enc;
    const int m = o0 + threadIdx.x % OUTER;
    valid = m < e.M;
    const int mm = valid ? m : 0;
    c = mm / e.K;
    i = mm - c * e.K;
    if constexpr (ALIGNED && (FEAT & FEAT_B0) != 0) ti = e.t[i];
  }
  __device__ __forceinline__ void fetch(int k0, int kend) {
    if constexpr (ALIGNED) {
      // indices come from the chunk start clamped to the last full chunk, so
      // every table access stays in bounds; ok[] masks columns >= kend
      const int n0 = min(k0, e.N - Cfg::BK) + (int)(threadIdx.x / OUTER);
      const int s = n0 / e.V;
      const int v0 = n0 - s * e.V;
      const int iy = v0 / e.nx;
      const int ix0 = v0 - iy * e.nx;
      const cx<T> py = reinterpret_cast<const cx<T>*>(e.py)[(size_t)i * e.ny + iy];
      cx<T> q{T(1), T(0)};
      if constexpr ((FEAT & FEAT_Q) != 0) q = reinterpret_cast<const cx<T>*>(e.q)[(size_t)i * e.S + s];
      const cx<T>* px = reinterpret_cast<const cx<T>*>(e.px) + (size_t)i * e.nx + ix0;
      const cx<T>* coil = reinterpret_cast<const cx<T>*>(e.coil) + (size_t)c * e.V + v0;
#pragma unroll
      for (int j = 0; j < PASSES; ++j) {
        ok[j] = valid && k0 + (int)(threadIdx.x / OUTER) + j * KPP < kend;
        raw[j].px = px[j * KPP];
        raw[j].py = py;
        if constexpr ((FEAT & FEAT_Q) != 0) raw[j].q = q;
        if constexpr ((FEAT & FEAT_B0) != 0) raw[j].b0t = e.b0[v0 + j * KPP] * ti;
        if constexpr ((FEAT & FEAT_COIL) != 0) raw[j].coil = coil[j * KPP];
      }
      return;
    }
    int n = k0 + threadIdx.x / OUTER;
    if (e.vxy) {   // voxel mask: each column's grid position from the voxel table
#pragma unroll
      for (int j = 0; j < PASSES; ++j) {
        const int nj = n + j * KPP;
        ok[j] = valid && nj < kend;
        const int nn = nj < e.N ? nj : 0;
        int s = 0, v = nn;   // without a species table there is one species
        if constexpr ((FEAT & FEAT_Q) != 0) {
          s = nn / e.V;
          v = nn - s * e.V;
        }
        int ix, iy;
        voxel_xy(e, v, &ix, &iy);
        gen_load<FEAT>(e, i, s, v, ix, iy, c, raw[j]);
      }
      return;
    }
    const int nn = n < e.N ? n : 0;
    int s = nn / e.V;
    const int v0 = nn - s * e.V;
    int iy = v0 / e.nx;
    int ix = v0 - iy * e.nx;
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      ok[j] = valid && n < kend;
      const bool in = n < e.N;
      gen_load<FEAT>(e, i, in ? s : 0, in ? iy * e.nx + ix : 0, in ? ix : 0, in ? iy : 0, c, raw[j]);
      n += KPP;
      ix += KPP;
#pragma unroll
      for (int q = 0; q < KPP; ++q)
        if (ix >= e.nx) {
          ix -= e.nx;
          if (++iy == e.ny) {
            iy = 0;
            ++s;
          }
        }
    }
  }
  __device__ __forceinline__ void finish(int step, int steps) {
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      if ((j * steps) / PASSES != step) continue;
      const cx<T> el = gen_product<FEAT>(raw[j]);
      re[j] = ok[j] ? el.re : T(0);
      im[j] = ok[j] ? (CONJ ? -el.im : el.im) : T(0);
    }
  }
  __device__ __forceinline__ void store(T* s_) {
    const int o = threadIdx.x % OUTER;
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int kk = threadIdx.x / OUTER + j * KPP;
      s_[kk * LD + o] = re[j];
      s_[Cfg::BK * LD + kk * LD + o] = im[j];
      if constexpr (IsM3<Cfg>::value) s_[2 * Cfg::BK * LD + kk * LD + o] = re[j] + im[j];
    }
  }
};

// ---------------------------------------------------------------------------
// Split-precision loaders and epilogue
// ---------------------------------------------------------------------------

// An SP matrix operand (rows = outer index, k contiguous): per chunk each row
// is 256 contiguous bytes (four 8-groups of four planes), moved by 16 threads
// with one 16-byte load and one 16-byte LDS store each.  Rows at or beyond
// oend, and every row of a chunk at or beyond kend, are zeros; within a range
// k needs no mask (the storage is zero beyond K and every chunk lies within
// Kp).  A tile whose rows are all valid (the common case, decided once per
// workgroup) loads from one base address per thread at a fixed row stride;
// an edge tile skips the loads of its missing rows.  Either way the values
// reach store_b3 final, so the LDS stores carry no masking.
template <class Cfg, int OUTER> struct LoadSP {
  static constexpr int PPR = Cfg::BK / 8 * 4;        // 16-byte pieces per row and chunk
  static constexpr int RPP = Cfg::NT / PPR;          // rows per pass
  static constexpr int PASSES = OUTER / RPP;
  static_assert(OUTER % RPP == 0, "loader shape");
  const uint4* p;   // the SP matrix as 16-byte pieces
  int64_t gpr;      // 8-groups per row (Kp / 8)
  int o0, oend;
  uint4 v[PASSES];
  __device__ __forceinline__ void fetch(int k0, int kend) {
    const int rl = threadIdx.x / PPR, q = threadIdx.x % PPR;
    if (o0 + OUTER <= oend && k0 < kend) {
      const uint4* b = p + ((int64_t)(o0 + rl) * gpr + (k0 >> 3)) * 4 + q;
      const int64_t st = (int64_t)RPP * gpr * 4;
#pragma unroll
      for (int j = 0; j < PASSES; ++j) v[j] = b[j * st];
      return;
    }
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int o = o0 + rl + j * RPP;
      v[j] = uint4{0, 0, 0, 0};
      if (o < oend && k0 < kend) v[j] = p[((int64_t)o * gpr + (k0 >> 3)) * 4 + q];
    }
  }
  __device__ __forceinline__ void finish(int, int) {}
  template <int ROW>
  __device__ __forceinline__ void store_b3(__bf16* s) {
    const int q = threadIdx.x % PPR;   // the piece's place in the row, as in memory
#pragma unroll
    for (int j = 0; j < PASSES; ++j) {
      const int o = threadIdx.x / PPR + j * RPP;
      *reinterpret_cast<uint4*>(s + o * ROW + 8 * q) = v[j];
    }
  }
};

// Generated operand for split-precision tiles: outer index = row m of E, k =
// column n of E, element (o, k) = E[o, k] (or its conjugate).  Each thread
// generates KPT consecutive columns of one row and splits them into packed
// hi/lo words as it goes (finish), so store_b3 only moves 16-byte pieces.
// ALIGNED as for LoadGenRow.
template <class Cfg, int OUTER, bool CONJ, int FEAT, bool ALIGNED = false>
struct LoadGenRowSP {
  typedef float T;
  static constexpr int TPR = Cfg::NT / OUTER;        // threads per row
  static constexpr int KPT = Cfg::BK / TPR;          // consecutive columns per thread
  static constexpr int GPT = KPT / 8;                // 8-groups per thread
  static_assert(Cfg::NT % OUTER == 0 && KPT % 8 == 0, "loader shape");
  EncDev<T> e;
  bool valid;
  int c, i, kk0;
  T ti;
  bool ok[KPT];
  GenRaw<T> raw[KPT];
  uint32_t pk[GPT][4][4];   // [group][plane][word]
  __device__ __forceinline__ void init(const EncDev<T>& enc, int o0) {
    e = enc;
    const int m = o0 + threadIdx.x % OUTER;
    valid = m < e.M;
    const int mm = valid ? m : 0;
    c = mm / e.K;
    i = mm - c * e.K;
    kk0 = (int)(threadIdx.x / OUTER) * KPT;
    if constexpr (ALIGNED && (FEAT & FEAT_B0) != 0) ti = e.t[i];
  }
  __device__ __forceinline__ void fetch(int k0, int kend) {
    if constexpr (ALIGNED) {
      // the chunk's columns lie in one image row; the start is clamped to the
      // last full chunk so every table access stays in bounds (ok[] masks)
      const int n0 = min(k0, e.N - Cfg::BK) + kk0;
      const int s = n0 / e.V;
      const int v0 = n0 - s * e.V;
      const int iy = v0 / e.nx;
      const int ix0 = v0 - iy * e.nx;
      const cx<T> py = reinterpret_cast<const cx<T>*>(e.py)[(size_t)i * e.ny + iy];
      cx<T> q{T(1), T(0)};
      if constexpr ((FEAT & FEAT_Q) != 0) q = reinterpret_cast<const cx<T>*>(e.q)[(size_t)i * e.S + s];
      const cx<T>* px = reinterpret_cast<const cx<T>*>(e.px) + (size_t)i * e.nx + ix0;
      const cx<T>* coil = reinterpret_cast<const cx<T>*>(e.coil) + (size_t)c * e.V + v0;
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        ok[j] = valid && k0 + kk0 + j < kend;
        raw[j].px = px[j];
        raw[j].py = py;
        if constexpr ((FEAT & FEAT_Q) != 0) raw[j].q = q;
        if constexpr ((FEAT & FEAT_B0) != 0) raw[j].b0t = e.b0[v0 + j] * ti;
        if constexpr ((FEAT & FEAT_COIL) != 0) raw[j].coil = coil[j];
      }
      return;
    }
    const int n = k0 + kk0;
    if (e.vxy) {   // voxel mask: each column's grid position from the voxel table
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int nj = n + j;
        ok[j] = valid && nj < kend;
        const int nn = nj < e.N ? nj : 0;
        int s = 0, v = nn;   // without a species table there is one species
        if constexpr ((FEAT & FEAT_Q) != 0) {
          s = nn / e.V;
          v = nn - s * e.V;
        }
        int ix, iy;
        voxel_xy(e, v, &ix, &iy);
        gen_load<FEAT>(e, i, s, v, ix, iy, c, raw[j]);
      }
      return;
    }
    const int nn = n < e.N ? n : 0;
    int s = nn / e.V;
    const int v0 = nn - s * e.V;
    int iy = v0 / e.nx;
    int ix = v0 - iy * e.nx;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      ok[j] = valid && n + j < kend;
      const bool in = n + j < e.N;
      gen_load<FEAT>(e, i, in ? s : 0, in ? iy * e.nx + ix : 0, in ? ix : 0, in ? iy : 0, c, raw[j]);
      if (++ix == e.nx) {
        ix = 0;
        if (++iy == e.ny) {
          iy = 0;
          ++s;
        }
      }
    }
  }
  // Step `step` of `steps` forms and splits its share of the columns, in pairs.
  __device__ __forceinline__ void finish(int step, int steps) {
#pragma unroll
    for (int j = 0; j < KPT; j += 2) {
      if ((j * steps) / KPT != step) continue;
      T re[2], im[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const cx<T> el = gen_product<FEAT>(raw[j + u]);
        re[u] = ok[j + u] ? el.re : T(0);
        im[u] = ok[j + u] ? (CONJ ? -el.im : el.im) : T(0);
      }
      const int g = j >> 3, w = (j & 7) >> 1;
      split2(re[0], re[1], pk[g][0][w], pk[g][1][w]);
      split2(im[0], im[1], pk[g][2][w], pk[g][3][w]);
    }
  }
  template <int ROW>
  __device__ __forceinline__ void store_b3(__bf16* s) {
    const int o = threadIdx.x % OUTER;
#pragma unroll
    for (int g = 0; g < GPT; ++g)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl)
        *reinterpret_cast<uint4*>(s + o * ROW + 32 * (kk0 / 8 + g) + 8 * pl) =
            uint4{pk[g][pl][0], pk[g][pl][1], pk[g][pl][2], pk[g][pl][3]};
  }
};

// Write a split-precision tile's accumulators to an SP matrix Y whose rows
// are the tile's columns and whose k index is the tile's row: tile element
// (row, col) goes to Y row col0 + col, k = row0 + row.  Each lane holds four
// consecutive tile rows of one column (half of an 8-group) and writes 8 bytes
// per plane.  Rows at or beyond krows and columns at or beyond cols are not
// written (krows a multiple of 4).
template <class Cfg>
__device__ __forceinline__ void acc_store_sp_t(const AccTile<Cfg>& acc, void* Y, int64_t gpr,
                                               int row0, int col0, int krows, int cols) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int wr = wid / Cfg::WGN, wc = wid % Cfg::WGN;
  char* y = reinterpret_cast<char*>(Y);
#pragma unroll
  for (int a = 0; a < Cfg::MB; ++a)
#pragma unroll
    for (int b = 0; b < Cfg::NB; ++b) {
      const int row = row0 + wr * Cfg::WTM + a * 16 + 4 * (lane >> 4);
      const int col = col0 + wc * Cfg::WTN + b * 16 + (lane & 15);
      if (row >= krows || col >= cols) continue;
      uint32_t rh[2], rl[2], ih[2], il[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        split2(acc.re[a][b][2 * u], acc.re[a][b][2 * u + 1], rh[u], rl[u]);
        split2(acc.im[a][b][2 * u], acc.im[a][b][2 * u + 1], ih[u], il[u]);
      }
      char* g = y + ((int64_t)col * gpr + (row >> 3)) * 64 + ((row & 7) >> 2) * 8;
      *reinterpret_cast<uint2*>(g) = uint2{rh[0], rh[1]};
      *reinterpret_cast<uint2*>(g + 16) = uint2{rl[0], rl[1]};
      *reinterpret_cast<uint2*>(g + 32) = uint2{ih[0], ih[1]};
      *reinterpret_cast<uint2*>(g + 48) = uint2{il[0], il[1]};
    }
}

}  // namespace pinv
