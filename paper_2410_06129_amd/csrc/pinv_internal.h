// Internal declarations shared by the kernel launchers and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "pinv_device.h"

namespace pinv {

struct ApplyItemDev {
  const void* D;   // [F][M]
  const void* R;   // [N][M]
  void* X;         // [F][N]
  int F, N, M;
  int tile0;       // first tile of this item in the grouped launch (set by the launcher)
  int ntile;       // tiles of one split (set by the launcher)
  int splits;      // contraction splits over M (set by the launcher from F, N, M alone)
  int kchunk;      // rows of M per split
  void* work;      // [splits][F][N] partial sums when splits > 1
};

constexpr int kMaxGroup = 32;
struct ApplyBatch {     // passed by value as a kernel argument
  int n;
  ApplyItemDev it[kMaxGroup];
};

// Scratch memory of one call (split-contraction partials, refinement
// vectors).  By default each request is a stream-ordered allocation from the
// device's default pool, returned by put().  Over a fixed region (the
// no-allocation entry point) it is a stack: get() hands out the next
// 256-aligned block, put() of the most recent block pops it (the stream runs
// the work in order, so a popped block is free for the next request), and a
// request beyond the region fails with hipErrorOutOfMemory.  `peak` records
// the most the stack ever held.  `reclaim`, when set, runs once after a
// pool allocation fails for lack of memory (it hands memory that other pools
// hold but do not use back to the device), and the allocation is tried again.
struct Scratch {
  char* base = nullptr;
  size_t cap = 0, top = 0, peak = 0;
  struct Block { void* p; size_t start; };
  Block stack[16];
  int depth = 0;
  void (*reclaim)(void* arg, hipStream_t s) = nullptr;
  void* reclaim_arg = nullptr;
  hipError_t get(void** p, size_t bytes, hipStream_t s) {
    if (!base) {
      hipError_t e = hipMallocAsync(p, bytes, s);
      if (e == hipErrorOutOfMemory && reclaim) {
        (void)hipGetLastError();
        reclaim(reclaim_arg, s);
        e = hipMallocAsync(p, bytes, s);
      }
      return e;
    }
    const size_t start = (top + 255) & ~size_t(255);
    if (depth >= 16 || start + bytes > cap) return hipErrorOutOfMemory;
    *p = base + start;
    stack[depth++] = Block{*p, top};
    top = start + bytes;
    peak = std::max(peak, top);
    return hipSuccess;
  }
  hipError_t put(void* p, hipStream_t s) {
    if (!base) return hipFreeAsync(p, s);
    if (depth > 0 && stack[depth - 1].p == p) top = stack[--depth].start;
    return hipSuccess;
  }
};

template <typename T> hipError_t launch_gram(const EncDev<T>& e, double* G, int flush, hipStream_t s);
template <typename T> hipError_t launch_gram_shared(const EncDev<T>& e, double* G, hipStream_t s);
// Cholesky of A + lam I (FP64, in place) with L^-1 formed alongside in Li
// (zeroed by the caller); nb = 64 or 128 (two-level).
hipError_t launch_cholinv(double* A, double* Li, int N, double lam, int* info, hipStream_t s,
                          hipStream_t aux, int nb);
// Triangular products forming R; m3 selects three real products per complex
// product (else four).  R may be stored in a narrower type TO than T.  With
// rows / kdim >= 0 the factor is dense instead of lower triangular: W has
// `rows` rows (W = Q^H E^H, Q^H rows x N) and R sums over kdim rows of W
// (R = Q W), the eigenvalue route's products.
template <typename T>
hipError_t launch_trmm_w(const EncDev<T>& e, const T* Li, T* W, bool m3, hipStream_t s,
                         int rows = -1);
template <typename T, typename TO>
hipError_t launch_trmm_r(const T* Li, const T* W, TO* R, int N, int M, bool m3, hipStream_t s,
                         int kdim = -1);
// seg: the FP32 contraction in segments folded into a second accumulator set
// (plans whose R is formed in FP64).
template <typename T>
hipError_t launch_apply(const ApplyBatch& b, bool m3, bool seg, Scratch& sc, hipStream_t s);
// Scratch bytes launch_apply needs for one item of F frames (split partials).
template <typename T> size_t apply_scratch_bytes(int F, int N, int M, bool m3, bool seg);
// Fewer samples than unknowns: the samples' Gram E E^H (FP64, M x M), and
// R = (L'^-H L'^-1 E)^H from the inverse factor L'^-1 (W, Z: M x N workspaces).
hipError_t launch_gram_rows(const EncDev<double>& e, double* G, hipStream_t s);
template <typename T, typename TO>
hipError_t launch_right_pinv(const EncDev<T>& e, const T* Li, T* W, T* Z, TO* R, bool m3,
                             hipStream_t s);
// Applies of at most kRowApplyMaxF frames stream R row by row (HBM-bound),
// their contraction cut into one slice per XCD when M >= kRowSliceMinM
// (partials in scratch, apply_rows_scratch_bytes); FP32 and BF16X3 plans do
// so up to kStreamMinF - 1 frames and stream R into the matrix cores from
// there (launch_apply_stream, launch_apply_stream_sp).  (Measured at
// N = 16384, M = 262144: 16-frame row variants took 25-42 ms for 9-16
// frames; at 4-8 frames the row kernels take 6.2-8.9 ms and the streamed
// one about 5.8 ms.)
constexpr int kRowApplyMaxF = 8;
constexpr int kStreamMinF = 3;
constexpr int kStreamMaxF = 32;
// The most frames a plan applies with the row kernel (streamed: an FP32 or
// BF16X3 plan, whose applies of kStreamMinF .. kStreamMaxF frames stream).
inline int row_apply_max_frames(bool streamed) { return streamed ? kStreamMinF - 1 : kRowApplyMaxF; }
constexpr int kRowSliceMinM = 8192;
int row_slices(int M);
template <typename T> size_t apply_rows_scratch_bytes(int F, int N, int M);
template <typename T>
hipError_t launch_apply_rows(const T* R, const T* D, T* X, int N, int M, int F, Scratch& sc,
                             hipStream_t s);
// FP32 applies of kStreamMinF to kStreamMaxF frames stream R through the
// matrix cores (m3: the plan's complex-product form), their contraction in
// slices of at most 4096 columns when M >= kRowSliceMinM (partials in
// scratch, apply_stream_scratch_bytes).
size_t apply_stream_scratch_bytes(int F, int N, int M);
hipError_t launch_apply_stream(const float* R, const float* D, float* X, int N, int M, int F,
                               bool m3, Scratch& sc, hipStream_t s);
// The same for a BF16X3 plan: split-packed R (N rows of Mp = sp_cols(M)
// columns) and data (F rows of Mp columns).
hipError_t launch_apply_stream_sp(const void* R, const void* D, float* X, int N, int Mp, int F,
                                  Scratch& sc, hipStream_t s);
template <typename T, typename SX, typename SD>
hipError_t launch_forward(const EncDev<T>& e, const SX* X, int F, const SD* Din, T* Dout,
                          hipStream_t s);
template <typename T, typename SD, typename SX, typename SO>
hipError_t launch_adjoint(const EncDev<T>& e, const SD* D, int F, const SX* X, double lam, SO* Z,
                          Scratch& sc, hipStream_t s);
// Scratch bytes of launch_adjoint<T, ...> for F frames (split partials).
template <typename T, typename SD, typename SX, typename SO>
size_t adjoint_scratch_bytes(const EncDev<T>& e, int F);
template <typename SX, typename SO>
hipError_t launch_resid(const double* G, const double* b, const SX* X, int F, int N, double lam,
                        SO* Out, hipStream_t s);
hipError_t launch_herm_fill(double* G, int N, hipStream_t s);
// The eigenvalue route: Jacobi eigendecomposition of the FP64 Hermitian N x N
// matrix A (A2, V, V2: same-size workspaces; the results end in *A_out and
// *V_out, two of the four), synchronising s once per sweep (*sweeps = -1 when
// max_sweeps did not converge); then the eigenvalues sorted largest first into
// spec, the kept count (PINV_TRUNC_* mode and value) into *rank, and
// Q^H = diag(1/sqrt(mu_j + lam)) P_r^H into Qh (N x N, rows >= rank zero).
// `work` holds eig_work_bytes(N).
size_t eig_work_bytes(int N);
hipError_t launch_jacobi_eig(double* A, double* A2, double* V, double* V2, int N, void* work,
                             int max_sweeps, hipStream_t s, int* sweeps, double** A_out,
                             double** V_out);
hipError_t launch_eig_select(const double* A, const double* V, int N, int mode, double value,
                             double lam, double* spec, double* Qh, int* info, void* work, int* rank,
                             hipStream_t s);

// Gram through the point-spread function (no off-resonance map): G and Gk
// (both full N x N FP64) from the FP64 tables; `work` holds psf_work_bytes.
size_t psf_work_bytes(const EncDev<double>& e, int* splits);
hipError_t launch_psf_gram(const EncDev<double>& e, void* work, double* G, double* Gk,
                           hipStream_t s);
template <typename T, int MODE, typename SO>
hipError_t launch_tri_frames(const T* Li, const T* In, int F, int N, SO* Out, hipStream_t s);
// Split-precision (BF16x3) plans keep their operands split-packed (SP): a
// complex matrix with k contiguous, rows of sp_cols(K) columns (zero past K),
// each 8 consecutive k of a row stored as bf16 planes re_hi, re_lo, im_hi,
// im_lo (64 bytes).
inline int64_t sp_cols(int64_t K) { return (K + 31) / 32 * 32; }
// dst (rows x sp_cols(K), SP) from complex src(r, k) = src[r*ld + k] (or
// src[k*ld + r] with trans), conjugated with conj.
template <typename S>
hipError_t launch_sp_pack(const S* src, int64_t ld, int rows, int K, bool trans, bool conj,
                          void* dst, hipStream_t s);
// dst (rows x K complex64) = hi + lo of an SP matrix.
hipError_t launch_sp_unpack(const void* sp, int rows, int K, float* dst, hipStream_t s);
// W^T (SP, M rows, k = n) from L^-1 (SP, N rows); R (SP, N rows, k = m) from
// W^T and L^-H (SP, N rows: conj(Li[n'][n]) at row n, k = n').
// W^T (SP, rows m, k = n) from L^-1 (SP rows) via conj(E) written to the
// workspace Es, slab_rows samples at a time (Es: 8 slab_rows sp_cols(N)
// bytes; slab_rows a multiple of 64, e_slab_rows).
hipError_t launch_trmm_w_sp(const EncDev<float>& e, const void* Li, void* W, void* Es,
                            int64_t slab_rows, hipStream_t s);
// Samples per conj(E) slab of the BF16X3 W product: about 4 GiB, a multiple
// of 512, at most M rounded up to 64.
constexpr int64_t kESlabBytes = 4ll << 30;
inline int64_t e_slab_rows(int64_t N, int64_t M) {
  const int64_t per = 8 * sp_cols(N);
  const int64_t s = std::max<int64_t>(512, kESlabBytes / per / 512 * 512);
  return std::min<int64_t>(s, (M + 63) / 64 * 64);
}
hipError_t launch_trmm_r_sp(const void* W, const void* Lh, void* R, int N, int M, hipStream_t s);
// Grouped apply on SP operands: items carry D (SP, F rows) and R (SP, N rows)
// with M = the padded contraction length sp_cols(M).
hipError_t launch_apply_b3(const ApplyBatch& b, Scratch& sc, hipStream_t s);
size_t apply_scratch_bytes_b3(int F, int N, int Mp);
// At most kRowApplyMaxF frames of complex64 data against an SP R.
hipError_t launch_apply_rows_sp(const void* R, const float* D, float* X, int N, int M, int F,
                                Scratch& sc, hipStream_t s);
hipError_t launch_to_f32(const double* in, float* out, size_t n_complex, hipStream_t s);
hipError_t launch_to_f64(const float* in, double* out, size_t n_complex, hipStream_t s);
template <typename T> hipError_t launch_srf_diag(const EncDev<T>& e, const T* R, T* out, hipStream_t s);
template <typename T> hipError_t launch_srf_full(const EncDev<T>& e, const T* R, T* out, hipStream_t s);
template <typename T>
hipError_t launch_noise_mix(const T* R, int N, int K, int C, const T* Lc, T* Rt, hipStream_t s);
template <typename T>
hipError_t launch_noise_diag(const T* R, int N, int K, int C, const T* Lc, T* out, hipStream_t s);
template <typename T> hipError_t launch_noise_full(const T* A, int N, int M, T* X, hipStream_t s);

// ---------------------------------------------------------------------------
// Tile kernels: shared device helpers and launch configuration
// ---------------------------------------------------------------------------
template <class Cfg>
__device__ __forceinline__ typename Cfg::T* smem_base() {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  return reinterpret_cast<typename Cfg::T*>(smem_raw);
}

// Workgroup t of a grid of T runs on XCD t % 8: the dispatcher deals
// workgroups round-robin over the eight XCDs, each with its own L2.  This
// renumbering gives every XCD a contiguous range of logical tiles (a
// bijection of [0, T)), so tiles that are adjacent in logical order, and
// share operands, run on one XCD and hit one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_contiguous(int t, int T) {
  const int x = t % kXcds, l = t / kXcds;
  const int per = T / kXcds, rem = T % kXcds;
  return x * per + min(x, rem) + l;
}

// Logical tile u of an nbi x nbj grid in column groups of GJ: within a group
// the GJ columns of one row come together, rows in the order `row_of` gives
// (so a block of resident tiles spans a few rows and GJ columns: each
// column's operand is shared by the rows, each row's by the columns).
template <int GJ>
__device__ __forceinline__ void grouped_tile(int u, int nbi, int nbj, int* r, int* col) {
  const int g = u / (nbi * GJ);
  const int gw = min(GJ, nbj - g * GJ);
  const int local = u - g * nbi * GJ;
  *r = local / gw;
  *col = g * GJ + local % gw;
}

// Lower-triangular tile index -> (bi, bj), bi >= bj.
__device__ __forceinline__ void tri_index(int t, int* bi, int* bj) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *bi = i;
  *bj = t - i * (i + 1) / 2;
}

// Workgroups per CU that a kernel's register budget is sized for: three for
// FP64 3M tiles whose generated operand carries no species or off-resonance
// factor (the refinement's FP64 products then fit 168 registers and their LDS
// fits three times), two otherwise (the Gram's accumulators and the extra
// factors spill at 168).
template <class Cfg, int FEAT = 0> struct MinBlocks {
  static constexpr int value =
      (sizeof(typename Cfg::T) == 8 && IsM3<Cfg>::value && (FEAT & ~FEAT_COIL) == 0) ? 3 : 2;
};

// FP32 tiles: 3M complex products on 128x64 tiles (a 64x32 tile per wave keeps
// the three accumulator sets at 96 registers, so two workgroups fit per CU)
typedef TileCfg<float, 128, 64, 8, true> F32Cfg;
typedef TileCfg<float, 128, 64, 8, false> F32Cfg4;   // the same tiles with four real products
typedef TileCfg<double, 64, 64, 8> F64Cfg;
// FP64 tiles with 3M products, for the FP64 work of FP32-class plans (Gram,
// refinement residuals), where 3M's rounding (a few units of 2^-53 more in the
// imaginary part) is far below what that work needs
typedef TileCfg<double, 64, 64, 8, true> F64Cfg3;

template <typename T> struct GramCfgOf;     // square tiles for the triangular Gram grid
template <> struct GramCfgOf<float> { typedef TileCfg<float, 128, 128, 8, false> type; };
template <> struct GramCfgOf<double> { typedef F64Cfg3 type; };

template <class Cfg> static size_t smem_bytes() { return Cfg::SMEM_ELEMS * sizeof(typename Cfg::T); }

// BF16x3 tiles: 128 x 64 over four wavefronts of 64 x 32 with one 52 KB LDS
// stage, so two workgroups share a CU (two wavefronts per SIMD, at most 256
// registers each) and one's stores and barriers overlap the other's matrix
// products.  Measured at N = 16384, M = 262144 (W, R product ms; MFMA busy):
//   128 x 128, 4 waves of 64 x 64, two stages, one workgroup per CU: 1060, 848
//   128 x 128, 8 waves of 64 x 32, two stages, one workgroup per CU:  916, 744 (0.38, 0.46)
//   128 x 64, 4 waves, one stage, two workgroups per CU:              820, 730 (0.44, 0.55)
//   the same with the issue priority raised over the products:        813, 686 (0.43, 0.56)
typedef TileCfgB3<128, 64, 2, 2, 1> B3Cfg;

// Kernels whose LDS exceeds the default 64 KB limit need the attribute once.
template <class K> static hipError_t allow_smem(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T> struct PickCfg;
template <> struct PickCfg<float> { typedef F32Cfg type; };
template <> struct PickCfg<double> { typedef F64Cfg type; };

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// The row-generated loaders' aligned chunk path (LoadGenRow): every BK
// consecutive columns lie in one image row, which needs nx % BK == 0 and no
// voxel mask.
template <typename T> static inline bool row_aligned(const EncDev<T>& e, int bk) {
  return e.nx % bk == 0 && e.vxy == nullptr;
}

// Calls f(std::integral_constant<int, FEAT>) for the runtime feature mask.
template <class F> static hipError_t with_feat(int feat, F&& f) {
  switch (feat & 7) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    default: return f(std::integral_constant<int, 7>{});
  }
}

// Workgroups of `kernel` resident on the current device at once (occupancy
// per CU times the CU count), cached per kernel and device.
template <class K> static int resident_blocks(K kernel, int threads, size_t smem) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  const auto key = std::make_pair((const void*)kernel, dev);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, smem) != hipSuccess)
    return 1;
  const int r = std::max(1, per) * std::max(1, cus);
  std::lock_guard<std::mutex> g(mu);
  cache[key] = r;
  return r;
}

// Split factor s of a contraction of `kchunks` chunks over a grid of `tiles`
// workgroups with `slots` resident at once: the s (1..4, at least 16 chunks
// per split) with the fewest full-length rounds ceil(tiles * s / slots) / s.
static inline int pick_split(long tiles, int slots, int kchunks, int max_split = 4) {
  int best = 1;
  double best_cost = (double)((tiles + slots - 1) / slots);
  for (int s = 2; s <= max_split && kchunks / s >= 16; ++s) {
    const double cost = (double)((tiles * s + slots - 1) / slots) / s;
    if (cost < best_cost - 1e-9) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}

// Z = sum_s work[s] (in split order) - lam X, elementwise over n complex values.
template <typename T, typename SX, typename SO>
__global__ __launch_bounds__(256) void k_split_reduce(const T* __restrict__ work, int splits,
                                                      int64_t n, const SX* __restrict__ X,
                                                      double lam, SO* __restrict__ Z) {
  const cx<T>* W = reinterpret_cast<const cx<T>*>(work);
  const cx<SX>* Xc = reinterpret_cast<const cx<SX>*>(X);
  cx<SO>* O = reinterpret_cast<cx<SO>*>(Z);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T zr = W[i].re, zi = W[i].im;
    for (int s = 1; s < splits; ++s) {
      zr += W[(int64_t)s * n + i].re;
      zi += W[(int64_t)s * n + i].im;
    }
    if (Xc) {
      zr -= T(lam) * T(Xc[i].re);
      zi -= T(lam) * T(Xc[i].im);
    }
    O[i] = cx<SO>{SO(zr), SO(zi)};
  }
}

// As with_feat, plus std::bool_constant<aligned> for the generated loaders'
// aligned chunk path (the launcher states the alignment condition).
template <class F> static hipError_t with_feat_al(int feat, bool aligned, F&& f) {
  return with_feat(feat, [&](auto fc) {
    return aligned ? f(fc, std::true_type{}) : f(fc, std::false_type{});
  });
}


}  // namespace pinv
