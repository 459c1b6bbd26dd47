// Forward model D = E X (Eq. 1), adjoint Z = E^H D, the normal-equation
// residual through the Gram (Eq. 6), triangular products on frame blocks
// (refinement correction and factor-only solves) and precision conversions.
#include <type_traits>

#include "pinv_internal.h"

namespace pinv {

// ---------------------------------------------------------------------------
// Forward model D[f][m] = sum_n X[f][n] E[m][n]  (S = storage type of X).
// With `sub` set the result is Dout = Din - E x (refinement residual).
// ---------------------------------------------------------------------------
template <class Cfg, int FEAT, typename SX, typename SD, bool AL>
__global__ __launch_bounds__(256, 2) void k_forward(EncDev<typename Cfg::T> e, const SX* __restrict__ X,
                                                 int F, const SD* __restrict__ Din,
                                                 typename Cfg::T* __restrict__ Dout) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbj = (M + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = t / nbj, bj = t % nbj;
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, SX, false> la;
  la.p = reinterpret_cast<const cx<SX>*>(X);
  la.ld = N;
  la.o0 = bi * Cfg::BM;
  la.oend = F;
  LoadGenRow<Cfg, Cfg::BN, Cfg::LDB, false, FEAT, AL> lb;
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, N, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(Dout);
  const cx<SD>* Di = reinterpret_cast<const cx<SD>*>(Din);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < F && col < M) {
      const size_t o = (size_t)row * M + col;
      if (Di) {
        cx<SD> d = Di[o];
        O[o] = cx<T>{T(d.re) - re, T(d.im) - im};
      } else {
        O[o] = cx<T>{re, im};
      }
    }
  });
}

// Adjoint Z[f][n] = sum_m D[f][m] conj(E[m][n]);  with X given, Z -= lam * X.
// The result is written with storage type SO.
// With a split of the contraction (ksplit > 1, `work` non-null) workgroup
// blockIdx = split * tiles + tile sums rows m in [split*kchunk, +kchunk) and
// stores its raw partial tile to work[split]; k_split_reduce then adds the
// partials in split order (deterministic) and applies the -lam x term.
template <class Cfg, int FEAT, typename SD, typename SX, typename SO, bool AL>
__global__ __launch_bounds__(256, (MinBlocks<Cfg, FEAT>::value)) void k_adjoint(EncDev<typename Cfg::T> e, const SD* __restrict__ D,
                                                 int F, const SX* __restrict__ X, double lam,
                                                 SO* __restrict__ Z, int tiles, int kchunk,
                                                 typename Cfg::T* __restrict__ work) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int split = blockIdx.x / tiles;
  const int t = blockIdx.x - split * tiles;
  const int bi = t / nbj, bj = t % nbj;
  const int k0 = split * kchunk, k1 = min(M, k0 + kchunk);
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, SD, false> la;
  la.p = reinterpret_cast<const cx<SD>*>(D);
  la.ld = M;
  la.o0 = bi * Cfg::BM;
  la.oend = F;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, true, FEAT, AL> lb;
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, k0, k1, acc, smem_base<Cfg>());
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  if (work) {
    cx<T>* W = reinterpret_cast<cx<T>*>(work) + (size_t)split * F * N;
    acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
      const int row = r0 + r, col = c0 + c;
      if (row < F && col < N) W[(size_t)row * N + col] = cx<T>{re, im};
    });
    return;
  }
  cx<SO>* O = reinterpret_cast<cx<SO>*>(Z);
  const cx<SX>* Xc = reinterpret_cast<const cx<SX>*>(X);
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < F && col < N) {
      const size_t o = (size_t)row * N + col;
      T zr = re, zi = im;
      if (Xc) {
        cx<SX> x = Xc[o];
        zr -= T(lam) * T(x.re);
        zi -= T(lam) * T(x.im);
      }
      O[o] = cx<SO>{SO(zr), SO(zi)};
    }
  });
}

// Apply for a few frames: X[f][n] = sum_m D[f][m] R[n][m], each wavefront

// Triangular products on frame blocks (refinement correction, factor-only solves):
//   mode 0: Y[f][i] = sum_{n <= i} Xin[f][n] Li[i][n]          (L^-1 x, per frame)
//   mode 1: X[f][i] += sum_{n >= i} Yin[f][n] conj(Li[n][i])   (L^-H y, accumulated)
//   mode 2: X[f][i] = sum_{n >= i} Yin[f][n] conj(Li[n][i])    (L^-H y)
template <class Cfg, int MODE, typename SO>
__global__ __launch_bounds__(256) void k_tri_frames(const typename Cfg::T* __restrict__ Li,
                                                    const typename Cfg::T* __restrict__ In, int F,
                                                    int N, SO* __restrict__ Out) {
  typedef typename Cfg::T T;
  const int nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int nbi = (F + Cfg::BM - 1) / Cfg::BM;
  // A tile's contraction length grows with its distance from the triangle's
  // short end.  Rank r = 0 is the longest tile; the grid's first half takes
  // ranks in descending length and its second half in ascending length, so
  // workgroups t and t + half, which the dispatcher tends to place on one CU,
  // carry one long and one short tile.
  const int total = nbi * nbj, half = (total + 1) / 2;
  const int t = (int)blockIdx.x;
  const int r = t < half ? t : total - 1 + half - t;
  const int jr = r / nbi;                       // 0 = longest block column
  const int bi = r - jr * nbi;
  const int bj = MODE == 0 ? nbj - 1 - jr : jr;
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;
  la.p = reinterpret_cast<const cx<T>*>(In);
  la.ld = N;
  la.o0 = bi * Cfg::BM;
  la.oend = F;
  AccTile<Cfg> acc;
  acc.zero();
  if (MODE == 0) {
    LoadDenseKC<Cfg, Cfg::BN, Cfg::LDB, T, false> lb;   // (o=i, k=n) at Li[i*N+n]
    lb.p = reinterpret_cast<const cx<T>*>(Li);
    lb.ld = N;
    lb.o0 = bj * Cfg::BN;
    lb.oend = N;
    mainloop<Cfg>(la, lb, 0, min(N, (bj + 1) * Cfg::BN), acc, smem_base<Cfg>());
  } else {
    LoadDenseOC<Cfg, Cfg::BN, Cfg::LDB, T, true> lb;    // (o=i, k=n) at conj Li[n*N+i]
    lb.p = reinterpret_cast<const cx<T>*>(Li);
    lb.ld = N;
    lb.o0 = bj * Cfg::BN;
    lb.oend = N;
    mainloop<Cfg>(la, lb, bj * Cfg::BN, N, acc, smem_base<Cfg>());
  }
  cx<SO>* O = reinterpret_cast<cx<SO>*>(Out);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < F && col < N) {
      const size_t o = (size_t)row * N + col;
      if (MODE != 1) {
        O[o] = cx<SO>{SO(re), SO(im)};
      } else {
        cx<SO> x = O[o];
        O[o] = cx<SO>{SO(x.re + re), SO(x.im + im)};
      }
    }
  });
}

// Normal-equation residual through the Gram (Eq. 6):
//   Out[f][a] = b[f][a] - sum_n G[a][n] X[f][n] - lam X[f][a]
// with G the full Hermitian FP64 Gram [N][N] and b = E^H d in FP64.
template <class Cfg, typename SX, typename SO>
__global__ __launch_bounds__(256, MinBlocks<Cfg>::value) void k_resid(const double* __restrict__ G,
                                               const double* __restrict__ b,
                                               const SX* __restrict__ X, int F, int N, double lam,
                                               SO* __restrict__ Out) {
  typedef typename Cfg::T T;
  const int nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = t / nbj, bj = t % nbj;
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, SX, false> la;     // X[f][n]
  la.p = reinterpret_cast<const cx<SX>*>(X);
  la.ld = N;
  la.o0 = bi * Cfg::BM;
  la.oend = F;
  LoadDenseKC<Cfg, Cfg::BN, Cfg::LDB, double, false> lb;  // (o=a, k=n) at G[a][n]
  lb.p = reinterpret_cast<const cx<double>*>(G);
  lb.ld = N;
  lb.o0 = bj * Cfg::BN;
  lb.oend = N;
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, N, acc, smem_base<Cfg>());
  cx<SO>* O = reinterpret_cast<cx<SO>*>(Out);
  const cx<double>* bc = reinterpret_cast<const cx<double>*>(b);
  const cx<SX>* Xc = reinterpret_cast<const cx<SX>*>(X);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < F && col < N) {
      const size_t o = (size_t)row * N + col;
      const cx<double> bb = bc[o];
      const cx<SX> x = Xc[o];
      O[o] = cx<SO>{SO(bb.re - (double)re - lam * (double)x.re),
                    SO(bb.im - (double)im - lam * (double)x.im)};
    }
  });
}


// Elementwise FP64 -> FP32 complex copy (n complex values).
__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// Elementwise FP32 -> FP64 complex copy (n complex values).
__global__ void k_to_f64(const float* __restrict__ in, double* __restrict__ out, size_t n2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}


// host launchers
template <typename T, typename SX, typename SD>
hipError_t launch_forward(const EncDev<T>& e, const SX* X, int F, const SD* Din, T* Dout,
                          hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(e.M, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  return with_feat_al(enc_features(e), row_aligned(e, Cfg::BK), [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_forward<Cfg, decltype(fc)::value, SX, SD, decltype(al)::value>),
                       dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, X, F, Din, Dout);
    return hipGetLastError();
  });
}

// The adjoint's tile kernel for this encoding and its contraction split:
// f(kernel, tiles, splits, kchunk) with the split chosen to fill the last
// round of the tile grid (pick_split).
template <typename T, typename SD, typename SX, typename SO, class Fn>
static hipError_t adjoint_plan(const EncDev<T>& e, int F, Fn&& f) {
  typedef typename std::conditional<std::is_same<T, double>::value, F64Cfg3, F32Cfg>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(e.N, Cfg::BN);
  return with_feat_al(enc_features(e), e.K % Cfg::BK == 0, [&](auto fc, auto al) {
    auto kern = k_adjoint<Cfg, decltype(fc)::value, SD, SX, SO, decltype(al)::value>;
    const int nchunks = cdiv(e.M, Cfg::BK);
    const int splits =
        tiles ? pick_split(tiles, resident_blocks(kern, 256, smem_bytes<Cfg>()), nchunks) : 1;
    return f(kern, Cfg{}, tiles, splits, cdiv(nchunks, splits) * Cfg::BK);
  });
}

template <typename T, typename SD, typename SX, typename SO>
size_t adjoint_scratch_bytes(const EncDev<T>& e, int F) {
  size_t bytes = 0;
  (void)adjoint_plan<T, SD, SX, SO>(e, F, [&](auto, auto, int tiles, int splits, int) {
    if (tiles > 0 && splits > 1) bytes = (size_t)splits * F * e.N * 2 * sizeof(T);
    return hipSuccess;
  });
  return bytes;
}

template <typename T, typename SD, typename SX, typename SO>
hipError_t launch_adjoint(const EncDev<T>& e, const SD* D, int F, const SX* X, double lam, SO* Z,
                          Scratch& sc, hipStream_t s) {
  return adjoint_plan<T, SD, SX, SO>(e, F, [&](auto kern, auto cfg, int tiles, int splits,
                                               int kchunk) {
    typedef decltype(cfg) Cfg;
    if (tiles == 0) return hipSuccess;
    // split the M contraction when one pass of the tile grid would leave the
    // GPU partly idle (the grid's last round is what the split fills)
    if (splits == 1) {
      hipLaunchKernelGGL(kern, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, D, F, X, lam, Z,
                         tiles, kchunk, (T*)nullptr);
      return hipGetLastError();
    }
    const int64_t n = (int64_t)F * e.N;
    void* work = nullptr;
    hipError_t err = sc.get(&work, (size_t)splits * n * 2 * sizeof(T), s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(tiles * splits), dim3(256), smem_bytes<Cfg>(), s, e, D, F, X, lam,
                       Z, tiles, kchunk, (T*)work);
    err = hipGetLastError();
    if (err == hipSuccess) {
      const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1 << 16);
      hipLaunchKernelGGL((k_split_reduce<T, SX, SO>), dim3(blocks), dim3(256), 0, s,
                         (const T*)work, splits, n, X, lam, Z);
      err = hipGetLastError();
    }
    const hipError_t ferr = sc.put(work, s);
    return err != hipSuccess ? err : ferr;
  });
}

template <typename SX, typename SO>
hipError_t launch_resid(const double* G, const double* b, const SX* X, int F, int N, double lam,
                        SO* Out, hipStream_t s) {
  typedef F64Cfg3 Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(N, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL((k_resid<Cfg, SX, SO>), dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, G, b, X,
                     F, N, lam, Out);
  return hipGetLastError();
}


template <typename T, int MODE, typename SO>
hipError_t launch_tri_frames(const T* Li, const T* In, int F, int N, SO* Out, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(N, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL((k_tri_frames<Cfg, MODE, SO>), dim3(tiles), dim3(256), smem_bytes<Cfg>(), s,
                     Li, In, F, N, Out);
  return hipGetLastError();
}


hipError_t launch_to_f64(const float* in, double* out, size_t n_complex, hipStream_t s) {
  const size_t n2 = 2 * n_complex;
  int blocks = (int)std::min<size_t>(4096, (n2 + 255) / 256);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_to_f64, dim3(blocks), dim3(256), 0, s, in, out, n2);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* in, float* out, size_t n_complex, hipStream_t s) {
  const size_t n2 = 2 * n_complex;
  int blocks = (int)std::min<size_t>(4096, (n2 + 255) / 256);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, s, in, out, n2);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_forward<float, float, float>(const EncDev<float>&, const float*, int,
                                                        const float*, float*, hipStream_t);
template hipError_t launch_forward<double, double, double>(const EncDev<double>&, const double*, int,
                                                           const double*, double*, hipStream_t);
template hipError_t launch_forward<double, float, float>(const EncDev<double>&, const float*, int,
                                                         const float*, double*, hipStream_t);
template hipError_t launch_resid<float, float>(const double*, const double*, const float*, int, int,
                                               double, float*, hipStream_t);
template hipError_t launch_resid<double, double>(const double*, const double*, const double*, int,
                                                 int, double, double*, hipStream_t);
template hipError_t launch_resid<double, float>(const double*, const double*, const double*, int,
                                                int, double, float*, hipStream_t);
template hipError_t launch_tri_frames<float, 1, double>(const float*, const float*, int, int, double*,
                                                        hipStream_t);
template hipError_t launch_tri_frames<float, 2, double>(const float*, const float*, int, int, double*,
                                                        hipStream_t);
template hipError_t launch_tri_frames<float, 0, float>(const float*, const float*, int, int, float*,
                                                       hipStream_t);
template hipError_t launch_tri_frames<float, 1, float>(const float*, const float*, int, int, float*,
                                                       hipStream_t);
template hipError_t launch_tri_frames<double, 0, double>(const double*, const double*, int, int,
                                                         double*, hipStream_t);
template hipError_t launch_tri_frames<double, 1, double>(const double*, const double*, int, int,
                                                         double*, hipStream_t);
template hipError_t launch_tri_frames<double, 2, double>(const double*, const double*, int, int,
                                                         double*, hipStream_t);
template hipError_t launch_tri_frames<float, 2, float>(const float*, const float*, int, int, float*,
                                                       hipStream_t);
template hipError_t launch_adjoint<double, double, float, float>(const EncDev<double>&, const double*, int,
    const float*, double, float*, Scratch&, hipStream_t);
template size_t adjoint_scratch_bytes<double, double, float, float>(const EncDev<double>&, int);
template hipError_t launch_adjoint<double, double, double, double>(const EncDev<double>&, const double*, int,
    const double*, double, double*, Scratch&, hipStream_t);
template size_t adjoint_scratch_bytes<double, double, double, double>(const EncDev<double>&, int);
template hipError_t launch_adjoint<double, float, float, double>(const EncDev<double>&, const float*, int,
    const float*, double, double*, Scratch&, hipStream_t);
template size_t adjoint_scratch_bytes<double, float, float, double>(const EncDev<double>&, int);
template hipError_t launch_adjoint<double, float, float, float>(const EncDev<double>&, const float*, int,
    const float*, double, float*, Scratch&, hipStream_t);
template size_t adjoint_scratch_bytes<double, float, float, float>(const EncDev<double>&, int);
template hipError_t launch_adjoint<float, float, float, float>(const EncDev<float>&, const float*, int,
    const float*, double, float*, Scratch&, hipStream_t);
template size_t adjoint_scratch_bytes<float, float, float, float>(const EncDev<float>&, int);

}  // namespace pinv
