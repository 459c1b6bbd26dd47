// Triangular products forming R (Eq. 8): W = L^-1 E^H with E^H generated per
// tile, R = L^-H W; and the right pseudoinverse's products (Sec. 2.2).
#include <type_traits>

#include "pinv_internal.h"

namespace pinv {

// ---------------------------------------------------------------------------
// W = L^-1 E^H : W[i][m] = sum_{n <= i} Li[i][n] conj(E[m][n])
// ---------------------------------------------------------------------------
// `rows` rows of W; Li is lower triangular (tri, rows = N) or dense
// (rows x N: the eigenvalue route's Q^H).
template <class Cfg, int FEAT, bool AL>
__global__ __launch_bounds__(256) void k_trmm_w(EncDev<typename Cfg::T> e,
                                                const typename Cfg::T* __restrict__ Li,
                                                typename Cfg::T* __restrict__ W, int rows, int tri) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbi = (rows + Cfg::BM - 1) / Cfg::BM, nbj = (M + Cfg::BN - 1) / Cfg::BN;
  // each XCD runs column groups of 8 sample blocks over every row block
  // (longest K ranges first): its resident tiles share the E tables of 8
  // sample blocks and the L^-1 rows of a few row blocks
  int r, bj;
  grouped_tile<8>(xcd_contiguous(blockIdx.x, nbi * nbj), nbi, nbj, &r, &bj);
  const int bi = nbi - 1 - r;
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;
  la.p = reinterpret_cast<const cx<T>*>(Li);
  la.ld = N;
  la.o0 = bi * Cfg::BM;
  la.oend = rows;
  LoadGenRow<Cfg, Cfg::BN, Cfg::LDB, true, FEAT, AL> lb;
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  const int kend = tri ? min(N, (bi + 1) * Cfg::BM) : N;
  mainloop<Cfg>(la, lb, 0, kend, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(W);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < rows && col < M) O[(size_t)row * M + col] = cx<T>{re, im};
  });
}

// Right pseudoinverse, first product: W'[i][n] = sum_{m <= i} Li'[i][m] E[m][n]
// with L' the factor of the samples' Gram (M x M) and E generated column-wise.
template <class Cfg, int FEAT, bool AL>
__global__ __launch_bounds__(256) void k_trmm_w_rows(EncDev<typename Cfg::T> e,
                                                     const typename Cfg::T* __restrict__ Li,
                                                     typename Cfg::T* __restrict__ W) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbi = (M + Cfg::BM - 1) / Cfg::BM, nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = nbi - 1 - t / nbj, bj = t % nbj;   // longest K ranges first
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;
  la.p = reinterpret_cast<const cx<T>*>(Li);
  la.ld = M;
  la.o0 = bi * Cfg::BM;
  la.oend = M;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, false, FEAT, AL> lb;
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, min(M, (bi + 1) * Cfg::BM), acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(W);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < M && col < N) O[(size_t)row * N + col] = cx<T>{re, im};
  });
}

// R[n][m] = conj(Z[m][n]) through 32 x 32 LDS tiles (Z: M x N, R: N x M).
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_conj_transpose(const T* __restrict__ Z, TO* __restrict__ R,
                                                        int M, int N) {
  __shared__ cx<T> tile[32][33];
  const int n0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  const cx<T>* z = reinterpret_cast<const cx<T>*>(Z);
  cx<TO>* r = reinterpret_cast<cx<TO>*>(R);
  for (int j = ty; j < 32; j += 8) {
    const int m = m0 + j, n = n0 + tx;
    if (m < M && n < N) tile[j][tx] = z[(size_t)m * N + n];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int n = n0 + j, m = m0 + tx;
    if (m < M && n < N) {
      const cx<T> v = tile[tx][j];
      r[(size_t)n * M + m] = cx<TO>{TO(v.re), TO(-v.im)};
    }
  }
}

// R = L^-H W : R[i][m] = sum_{n >= i} conj(Li[n][i]) W[n][m], stored as TO
// (an FP64 product rounded once to complex64 for FP32 plans whose R is formed
// in FP64)
// Li is lower triangular (tri, kdim = N: the sum runs over n >= i) or dense
// (kdim x N, the eigenvalue route's Q^H: the sum runs over n < kdim).
template <class Cfg, typename TO = typename Cfg::T>
__global__ __launch_bounds__(256) void k_trmm_r(const typename Cfg::T* __restrict__ Li,
                                                const typename Cfg::T* __restrict__ W,
                                                TO* __restrict__ R, int N, int M, int kdim, int tri) {
  typedef typename Cfg::T T;
  const int nbi = (N + Cfg::BM - 1) / Cfg::BM, nbj = (M + Cfg::BN - 1) / Cfg::BN;
  // each XCD runs column groups of 8 W panels over every row block (longest K
  // ranges first), and the contraction runs from n = N down: every tile's
  // range ends at N, so the resident tiles of several row blocks read the
  // same W rows at the same time, and those of one row block the same L^-1
  // rows
  int bi, bj;
  grouped_tile<8>(xcd_contiguous(blockIdx.x, nbi * nbj), nbi, nbj, &bi, &bj);
  LoadDenseOC<Cfg, Cfg::BM, Cfg::LDA, T, true> la;    // conj(Li[n][i]), i contiguous
  la.p = reinterpret_cast<const cx<T>*>(Li);
  la.ld = N;
  la.o0 = bi * Cfg::BM;
  la.oend = N;
  LoadDenseOC<Cfg, Cfg::BN, Cfg::LDB, T, false> lb;   // W[n][m], m contiguous
  lb.p = reinterpret_cast<const cx<T>*>(W);
  lb.ld = M;
  lb.o0 = bj * Cfg::BN;
  lb.oend = M;
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg, true, true>(la, lb, tri ? bi * Cfg::BM : 0, kdim, acc, smem_base<Cfg>());
  cx<TO>* O = reinterpret_cast<cx<TO>*>(R);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < M) O[(size_t)row * M + col] = cx<TO>{TO(re), TO(im)};
  });
}


// host launchers.  `m3` picks the complex-product form of the tiles: three
// real products per complex product (Gauss) or four.
template <typename T> struct TrmmCfg;
template <> struct TrmmCfg<float> { typedef F32Cfg m3; typedef F32Cfg4 m4; };
template <> struct TrmmCfg<double> { typedef F64Cfg3 m3; typedef F64Cfg m4; };

template <typename T, class F> static hipError_t with_form(bool m3, F&& f) {
  if (m3) return f(typename TrmmCfg<T>::m3{});
  return f(typename TrmmCfg<T>::m4{});
}

template <typename T, typename TO>
hipError_t launch_right_pinv(const EncDev<T>& e, const T* Li, T* W, T* Z, TO* R, bool m3,
                             hipStream_t s) {
  hipError_t err = with_form<T>(m3, [&](auto cfg) {
    typedef decltype(cfg) Cfg;
    const int tiles = cdiv(e.M, Cfg::BM) * cdiv(e.N, Cfg::BN);
    return with_feat_al(enc_features(e), e.K % Cfg::BK == 0, [&](auto fc, auto al) {
      hipLaunchKernelGGL((k_trmm_w_rows<Cfg, decltype(fc)::value, decltype(al)::value>),
                         dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, Li, W);
      return hipGetLastError();
    });
  });
  if (err != hipSuccess) return err;
  err = launch_trmm_r<T, T>(Li, W, Z, e.M, e.N, m3, s, -1);   // Z = L'^-H W' (M x N)
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL((k_conj_transpose<T, TO>), dim3(cdiv(e.N, 32), cdiv(e.M, 32)), dim3(256), 0, s,
                     Z, R, e.M, e.N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trmm_w(const EncDev<T>& e, const T* Li, T* W, bool m3, hipStream_t s, int rows) {
  const int tri = rows < 0;
  if (tri) rows = e.N;
  return with_form<T>(m3, [&](auto cfg) {
    typedef decltype(cfg) Cfg;
    const int tiles = cdiv(rows, Cfg::BM) * cdiv(e.M, Cfg::BN);
    if (tiles == 0) return hipSuccess;
    return with_feat_al(enc_features(e), row_aligned(e, Cfg::BK), [&](auto fc, auto al) {
      hipLaunchKernelGGL((k_trmm_w<Cfg, decltype(fc)::value, decltype(al)::value>), dim3(tiles),
                         dim3(256), smem_bytes<Cfg>(), s, e, Li, W, rows, tri);
      return hipGetLastError();
    });
  });
}

template <typename T, typename TO>
hipError_t launch_trmm_r(const T* Li, const T* W, TO* R, int N, int M, bool m3, hipStream_t s,
                         int kdim) {
  const int tri = kdim < 0;
  if (tri) kdim = N;
  return with_form<T>(m3, [&](auto cfg) {
    typedef decltype(cfg) Cfg;
    const int tiles = cdiv(N, Cfg::BM) * cdiv(M, Cfg::BN);
    hipLaunchKernelGGL((k_trmm_r<Cfg, TO>), dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, Li, W, R,
                       N, M, kdim, tri);
    return hipGetLastError();
  });
}

// explicit instantiations
template hipError_t launch_right_pinv<float, float>(const EncDev<float>&, const float*, float*,
                                                    float*, float*, bool, hipStream_t);
template hipError_t launch_right_pinv<double, double>(const EncDev<double>&, const double*, double*,
                                                      double*, double*, bool, hipStream_t);
template hipError_t launch_right_pinv<double, float>(const EncDev<double>&, const double*, double*,
                                                     double*, float*, bool, hipStream_t);
template hipError_t launch_trmm_w<float>(const EncDev<float>&, const float*, float*, bool,
                                         hipStream_t, int);
template hipError_t launch_trmm_w<double>(const EncDev<double>&, const double*, double*, bool,
                                          hipStream_t, int);
template hipError_t launch_trmm_r<float, float>(const float*, const float*, float*, int, int, bool,
                                                hipStream_t, int);
template hipError_t launch_trmm_r<double, double>(const double*, const double*, double*, int, int,
                                                  bool, hipStream_t, int);
template hipError_t launch_trmm_r<double, float>(const double*, const double*, float*, int, int,
                                                 bool, hipStream_t, int);

}  // namespace pinv
