// Image-quality metrics from an explicit reconstruction matrix R (Sec. 2.5):
//
//   srf_diag    SRF map      out[n]     = sum_m R[n][m] E[m][n]            (Eq. 9, diagonal)
//   srf_full    SRF matrix   out[n][n'] = sum_m R[n][m] E[m][n']           (Eq. 9)
//   noise_mix   R~ = R (Lc kron I_K), Psi_c = Lc Lc^H the coil noise covariance
//   noise_diag  noise map    out[n]     = sum_m |R~[n][m]|^2               (Eq. 10, diagonal)
//   noise_full  noise matrix X[n][n']   = sum_m R~[n][m] conj(R~[n'][m])   (Eq. 10)
//
// E is regenerated from the plan's tables exactly as in the build; R is read
// once per row (diagonals) or streamed through the MFMA tile mainloop (full
// matrices).
#include "pinv_internal.h"

namespace pinv {

// ---------------------------------------------------------------------------
// SRF map.  A workgroup owns 8 rows n; within each wave lane l takes row
// n0 + l/8 and the samples m = 8 w + l%8 + 32 t (w = wave), so one load
// instruction reads 8 rows x 64 contiguous bytes of R.  Partial sums are FP64,
// reduced over the 8 lanes of a row by shuffles and over the 4 waves in LDS.
// ---------------------------------------------------------------------------
template <typename T, int FEAT>
__global__ __launch_bounds__(256) void k_srf_diag(EncDev<T> e, const T* __restrict__ R,
                                                  T* __restrict__ out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = blockIdx.x * 8 + (lane >> 3);
  const int nn = n < e.N ? n : 0;
  const int s = nn / e.V, v = nn - s * e.V;
  int ix, iy;
  voxel_xy(e, v, &ix, &iy);
  const cx<T>* Rr = reinterpret_cast<const cx<T>*>(R) + (size_t)nn * e.M;
  double ar = 0.0, ai = 0.0;
  int m = w * 8 + (lane & 7);
  int c = m / e.K, i = m - c * e.K;
  for (; m < e.M; m += 32) {
    GenRaw<T> raw;
    gen_load<FEAT>(e, i, s, v, ix, iy, c, raw);
    const cx<T> el = gen_product<FEAT>(raw);
    const cx<T> r = Rr[m];
    ar += (double)r.re * (double)el.re - (double)r.im * (double)el.im;
    ai += (double)r.re * (double)el.im + (double)r.im * (double)el.re;
    i += 32;
    while (i >= e.K) {
      i -= e.K;
      ++c;
    }
  }
#pragma unroll
  for (int off = 4; off >= 1; off >>= 1) {
    ar += __shfl_xor(ar, off);
    ai += __shfl_xor(ai, off);
  }
  __shared__ double red[4][8][2];
  if ((lane & 7) == 0) {
    red[w][lane >> 3][0] = ar;
    red[w][lane >> 3][1] = ai;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int r = threadIdx.x;
    const int n2 = blockIdx.x * 8 + r;
    if (n2 < e.N) {
      const double sr = red[0][r][0] + red[1][r][0] + red[2][r][0] + red[3][r][0];
      const double si = red[0][r][1] + red[1][r][1] + red[2][r][1] + red[3][r][1];
      reinterpret_cast<cx<T>*>(out)[n2] = cx<T>{T(sr), T(si)};
    }
  }
}

// SRF matrix: tile (bi, bj) of R E, A = rows of R (k = m contiguous), B = E
// generated with a fixed column n' per thread.
template <class Cfg, int FEAT, bool AL>
__global__ __launch_bounds__(256, 2) void k_srf_full(EncDev<typename Cfg::T> e,
                                                     const typename Cfg::T* __restrict__ R,
                                                     typename Cfg::T* __restrict__ out) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int bi = blockIdx.x / nbj, bj = blockIdx.x % nbj;
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;   // R[n][m]
  la.p = reinterpret_cast<const cx<T>*>(R);
  la.ld = M;
  la.o0 = bi * Cfg::BM;
  la.oend = N;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, false, FEAT, AL> lb;   // E[m][n']
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, M, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(out);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < N) O[(size_t)row * N + col] = cx<T>{re, im};
  });
}

// ---------------------------------------------------------------------------
// Noise.  With Psi = Psi_c kron I_K and Psi_c = Lc Lc^H (Lc lower, C x C),
// X = R~ R~^H with R~[n][c' K + i] = sum_{c >= c'} R[n][c K + i] Lc[c][c'].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_noise_mix(const T* __restrict__ R, int N, int K, int C,
                                                   const T* __restrict__ Lc, T* __restrict__ Rt) {
  const cx<T>* Rc = reinterpret_cast<const cx<T>*>(R);
  const cx<T>* L = reinterpret_cast<const cx<T>*>(Lc);
  cx<T>* O = reinterpret_cast<cx<T>*>(Rt);
  const int64_t M = (int64_t)C * K;
  const int64_t total = (int64_t)N * M;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = idx / M;
    const int rem = (int)(idx - n * M);
    const int cp = rem / K, i = rem - cp * K;
    const cx<T>* row = Rc + n * M;
    T zr = T(0), zi = T(0);
    for (int c = cp; c < C; ++c) {
      const cx<T> r = row[(int64_t)c * K + i];
      const cx<T> l = L[c * C + cp];
      zr += r.re * l.re - r.im * l.im;
      zi += r.re * l.im + r.im * l.re;
    }
    O[idx] = cx<T>{zr, zi};
  }
}

// Noise map: one workgroup per row, FP64 accumulation, then a block reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_noise_diag(const T* __restrict__ R, int N, int K, int C,
                                                    const T* __restrict__ Lc, T* __restrict__ out) {
  const int n = blockIdx.x;
  const int64_t M = (int64_t)C * K;
  const cx<T>* row = reinterpret_cast<const cx<T>*>(R) + (int64_t)n * M;
  const cx<T>* L = reinterpret_cast<const cx<T>*>(Lc);
  double acc = 0.0;
  if (!Lc) {
    for (int64_t m = threadIdx.x; m < M; m += blockDim.x) {
      const cx<T> r = row[m];
      acc += (double)r.re * r.re + (double)r.im * r.im;
    }
  } else {
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
      for (int cp = 0; cp < C; ++cp) {
        double zr = 0.0, zi = 0.0;
        for (int c = cp; c < C; ++c) {
          const cx<T> r = row[(int64_t)c * K + i];
          const cx<T> l = L[c * C + cp];
          zr += (double)r.re * l.re - (double)r.im * l.im;
          zi += (double)r.re * l.im + (double)r.im * l.re;
        }
        acc += zr * zr + zi * zi;
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[n] = T(red[0] + red[1] + red[2] + red[3]);
}

// Noise matrix: lower tiles bi >= bj of A A^H.  Each entry on or below the
// diagonal is written together with its conjugate above it, so X is returned
// in full and exactly Hermitian (in diagonal tiles only the lower half of the
// tile is used).
template <class Cfg>
__global__ __launch_bounds__(256, 2) void k_noise_full(const typename Cfg::T* __restrict__ A, int N,
                                                       int M, typename Cfg::T* __restrict__ X,
                                                       int tiles, int kchunk) {
  typedef typename Cfg::T T;
  static_assert(Cfg::BM == Cfg::BN, "square tiles");
  // with a split of the M contraction, X points at work[split] (partial sums)
  const int split = blockIdx.x / tiles;
  int bi, bj;
  tri_index(blockIdx.x - split * tiles, &bi, &bj);
  X += (size_t)split * N * N * 2;
  const int k0 = split * kchunk, k1 = min(M, k0 + kchunk);
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;   // A[n][m]
  la.p = reinterpret_cast<const cx<T>*>(A);
  la.ld = M;
  la.o0 = bi * Cfg::BM;
  la.oend = N;
  LoadDenseKC<Cfg, Cfg::BN, Cfg::LDB, T, true> lb;    // conj(A[n'][m])
  lb.p = reinterpret_cast<const cx<T>*>(A);
  lb.ld = M;
  lb.o0 = bj * Cfg::BN;
  lb.oend = N;
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, k0, k1, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(X);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < N && row >= col) {
      if (row == col) {
        O[(size_t)row * N + col] = cx<T>{re, T(0)};   // a Hermitian diagonal is real
      } else {
        O[(size_t)row * N + col] = cx<T>{re, im};
        O[(size_t)col * N + row] = cx<T>{re, -im};
      }
    }
  });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_srf_diag(const EncDev<T>& e, const T* R, T* out, hipStream_t s) {
  return with_feat(enc_features(e), [&](auto fc) {
    hipLaunchKernelGGL((k_srf_diag<T, decltype(fc)::value>), dim3(cdiv(e.N, 8)), dim3(256), 0, s, e,
                       R, out);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_srf_full(const EncDev<T>& e, const T* R, T* out, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(e.N, Cfg::BM) * cdiv(e.N, Cfg::BN);
  return with_feat_al(enc_features(e), e.K % Cfg::BK == 0, [&](auto fc, auto al) {
    auto kern = k_srf_full<Cfg, decltype(fc)::value, decltype(al)::value>;
    hipError_t err = allow_smem(kern, smem_bytes<Cfg>());
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, R, out);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_noise_mix(const T* R, int N, int K, int C, const T* Lc, T* Rt, hipStream_t s) {
  const int64_t total = (int64_t)N * C * K;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_noise_mix<T>, dim3(blocks), dim3(256), 0, s, R, N, K, C, Lc, Rt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_noise_diag(const T* R, int N, int K, int C, const T* Lc, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_noise_diag<T>, dim3(N), dim3(256), 0, s, R, N, K, C, Lc, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_noise_full(const T* A, int N, int M, T* X, hipStream_t s) {
  typedef typename GramCfgOf<T>::type Cfg;   // square tiles for the triangular grid
  const int nb = cdiv(N, Cfg::BM);
  const int tiles = nb * (nb + 1) / 2;
  hipError_t err = allow_smem(k_noise_full<Cfg>, smem_bytes<Cfg>());
  if (err != hipSuccess) return err;
  const int nchunks = cdiv(M, Cfg::BK);
  const int splits = pick_split(tiles, resident_blocks(k_noise_full<Cfg>, 256, smem_bytes<Cfg>()),
                                nchunks);
  const int kchunk = cdiv(nchunks, splits) * Cfg::BK;
  if (splits == 1) {
    hipLaunchKernelGGL(k_noise_full<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, A, N, M, X,
                       tiles, kchunk);
    return hipGetLastError();
  }
  const int64_t n = (int64_t)N * N;
  void* work = nullptr;
  err = hipMallocAsync(&work, (size_t)splits * n * 2 * sizeof(T), s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_noise_full<Cfg>, dim3(tiles * splits), dim3(256), smem_bytes<Cfg>(), s, A, N,
                     M, (T*)work, tiles, kchunk);
  err = hipGetLastError();
  if (err == hipSuccess) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL((k_split_reduce<T, T, T>), dim3(blocks), dim3(256), 0, s, (const T*)work,
                       splits, n, (const T*)nullptr, 0.0, X);
    err = hipGetLastError();
  }
  const hipError_t ferr = hipFreeAsync(work, s);
  return err != hipSuccess ? err : ferr;
}

template hipError_t launch_srf_diag<float>(const EncDev<float>&, const float*, float*, hipStream_t);
template hipError_t launch_srf_diag<double>(const EncDev<double>&, const double*, double*,
                                            hipStream_t);
template hipError_t launch_srf_full<float>(const EncDev<float>&, const float*, float*, hipStream_t);
template hipError_t launch_srf_full<double>(const EncDev<double>&, const double*, double*,
                                            hipStream_t);
template hipError_t launch_noise_mix<float>(const float*, int, int, int, const float*, float*,
                                            hipStream_t);
template hipError_t launch_noise_mix<double>(const double*, int, int, int, const double*, double*,
                                             hipStream_t);
template hipError_t launch_noise_diag<float>(const float*, int, int, int, const float*, float*,
                                             hipStream_t);
template hipError_t launch_noise_diag<double>(const double*, int, int, int, const double*, double*,
                                              hipStream_t);
template hipError_t launch_noise_full<float>(const float*, int, int, float*, hipStream_t);
template hipError_t launch_noise_full<double>(const double*, int, int, double*, hipStream_t);

}  // namespace pinv
