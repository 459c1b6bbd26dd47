// Kernels of the Pinv-Recon hot path for gfx950 and their host-side launchers.
//
//   gram        G = E^H E, lower block tiles, E generated per tile   (Sec. 2.2; Eq. 11)
//   chol_*      blocked right-looking Cholesky of G + lam I in FP64,  (Eq. 6, Eq. 8; Sec. 2.3)
//               producing L^-1 alongside (forward substitution on I)
//   trmm_w      W = L^-1 E^H, E^H generated per tile                  (Eq. 8)
//   trmm_r      R = L^-H W                                            (Eq. 8)
//   apply       X = D R^T  (image = R data for every frame)          (Eq. 3)
//   forward     D = X E^T  (data = E image, Eq. 1), optionally d - E x
//   adjoint     Z = D conj(E), optionally minus lam x                 (Eq. 6 residual)
//   tri_apply   products with L^-1 and L^-H for the refinement correction
#include "pinv_internal.h"

namespace pinv {

// ---------------------------------------------------------------------------
// generic tile driver
// ---------------------------------------------------------------------------
template <class Cfg>
__device__ __forceinline__ typename Cfg::T* smem_base() {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  return reinterpret_cast<typename Cfg::T*>(smem_raw);
}

// Lower-triangular tile index -> (bi, bj), bi >= bj.
__device__ __forceinline__ void tri_index(int t, int* bi, int* bj) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *bi = i;
  *bj = t - i * (i + 1) / 2;
}

// ---------------------------------------------------------------------------
// Gram: G[n1][n2] = sum_m conj(E[m][n1]) E[m][n2] for tiles bi >= bj.
// FP32 tiles flush their FP32 partial sums into the FP64 Gram every `flush`
// rows so the long sum over M is carried in FP64.
// ---------------------------------------------------------------------------
template <class Cfg>
__global__ __launch_bounds__(256) void k_gram(EncDev<typename Cfg::T> e, double* __restrict__ G,
                                              int flush) {
  typedef typename Cfg::T T;
  static_assert(Cfg::BM == Cfg::BN, "square tiles");
  int bi, bj;
  tri_index(blockIdx.x, &bi, &bj);
  const int N = e.N;
  LoadGenCol<Cfg, Cfg::BM, Cfg::LDA, true> la;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, false> lb;
  la.init(e, bi * Cfg::BM);
  lb.init(e, bj * Cfg::BN);
  T* smem = smem_base<Cfg>();
  AccTile<Cfg> acc;
  cx<double>* Gc = reinterpret_cast<cx<double>*>(G);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  bool first = true;
  for (int seg = 0; seg < e.M; seg += flush) {
    const int send = min(e.M, seg + flush);
    acc.zero();
    mainloop<Cfg>(la, lb, seg, send, acc, smem);
    acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
      const int row = r0 + r, col = c0 + c;
      if (row < N && col < N) {
        cx<double>* g = Gc + (size_t)row * N + col;
        if (first) {
          *g = cx<double>{(double)re, (double)im};
        } else {
          cx<double> o = *g;
          *g = cx<double>{o.re + (double)re, o.im + (double)im};
        }
      }
    });
    first = false;
  }
}

// ---------------------------------------------------------------------------
// Cholesky diagonal block (FP64, one workgroup): A_kk + lam I = L_kk L_kk^H,
// then L_kk^-1 by in-place triangular inversion.  The block is square nbk<=64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ A, double* __restrict__ Li,
                                                   int N, int nb, int k, double lam,
                                                   int* __restrict__ info) {
  if (*info) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<double>* S = reinterpret_cast<cx<double>*>(smem_raw);      // [nb][nb]
  cx<double>* tmp = S + 64 * 64;                                  // [64]
  __shared__ int fail;
  const int tid = threadIdx.x;
  const int k0 = k * nb;
  const int nbk = min(nb, N - k0);
  cx<double>* Ac = reinterpret_cast<cx<double>*>(A);
  cx<double>* Lc = reinterpret_cast<cx<double>*>(Li);
  for (int idx = tid; idx < nbk * nbk; idx += 256) {
    const int i = idx / nbk, j = idx - (idx / nbk) * nbk;
    cx<double> v = (j <= i) ? Ac[(size_t)(k0 + i) * N + k0 + j] : cx<double>{0.0, 0.0};
    if (i == j) v = cx<double>{v.re + lam, 0.0};
    S[i * 64 + j] = v;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  // right-looking unblocked factorisation
  for (int j = 0; j < nbk; ++j) {
    const double piv = S[j * 64 + j].re;
    if (!(piv > 0.0)) {     // also catches NaN
      if (tid == 0) {
        atomicCAS(info, 0, k0 + j + 1);
        fail = 1;
      }
      break;
    }
    const double d = sqrt(piv);
    const double inv = 1.0 / d;
    for (int i = j + 1 + tid; i < nbk; i += 256) {
      cx<double> v = S[i * 64 + j];
      S[i * 64 + j] = cx<double>{v.re * inv, v.im * inv};
    }
    __syncthreads();
    if (tid == 0) S[j * 64 + j] = cx<double>{d, 0.0};
    const int w = nbk - j - 1;
    for (int idx = tid; idx < w * w; idx += 256) {
      const int i = j + 1 + idx / w, l = j + 1 + (idx - (idx / w) * w);
      if (l <= i) {
        cx<double> a = S[i * 64 + j], b = S[l * 64 + j];
        cx<double> c = S[i * 64 + l];
        // c -= a * conj(b)
        S[i * 64 + l] = cx<double>{c.re - (a.re * b.re + a.im * b.im),
                                   c.im - (a.im * b.re - a.re * b.im)};
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail) return;
  // store L_kk (lower; zero above)
  for (int idx = tid; idx < nbk * nbk; idx += 256) {
    const int i = idx / nbk, j = idx - (idx / nbk) * nbk;
    Ac[(size_t)(k0 + i) * N + k0 + j] = (j <= i) ? S[i * 64 + j] : cx<double>{0.0, 0.0};
  }
  __syncthreads();
  // in-place inversion, last column first: with T = inverse of the trailing
  // block (already in place), column j becomes -T * L[j+1:, j] / L[j][j].
  for (int j = nbk - 1; j >= 0; --j) {
    const double ljj = S[j * 64 + j].re;
    const double ijj = 1.0 / ljj;
    // tmp[i] = sum_{l=j+1..i} T[i][l] * L[l][j],  i in (j, nbk)
    for (int i = j + 1 + tid; i < nbk; i += 256) {
      cx<double> s{0.0, 0.0};
      for (int l = j + 1; l <= i; ++l) {
        cx<double> t = S[i * 64 + l], x = S[l * 64 + j];
        s.re += t.re * x.re - t.im * x.im;
        s.im += t.re * x.im + t.im * x.re;
      }
      tmp[i] = s;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < nbk; i += 256)
      S[i * 64 + j] = cx<double>{-tmp[i].re * ijj, -tmp[i].im * ijj};
    if (tid == 0) S[j * 64 + j] = cx<double>{ijj, 0.0};
    __syncthreads();
  }
  for (int idx = tid; idx < nbk * nbk; idx += 256) {
    const int i = idx / nbk, j = idx - (idx / nbk) * nbk;
    Lc[(size_t)(k0 + i) * N + k0 + j] = (j <= i) ? S[i * 64 + j] : cx<double>{0.0, 0.0};
  }
}

// Block (bi, bj) store helper for nb x nb FP64 blocks of an N x N matrix.
typedef TileCfg<double, 64, 64, 8> CholCfg;

// Step k, after the diagonal block: for t < nblk-k-1 the panel block
// i = k+1+t becomes L_ik = A_ik L_kk^-H (in place); for the remaining k tiles
// the inverse row block becomes Y_kj = L_kk^-1 B_kj (in place), j < k.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, double* __restrict__ Li,
                                                    int N, int k, const int* __restrict__ info) {
  if (*info) return;
  typedef CholCfg Cfg;
  const int nb = 64;
  const int nblk = (N + nb - 1) / nb;
  const int npanel = nblk - k - 1;
  const int t = blockIdx.x;
  const cx<double>* Ac = reinterpret_cast<const cx<double>*>(A);
  const cx<double>* Lc = reinterpret_cast<const cx<double>*>(Li);
  double* smem = smem_base<Cfg>();
  AccTile<Cfg> acc;
  acc.zero();
  const int kend = min(N, (k + 1) * nb) - k * nb;
  int r0, c0;
  double* out;
  if (t < npanel) {
    const int i = k + 1 + t;
    r0 = i * nb;
    c0 = k * nb;
    out = A;
    LoadDenseKC<Cfg, 64, Cfg::LDA, double, false> la;   // A_ik: rows r0.., k contiguous
    la.p = Ac + (size_t)0 + k * nb;
    la.ld = N;
    la.o0 = r0;
    la.oend = N;
    LoadDenseKC<Cfg, 64, Cfg::LDB, double, true> lb;    // conj(Linv_kk[n][l])
    lb.p = Lc + (size_t)(k * nb) * N + k * nb;
    lb.ld = N;
    lb.o0 = 0;
    lb.oend = kend;
    // la indexes rows absolutely: shift its base to column k*nb of row 0
    mainloop<Cfg>(la, lb, 0, kend, acc, smem);
  } else {
    const int j = t - npanel;   // j < k
    r0 = k * nb;
    c0 = j * nb;
    out = Li;
    LoadDenseKC<Cfg, 64, Cfg::LDA, double, false> la;   // Linv_kk[m][l]
    la.p = Lc + (size_t)(k * nb) * N + k * nb;
    la.ld = N;
    la.o0 = 0;
    la.oend = kend;
    LoadDenseOC<Cfg, 64, Cfg::LDB, double, false> lb;   // B_kj[l][n] at Li[(k*nb+l)*N + j*nb+n]
    lb.p = Lc + (size_t)(k * nb) * N + j * nb;
    lb.ld = N;
    lb.o0 = 0;
    lb.oend = nb;
    mainloop<Cfg>(la, lb, 0, kend, acc, smem);
  }
  __syncthreads();
  cx<double>* O = reinterpret_cast<cx<double>*>(out);
  acc_foreach<Cfg>(acc, [&](int r, int c, double re, double im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < N) O[(size_t)row * N + col] = cx<double>{re, im};
  });
}

// Step k trailing update.  Tiles [0, nherk): A_ij -= L_ik L_jk^H for
// k < j <= i; tiles [nherk, ...): B_ij -= L_ik Y_kj for i > k, j <= k.
__global__ __launch_bounds__(256) void k_chol_trailing(double* __restrict__ A, double* __restrict__ Li,
                                                       int N, int k, const int* __restrict__ info) {
  if (*info) return;
  typedef CholCfg Cfg;
  const int nb = 64;
  const int nblk = (N + nb - 1) / nb;
  const int rem = nblk - k - 1;
  const int nherk = rem * (rem + 1) / 2;
  const int t = blockIdx.x;
  const cx<double>* Ac = reinterpret_cast<const cx<double>*>(A);
  const cx<double>* Lc = reinterpret_cast<const cx<double>*>(Li);
  double* smem = smem_base<Cfg>();
  AccTile<Cfg> acc;
  acc.zero();
  const int kw = min(N, (k + 1) * nb) - k * nb;
  int r0, c0;
  double* out;
  LoadDenseKC<Cfg, 64, Cfg::LDA, double, false> la;      // L_ik[m][l] at A[(i*nb+m)*N + k*nb + l]
  la.ld = N;
  la.oend = N;
  if (t < nherk) {
    int ti, tj;
    tri_index(t, &ti, &tj);
    const int i = k + 1 + ti, j = k + 1 + tj;
    r0 = i * nb;
    c0 = j * nb;
    out = A;
    la.p = Ac + k * nb;
    la.o0 = r0;
    LoadDenseKC<Cfg, 64, Cfg::LDB, double, true> lb;     // conj(L_jk[n][l])
    lb.p = Ac + k * nb;
    lb.ld = N;
    lb.o0 = c0;
    lb.oend = N;
    mainloop<Cfg>(la, lb, 0, kw, acc, smem);
  } else {
    const int u = t - nherk;
    const int i = k + 1 + u / (k + 1), j = u % (k + 1);
    r0 = i * nb;
    c0 = j * nb;
    out = Li;
    la.p = Ac + k * nb;
    la.o0 = r0;
    LoadDenseOC<Cfg, 64, Cfg::LDB, double, false> lb;    // Y_kj[l][n] at Li[(k*nb+l)*N + j*nb + n]
    lb.p = Lc + (size_t)(k * nb) * N;
    lb.ld = N;
    lb.o0 = c0;
    lb.oend = min(N, c0 + nb);
    mainloop<Cfg>(la, lb, 0, kw, acc, smem);
  }
  cx<double>* O = reinterpret_cast<cx<double>*>(out);
  acc_foreach<Cfg>(acc, [&](int r, int c, double re, double im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < N) {
      cx<double> o = O[(size_t)row * N + col];
      O[(size_t)row * N + col] = cx<double>{o.re - re, o.im - im};
    }
  });
}

// ---------------------------------------------------------------------------
// W = L^-1 E^H : W[i][m] = sum_{n <= i} Li[i][n] conj(E[m][n])
// ---------------------------------------------------------------------------
template <class Cfg>
__global__ __launch_bounds__(256) void k_trmm_w(EncDev<typename Cfg::T> e,
                                                const typename Cfg::T* __restrict__ Li,
                                                typename Cfg::T* __restrict__ W) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbi = (N + Cfg::BM - 1) / Cfg::BM, nbj = (M + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = nbi - 1 - t / nbj, bj = t % nbj;   // longest K ranges first
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;
  la.p = reinterpret_cast<const cx<T>*>(Li);
  la.ld = N;
  la.o0 = bi * Cfg::BM;
  la.oend = N;
  LoadGenRow<Cfg, Cfg::BN, Cfg::LDB, true> lb;
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  const int kend = min(N, (bi + 1) * Cfg::BM);
  mainloop<Cfg>(la, lb, 0, kend, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(W);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < M) O[(size_t)row * M + col] = cx<T>{re, im};
  });
}

// R = L^-H W : R[i][m] = sum_{n >= i} conj(Li[n][i]) W[n][m]
template <class Cfg>
__global__ __launch_bounds__(256) void k_trmm_r(const typename Cfg::T* __restrict__ Li,
                                                const typename Cfg::T* __restrict__ W,
                                                typename Cfg::T* __restrict__ R, int N, int M) {
  typedef typename Cfg::T T;
  const int nbj = (M + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = t / nbj, bj = t % nbj;               // longest K ranges first
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
  mainloop<Cfg>(la, lb, bi * Cfg::BM, N, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(R);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < M) O[(size_t)row * M + col] = cx<T>{re, im};
  });
}

// ---------------------------------------------------------------------------
// Apply (grouped): for each item, X[f][n] = sum_m D[f][m] R[n][m]
// ---------------------------------------------------------------------------
template <class Cfg>
__global__ __launch_bounds__(256) void k_apply(const ApplyBatch batch) {
  typedef typename Cfg::T T;
  // locate the item owning this tile (items carry exclusive tile prefix sums)
  int lo = 0, hi = batch.n - 1;
  const int t = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (batch.it[mid].tile0 <= t) lo = mid; else hi = mid - 1;
  }
  const ApplyItemDev it = batch.it[lo];
  const int u = t - it.tile0;
  const int nbj = (it.N + Cfg::BN - 1) / Cfg::BN;
  const int bi = u / nbj, bj = u % nbj;
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
  acc.zero();
  mainloop<Cfg>(la, lb, 0, it.M, acc, smem_base<Cfg>());
  cx<T>* O = reinterpret_cast<cx<T>*>(it.X);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < it.F && col < it.N) O[(size_t)row * it.N + col] = cx<T>{re, im};
  });
}

// ---------------------------------------------------------------------------
// Forward model D[f][m] = sum_n X[f][n] E[m][n]  (S = storage type of X).
// With `sub` set the result is Dout = Din - E x (refinement residual).
// ---------------------------------------------------------------------------
template <class Cfg, typename SX, typename SD>
__global__ __launch_bounds__(256) void k_forward(EncDev<typename Cfg::T> e, const SX* __restrict__ X,
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
  LoadGenRow<Cfg, Cfg::BN, Cfg::LDB, false> lb;
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
template <class Cfg, typename SX, typename SO>
__global__ __launch_bounds__(256) void k_adjoint(EncDev<typename Cfg::T> e,
                                                 const typename Cfg::T* __restrict__ D, int F,
                                                 const SX* __restrict__ X, double lam,
                                                 SO* __restrict__ Z) {
  typedef typename Cfg::T T;
  const int N = e.N, M = e.M;
  const int nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = t / nbj, bj = t % nbj;
  LoadDenseKC<Cfg, Cfg::BM, Cfg::LDA, T, false> la;
  la.p = reinterpret_cast<const cx<T>*>(D);
  la.ld = M;
  la.o0 = bi * Cfg::BM;
  la.oend = F;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, true> lb;
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, M, acc, smem_base<Cfg>());
  cx<SO>* O = reinterpret_cast<cx<SO>*>(Z);
  const cx<SX>* Xc = reinterpret_cast<const cx<SX>*>(X);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
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

// Triangular products on frame blocks (refinement correction):
//   mode 0: Y[f][i] = sum_{n <= i} Xin[f][n] Li[i][n]          (L^-1 x, per frame)
//   mode 1: X[f][i] += sum_{n >= i} Yin[f][n] conj(Li[n][i])   (L^-H y, accumulated)
template <class Cfg, int MODE, typename SO>
__global__ __launch_bounds__(256) void k_tri_frames(const typename Cfg::T* __restrict__ Li,
                                                    const typename Cfg::T* __restrict__ In, int F,
                                                    int N, SO* __restrict__ Out) {
  typedef typename Cfg::T T;
  const int nbj = (N + Cfg::BN - 1) / Cfg::BN;
  const int t = blockIdx.x;
  const int bi = t / nbj, bj = t % nbj;
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
      if (MODE == 0) {
        O[o] = cx<SO>{SO(re), SO(im)};
      } else {
        cx<SO> x = O[o];
        O[o] = cx<SO>{SO(x.re + re), SO(x.im + im)};
      }
    }
  });
}

// Elementwise FP64 -> FP32 complex copy (n complex values).
__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
typedef TileCfg<float, 128, 128, 8> F32Cfg;
typedef TileCfg<double, 64, 64, 8> F64Cfg;

template <class Cfg> static size_t smem_bytes() { return Cfg::SMEM_ELEMS * sizeof(typename Cfg::T); }

template <typename T> struct PickCfg;
template <> struct PickCfg<float> { typedef F32Cfg type; };
template <> struct PickCfg<double> { typedef F64Cfg type; };

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T>
hipError_t launch_gram(const EncDev<T>& e, double* G, int flush, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int nb = cdiv(e.N, Cfg::BM);
  const int tiles = nb * (nb + 1) / 2;
  if (flush <= 0 || sizeof(T) == 8) flush = e.M;
  flush = ((flush + Cfg::BK - 1) / Cfg::BK) * Cfg::BK;
  hipLaunchKernelGGL(k_gram<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, G, flush);
  return hipGetLastError();
}

hipError_t launch_cholinv(double* A, double* Li, int N, double lam, int* info, hipStream_t s) {
  const int nb = 64;
  const int nblk = cdiv(N, nb);
  const size_t diag_smem = (64 * 64 + 64) * sizeof(cx<double>);
  static bool attr = false;
  if (!attr) {
    hipError_t err = hipFuncSetAttribute((const void*)k_chol_diag,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)diag_smem);
    if (err != hipSuccess) return err;
    attr = true;
  }
  for (int k = 0; k < nblk; ++k) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), diag_smem, s, A, Li, N, nb, k, lam, info);
    const int ntiles = nblk - 1;   // (nblk-k-1) panel + k inverse blocks
    if (ntiles > 0)
      hipLaunchKernelGGL(k_chol_panel, dim3(ntiles), dim3(256), smem_bytes<CholCfg>(), s, A, Li, N,
                         k, (const int*)info);
    const int rem = nblk - k - 1;
    const int tt = rem * (rem + 1) / 2 + rem * (k + 1);
    if (tt > 0)
      hipLaunchKernelGGL(k_chol_trailing, dim3(tt), dim3(256), smem_bytes<CholCfg>(), s, A, Li, N,
                         k, (const int*)info);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trmm_w(const EncDev<T>& e, const T* Li, T* W, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(e.N, Cfg::BM) * cdiv(e.M, Cfg::BN);
  hipLaunchKernelGGL(k_trmm_w<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, Li, W);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trmm_r(const T* Li, const T* W, T* R, int N, int M, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(N, Cfg::BM) * cdiv(M, Cfg::BN);
  hipLaunchKernelGGL(k_trmm_r<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, Li, W, R, N, M);
  return hipGetLastError();
}

template <typename T>
int apply_tiles(int F, int N) {
  typedef typename PickCfg<T>::type Cfg;
  return cdiv(F, Cfg::BM) * cdiv(N, Cfg::BN);
}

template <typename T>
hipError_t launch_apply(const ApplyBatch& b, int total_tiles, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  if (total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply<Cfg>, dim3(total_tiles), dim3(256), smem_bytes<Cfg>(), s, b);
  return hipGetLastError();
}

template <typename T, typename SX, typename SD>
hipError_t launch_forward(const EncDev<T>& e, const SX* X, int F, const SD* Din, T* Dout,
                          hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(e.M, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL((k_forward<Cfg, SX, SD>), dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, X,
                     F, Din, Dout);
  return hipGetLastError();
}

template <typename T, typename SX, typename SO>
hipError_t launch_adjoint(const EncDev<T>& e, const T* D, int F, const SX* X, double lam, SO* Z,
                          hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(e.N, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL((k_adjoint<Cfg, SX, SO>), dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, D,
                     F, X, lam, Z);
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

hipError_t launch_to_f32(const double* in, float* out, size_t n_complex, hipStream_t s) {
  const size_t n2 = 2 * n_complex;
  int blocks = (int)std::min<size_t>(4096, (n2 + 255) / 256);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, s, in, out, n2);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_gram<float>(const EncDev<float>&, double*, int, hipStream_t);
template hipError_t launch_gram<double>(const EncDev<double>&, double*, int, hipStream_t);
template hipError_t launch_trmm_w<float>(const EncDev<float>&, const float*, float*, hipStream_t);
template hipError_t launch_trmm_w<double>(const EncDev<double>&, const double*, double*, hipStream_t);
template hipError_t launch_trmm_r<float>(const float*, const float*, float*, int, int, hipStream_t);
template hipError_t launch_trmm_r<double>(const double*, const double*, double*, int, int, hipStream_t);
template int apply_tiles<float>(int, int);
template int apply_tiles<double>(int, int);
template hipError_t launch_apply<float>(const ApplyBatch&, int, hipStream_t);
template hipError_t launch_apply<double>(const ApplyBatch&, int, hipStream_t);
template hipError_t launch_forward<float, float, float>(const EncDev<float>&, const float*, int,
                                                        const float*, float*, hipStream_t);
template hipError_t launch_forward<double, double, double>(const EncDev<double>&, const double*, int,
                                                           const double*, double*, hipStream_t);
template hipError_t launch_forward<double, float, float>(const EncDev<double>&, const float*, int,
                                                         const float*, double*, hipStream_t);
template hipError_t launch_adjoint<double, float, float>(const EncDev<double>&, const double*, int,
                                                         const float*, double, float*, hipStream_t);
template hipError_t launch_adjoint<double, double, double>(const EncDev<double>&, const double*, int,
                                                           const double*, double, double*,
                                                           hipStream_t);
template hipError_t launch_adjoint<float, float, float>(const EncDev<float>&, const float*, int,
                                                        const float*, double, float*, hipStream_t);
template hipError_t launch_tri_frames<float, 0, float>(const float*, const float*, int, int, float*,
                                                       hipStream_t);
template hipError_t launch_tri_frames<float, 1, float>(const float*, const float*, int, int, float*,
                                                       hipStream_t);
template hipError_t launch_tri_frames<double, 0, double>(const double*, const double*, int, int,
                                                         double*, hipStream_t);
template hipError_t launch_tri_frames<double, 1, double>(const double*, const double*, int, int,
                                                         double*, hipStream_t);

}  // namespace pinv
