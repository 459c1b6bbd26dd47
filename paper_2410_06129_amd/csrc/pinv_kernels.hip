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
#include <type_traits>

#include "pinv_internal.h"

namespace pinv {

// Workgroups per CU that a kernel's register budget is sized for: three for
// FP64 3M tiles whose generated operand carries no species or off-resonance
// factor (the refinement's FP64 products then fit 168 registers and their LDS
// fits three times), two otherwise (the Gram's accumulators and the extra
// factors spill at 168).
template <class Cfg, int FEAT = 0> struct MinBlocks {
  static constexpr int value =
      (sizeof(typename Cfg::T) == 8 && IsM3<Cfg>::value && (FEAT & ~FEAT_COIL) == 0) ? 3 : 2;
};

// ---------------------------------------------------------------------------
// Gram: G[n1][n2] = sum_m conj(E[m][n1]) E[m][n2] for tiles bi >= bj.
// FP32 tiles flush their FP32 partial sums into the FP64 Gram every `flush`
// rows so the long sum over M is carried in FP64.
// ---------------------------------------------------------------------------
template <class Cfg, int FEAT, bool AL>
__global__ __launch_bounds__(256, 2) void k_gram(EncDev<typename Cfg::T> e, double* __restrict__ G,
                                              int flush) {
  typedef typename Cfg::T T;
  static_assert(Cfg::BM == Cfg::BN, "square tiles");
  int bi, bj;
  tri_index(blockIdx.x, &bi, &bj);
  const int N = e.N;
  LoadGenCol<Cfg, Cfg::BM, Cfg::LDA, true, FEAT, AL> la;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, false, FEAT, AL> lb;
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
// Fewer samples than unknowns (Sec. 2.2, right pseudoinverse): the samples'
// Gram G'[m][m'] = sum_n E[m][n] conj(E[m'][n]) over the N unknowns, lower
// triangle of M x M tiles, E generated row-wise on both sides, FP64.
// ---------------------------------------------------------------------------
template <class Cfg, int FEAT, bool AL>
__global__ __launch_bounds__(256, 2) void k_gram_rows(EncDev<typename Cfg::T> e,
                                                   double* __restrict__ G) {
  typedef typename Cfg::T T;
  static_assert(Cfg::BM == Cfg::BN, "square tiles");
  int bi, bj;
  tri_index(blockIdx.x, &bi, &bj);
  const int M = e.M;
  LoadGenRow<Cfg, Cfg::BM, Cfg::LDA, false, FEAT, AL> la;
  LoadGenRow<Cfg, Cfg::BN, Cfg::LDB, true, FEAT, AL> lb;
  la.init(e, bi * Cfg::BM);
  lb.init(e, bj * Cfg::BN);
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, e.N, acc, smem_base<Cfg>());
  cx<double>* Gc = reinterpret_cast<cx<double>*>(G);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < M && col < M) Gc[(size_t)row * M + col] = cx<double>{(double)re, (double)im};
  });
}

// ---------------------------------------------------------------------------
// Gram through the shared trajectory (Eq. 11): every coil's rows are the
// coil-free encoding F (Fourier, species and off-resonance factors) scaled by
// the coil map, E_c = F diag(C_c), so
//     G[a][b] = sum_c conj(C_c(v_a)) C_c(v_b) (F^H F)[a][b].
// F^H F is accumulated over the K rows of one coil on MFMA (F generated per
// tile), the coil cross-product is formed in the epilogue from coil columns
// staged in LDS.  `e` must describe F (no coil table, C = 1, M = K); `coil`
// is the [C][V] coil table (or null for one unit coil).
// ---------------------------------------------------------------------------
template <class Cfg, int FEAT, bool AL>
__global__ __launch_bounds__(256, 2) void k_gram_shared(EncDev<typename Cfg::T> e,
                                                     const typename Cfg::T* __restrict__ coil,
                                                     int C, double* __restrict__ G) {
  typedef typename Cfg::T T;
  static_assert(Cfg::BM == Cfg::BN, "square tiles");
  int bi, bj;
  tri_index(blockIdx.x, &bi, &bj);
  const int N = e.N, V = e.V;
  LoadGenCol<Cfg, Cfg::BM, Cfg::LDA, true, FEAT, AL> la;
  LoadGenCol<Cfg, Cfg::BN, Cfg::LDB, false, FEAT, AL> lb;
  la.init(e, bi * Cfg::BM);
  lb.init(e, bj * Cfg::BN);
  T* smem = smem_base<Cfg>();
  AccTile<Cfg> acc;
  acc.zero();
  mainloop<Cfg>(la, lb, 0, e.M, acc, smem);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  cx<double>* Gc = reinterpret_cast<cx<double>*>(G);
  if (!coil) {
    acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
      const int row = r0 + r, col = c0 + c;
      if (row < N && col < N) Gc[(size_t)row * N + col] = cx<double>{(double)re, (double)im};
    });
    return;
  }
  // coil cross-products: stage the coil values of the tile's rows and columns,
  // CC coils at a time, and accumulate F^H F * sum_c conj(C_c(v_a)) C_c(v_b)
  // into G (written by the first chunk, updated by later ones)
  constexpr int CC = (Cfg::SMEM_ELEMS * sizeof(T)) / (sizeof(cx<T>) * (Cfg::BM + Cfg::BN));
  static_assert(CC >= 1, "no room for coil staging");
  cx<T>* sa = reinterpret_cast<cx<T>*>(smem);          // [CC][BM]
  cx<T>* sb = sa + CC * Cfg::BM;                       // [CC][BN]
  const cx<T>* cc = reinterpret_cast<const cx<T>*>(coil);
  for (int c0c = 0; c0c < C; c0c += CC) {
    const int nc = min(CC, C - c0c);
    for (int idx = threadIdx.x; idx < nc * (Cfg::BM + Cfg::BN); idx += Cfg::NT) {
      const int c = idx / (Cfg::BM + Cfg::BN), o = idx - c * (Cfg::BM + Cfg::BN);
      const int g = o < Cfg::BM ? r0 + o : c0 + (o - Cfg::BM);
      cx<T> v{T(0), T(0)};
      if (g < N) v = cc[(size_t)(c0c + c) * V + (g % V)];
      if (o < Cfg::BM) sa[c * Cfg::BM + o] = v; else sb[c * Cfg::BN + (o - Cfg::BM)] = v;
    }
    __syncthreads();
    acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
      const int row = r0 + r, col = c0 + c;
      double sr = 0.0, si = 0.0;
      for (int q = 0; q < nc; ++q) {
        const cx<T> x = sa[q * Cfg::BM + r], y = sb[q * Cfg::BN + c];
        sr += (double)x.re * (double)y.re + (double)x.im * (double)y.im;   // conj(x) * y
        si += (double)x.re * (double)y.im - (double)x.im * (double)y.re;
      }
      if (row < N && col < N) {
        const double fr = (double)re, fi = (double)im;
        cx<double> v{fr * sr - fi * si, fr * si + fi * sr};
        cx<double>* g = Gc + (size_t)row * N + col;
        if (c0c > 0) {
          const cx<double> o = *g;
          v.re += o.re;
          v.im += o.im;
        }
        *g = v;
      }
    });
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Cholesky diagonal block (FP64, one workgroup).  Hermitian elimination of the
// augmented block [A_kk + lam I | I] without pivoting: at column j every row
// i > j subtracts A_ij / A_jj times row j, on the lower triangle of A and on
// B = Lt^-1 (unit lower), where A = Lt D Lt^H.  Row j of A is read as the
// conjugate of column j, so the updated matrix stays exactly Hermitian with a
// real diagonal; updating a full, unsymmetric copy lets the two triangles
// drift apart and fails on ill-conditioned blocks.  The pivots are D, and
// L^-1 = D^-1/2 Lt^-1 = D^-1/2 B.
//
// Storage: one complex per (row, column) in registers.  Column c of row i
// holds A_ic while c is still to be eliminated and B_ic once it has been
// (A_ic is dead from then on, and B_ic is zero before); B_ii = 1 is implicit.
// Lane c of every wave owns column c, wave w owns rows w, w + NW, ... (four
// rows per thread at NW = 16, so the waves of a SIMD hide each other's LDS
// and barrier latency).  With the pivot folded into a per-lane factor rp_c
// (row j of B, of 1, or of A, divided by A_jj) each entry costs one complex
// multiply-add.  Column j+1 and
// row j+1 are published for the next step as soon as they are final, into the
// other half of a double-buffered LDS pair: one barrier per column.  Only
// L_kk^-1 is stored: the panel, trailing and inverse updates need no L_kk.
// ---------------------------------------------------------------------------
constexpr int kDiagSmem = 0;
constexpr int kDiagWaves = 16;   // measured: 16 waves 7.5 ms per 4096 factorisation, 8: 7.7, 4: 8.7

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_chol_diag(double* __restrict__ A,
                                                       double* __restrict__ Li, int N, int nb,
                                                       int k, double lam,
                                                       int* __restrict__ info) {
  if (*info) return;
  constexpr int RPT = 64 / NW;
  __shared__ cx<double> colA[2][64];
  __shared__ cx<double> rowZ[2][64];
  __shared__ double dpiv[64];
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = tid & 63;
  const int k0 = k * nb;
  const int nbk = min(nb, N - k0);
  const cx<double>* Ac = reinterpret_cast<const cx<double>*>(A);
  cx<double>* Lc = reinterpret_cast<cx<double>*>(Li);
  cx<double> z[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = w + NW * q;
    cx<double> v{0.0, 0.0};
    if (i < nbk && c <= i) v = Ac[(size_t)(k0 + i) * N + k0 + c];
    if (i == c) v = cx<double>{v.re + lam, 0.0};
    z[q] = v;
  }
  if (c == 0) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) colA[0][w + NW * q] = z[q];
  }
  __syncthreads();
  bool failed = false;
  for (int j = 0; j < nbk; ++j) {
    const int p = j & 1;
    const double piv = colA[p][j].re;   // the same value for every thread
    if (!(piv > 0.0)) {                 // also catches NaN
      if (tid == 0) atomicCAS(info, 0, k0 + j + 1);
      failed = true;
      break;
    }
    const double inv = 1.0 / piv;
    if (tid == 0) dpiv[j] = piv;
    cx<double> rp;
    if (c < j) {
      const cx<double> t = rowZ[p][c];
      rp = cx<double>{t.re * inv, t.im * inv};
    } else if (c == j) {
      rp = cx<double>{inv, 0.0};
    } else {
      const cx<double> t = colA[p][c];   // row j of A = conj(column j)
      rp = cx<double>{t.re * inv, -t.im * inv};
    }
    const bool cj = (c == j);
    cx<double> col[RPT];   // all loads in flight before the first use
#pragma unroll
    for (int q = 0; q < RPT; ++q) col[q] = colA[p][w + NW * q];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int i = w + NW * q;
      if (i > j) {   // uniform over the wave
        const cx<double> a = col[q];
        cx<double> o = cj ? cx<double>{0.0, 0.0} : z[q];
        o.re -= a.re * rp.re - a.im * rp.im;
        o.im -= a.re * rp.im + a.im * rp.re;
        z[q] = o;
        if (c == j + 1) colA[p ^ 1][i] = o;
        if (i == j + 1) rowZ[p ^ 1][c] = o;
      }
    }
    __syncthreads();
  }
  if (failed) return;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = w + NW * q;
    if (i < nbk && c < nbk) {
      const double sc = 1.0 / sqrt(dpiv[i]);
      cx<double> v{0.0, 0.0};
      if (c < i) v = cx<double>{z[q].re * sc, z[q].im * sc};
      else if (c == i) v = cx<double>{sc, 0.0};
      Lc[(size_t)(k0 + i) * N + k0 + c] = v;
    }
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
    mainloop<Cfg, false>(la, lb, 0, kend, acc, smem);
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
    mainloop<Cfg, false>(la, lb, 0, kend, acc, smem);
  }
  __syncthreads();
  cx<double>* O = reinterpret_cast<cx<double>*>(out);
  acc_foreach<Cfg>(acc, [&](int r, int c, double re, double im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < N) O[(size_t)row * N + col] = cx<double>{re, im};
  });
}

// Step k trailing update: A_ij -= L_ik L_jk^H for k < j <= i ("herk" tiles)
// and B_ij -= L_ik Y_kj for i > k, j <= k (inverse tiles).  `part` selects
// the tiles of one launch:
//   0  all of them;
//   1  the look-ahead set: block column k+1 of A and block row k+1 of B, all
//      that step k+1's diagonal block and panel read;
//   2  the rest (A columns >= k+2, B rows >= k+2), which can run beside
//      step k+1's diagonal and panel kernels.
// The accumulators start from -(old tile), loaded together with the first
// operand chunk, and the tile is stored negated: no read after the products.
__global__ __launch_bounds__(256) void k_chol_trailing(double* __restrict__ A, double* __restrict__ Li,
                                                       int N, int k, const int* __restrict__ info,
                                                       int part) {
  if (*info) return;
  typedef CholCfg Cfg;
  const int nb = 64;
  const int nblk = (N + nb - 1) / nb;
  const int rem = nblk - k - 1;
  const int t = blockIdx.x;
  const cx<double>* Ac = reinterpret_cast<const cx<double>*>(A);
  const cx<double>* Lc = reinterpret_cast<const cx<double>*>(Li);
  double* smem = smem_base<Cfg>();
  const int kw = min(N, (k + 1) * nb) - k * nb;
  bool herk;
  int r0, c0;
  if (part == 1) {
    herk = t < rem;
    r0 = herk ? (k + 1 + t) * nb : (k + 1) * nb;
    c0 = herk ? (k + 1) * nb : (t - rem) * nb;
  } else {
    const int first = part == 2 ? k + 2 : k + 1;   // first trailing block row/column
    const int r = nblk - first;
    const int nherk = r * (r + 1) / 2;
    herk = t < nherk;
    if (herk) {
      int ti, tj;
      tri_index(t, &ti, &tj);
      r0 = (first + ti) * nb;
      c0 = (first + tj) * nb;
    } else {
      const int u = t - nherk;
      r0 = (first + u / (k + 1)) * nb;
      c0 = (u % (k + 1)) * nb;
    }
  }
  cx<double>* O = reinterpret_cast<cx<double>*>(herk ? A : Li);
  AccTile<Cfg> acc;
  acc_foreach_mut<Cfg>(acc, [&](int r, int c, double& re, double& im) {
    const int row = r0 + r, col = c0 + c;
    cx<double> o{0.0, 0.0};
    if (row < N && col < N) o = O[(size_t)row * N + col];
    re = -o.re;
    im = -o.im;
  });
  LoadDenseKC<Cfg, 64, Cfg::LDA, double, false> la;      // L_ik[m][l] at A[(i*nb+m)*N + k*nb + l]
  la.p = Ac + k * nb;
  la.ld = N;
  la.o0 = r0;
  la.oend = N;
  if (herk) {
    LoadDenseKC<Cfg, 64, Cfg::LDB, double, true> lb;     // conj(L_jk[n][l])
    lb.p = Ac + k * nb;
    lb.ld = N;
    lb.o0 = c0;
    lb.oend = N;
    mainloop<Cfg, false>(la, lb, 0, kw, acc, smem);
  } else {
    LoadDenseOC<Cfg, 64, Cfg::LDB, double, false> lb;    // Y_kj[l][n] at Li[(k*nb+l)*N + j*nb + n]
    lb.p = Lc + (size_t)(k * nb) * N;
    lb.ld = N;
    lb.o0 = c0;
    lb.oend = min(N, c0 + nb);
    mainloop<Cfg, false>(la, lb, 0, kw, acc, smem);
  }
  acc_foreach<Cfg>(acc, [&](int r, int c, double re, double im) {
    const int row = r0 + r, col = c0 + c;
    if (row < N && col < N) O[(size_t)row * N + col] = cx<double>{-re, -im};
  });
}

// ---------------------------------------------------------------------------
// W = L^-1 E^H : W[i][m] = sum_{n <= i} Li[i][n] conj(E[m][n])
// ---------------------------------------------------------------------------
template <class Cfg, int FEAT, bool AL>
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
  LoadGenRow<Cfg, Cfg::BN, Cfg::LDB, true, FEAT, AL> lb;
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
template <typename T>
__global__ __launch_bounds__(256) void k_conj_transpose(const T* __restrict__ Z, T* __restrict__ R,
                                                        int M, int N) {
  __shared__ cx<T> tile[32][33];
  const int n0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  const cx<T>* z = reinterpret_cast<const cx<T>*>(Z);
  cx<T>* r = reinterpret_cast<cx<T>*>(R);
  for (int j = ty; j < 32; j += 8) {
    const int m = m0 + j, n = n0 + tx;
    if (m < M && n < N) tile[j][tx] = z[(size_t)m * N + n];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int n = n0 + j, m = m0 + tx;
    if (m < M && n < N) {
      const cx<T> v = tile[tx][j];
      r[(size_t)n * M + m] = cx<T>{v.re, -v.im};
    }
  }
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
// An item whose tile grid alone would leave the GPU partly idle is split over
// M (the split depends only on the item's F, N and M, so a result is the same
// alone and in any group); its splits write partial tiles to item.work and
// k_apply_reduce adds them in split order.
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
  const int u0 = t - it.tile0;
  const int split = u0 / it.ntile;
  const int u = u0 - split * it.ntile;
  const int nbj = (it.N + Cfg::BN - 1) / Cfg::BN;
  const int bi = u / nbj, bj = u % nbj;
  const int k0 = split * it.kchunk, k1 = min(it.M, k0 + it.kchunk);
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
  mainloop<Cfg>(la, lb, k0, k1, acc, smem_base<Cfg>());
  cx<T>* O = it.splits > 1
                 ? reinterpret_cast<cx<T>*>(it.work) + (size_t)split * it.F * it.N
                 : reinterpret_cast<cx<T>*>(it.X);
  const int r0 = bi * Cfg::BM, c0 = bj * Cfg::BN;
  acc_foreach<Cfg>(acc, [&](int r, int c, T re, T im) {
    const int row = r0 + r, col = c0 + c;
    if (row < it.F && col < it.N) O[(size_t)row * it.N + col] = cx<T>{re, im};
  });
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
    T zr = W[i].re, zi = W[i].im;
    for (int s = 1; s < it.splits; ++s) {
      zr += W[(int64_t)s * n + i].re;
      zi += W[(int64_t)s * n + i].im;
    }
    X[i] = cx<T>{zr, zi};
  }
}

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
// streaming RW rows of R.  At small F each element of R feeds only F
// multiply-adds, so the apply is bound by memory bandwidth, not by MFMA: rows
// stream through wide coalesced loads (two complex64 per lane and load when
// VEC = 2), and each data element loaded serves RW rows, which keeps the
// data's cache traffic (F / RW times that of R) below R's own.  Every wave
// reduces its lane partial sums in a fixed butterfly order, so a result
// depends only on its own row and frame.
template <typename T, int FM, int RW, int VEC>
__global__ __launch_bounds__(256) void k_apply_rows(const T* __restrict__ R, const T* __restrict__ D,
                                                    T* __restrict__ X, int N, int M, int F) {
  const int lane = threadIdx.x & 63;
  const int n0 = (blockIdx.x * 4 + (int)(threadIdx.x >> 6)) * RW;
  if (n0 >= N) return;   // the whole wavefront leaves; no barrier follows
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
  for (int m0 = lane * VEC; m0 < M; m0 += 64 * VEC) {
    cx<T> rv[RW][VEC];
#pragma unroll
    for (int j = 0; j < RW; ++j) {
      if constexpr (VEC == 2) {
        // M even and 16-byte aligned rows (checked by the launcher): m0 + 1 < M
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
    cx<T>* x = reinterpret_cast<cx<T>*>(X);
#pragma unroll
    for (int j = 0; j < RW; ++j)
#pragma unroll
      for (int f = 0; f < FM; ++f)
        if (f < F && n0 + j < N) x[(size_t)f * N + n0 + j] = cx<T>{ar[j][f], ai[j][f]};
  }
}

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

// Fill the strict upper triangle of an N x N complex matrix from its lower part.
__global__ void k_herm_fill(double* __restrict__ G, int N) {
  cx<double>* g = reinterpret_cast<cx<double>*>(G);
  const int col = blockIdx.x * 16 + (threadIdx.x & 15);
  const int row = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (row < N && col < N && row < col) {
    const cx<double> v = g[(size_t)col * N + row];
    g[(size_t)row * N + col] = cx<double>{v.re, -v.im};
  }
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

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_gram(const EncDev<T>& e, double* G, int flush, hipStream_t s) {
  typedef typename GramCfgOf<T>::type Cfg;
  const int nb = cdiv(e.N, Cfg::BM);
  const int tiles = nb * (nb + 1) / 2;
  if (flush <= 0 || sizeof(T) == 8) flush = e.M;
  flush = ((flush + Cfg::BK - 1) / Cfg::BK) * Cfg::BK;
  return with_feat_al(enc_features(e), e.K % Cfg::BK == 0, [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_gram<Cfg, decltype(fc)::value, decltype(al)::value>), dim3(tiles),
                       dim3(256), smem_bytes<Cfg>(), s, e, G, flush);
    return hipGetLastError();
  });
}

hipError_t launch_gram_rows(const EncDev<double>& e, double* G, hipStream_t s) {
  typedef GramCfgOf<double>::type Cfg;
  const int nb = cdiv(e.M, Cfg::BM);
  const int tiles = nb * (nb + 1) / 2;
  return with_feat_al(enc_features(e), e.nx % Cfg::BK == 0, [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_gram_rows<Cfg, decltype(fc)::value, decltype(al)::value>), dim3(tiles),
                       dim3(256), smem_bytes<Cfg>(), s, e, G);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_right_pinv(const EncDev<T>& e, const T* Li, T* W, T* Z, T* R, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(e.M, Cfg::BM) * cdiv(e.N, Cfg::BN);
  hipError_t err = with_feat_al(enc_features(e), e.K % Cfg::BK == 0, [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_trmm_w_rows<Cfg, decltype(fc)::value, decltype(al)::value>), dim3(tiles),
                       dim3(256), smem_bytes<Cfg>(), s, e, Li, W);
    return hipGetLastError();
  });
  if (err != hipSuccess) return err;
  err = launch_trmm_r<T>(Li, W, Z, e.M, e.N, s);   // Z = L'^-H W' (M x N)
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_conj_transpose<T>, dim3(cdiv(e.N, 32), cdiv(e.M, 32)), dim3(256), 0, s, Z, R,
                     e.M, e.N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gram_shared(const EncDev<T>& e, double* G, hipStream_t s) {
  typedef typename GramCfgOf<T>::type Cfg;
  EncDev<T> f = e;       // the coil-free encoding F over one coil's K rows
  f.coil = nullptr;
  f.C = 1;
  f.M = e.K;
  const int nb = cdiv(e.N, Cfg::BM);
  const int tiles = nb * (nb + 1) / 2;
  return with_feat_al(enc_features(f) & 3, f.K % Cfg::BK == 0, [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_gram_shared<Cfg, decltype(fc)::value & 3, decltype(al)::value>),
                       dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, f, e.coil, e.coil ? e.C : 1, G);
    return hipGetLastError();
  });
}

// With an auxiliary stream `aux` the factorisation looks ahead one step: on
// s, step k's look-ahead tiles (part 1) then step k+1's diagonal block and
// panel; on aux, step k's remaining tiles (part 2) beside them.  Events order
// part 2 of step k after step k's panel, and step k+1's part 1 after step k's
// part 2 (which updated the blocks it reads and writes).  Without aux, one
// launch per step does all trailing tiles on s.
hipError_t launch_cholinv(double* A, double* Li, int N, double lam, int* info, hipStream_t s,
                          hipStream_t aux) {
  const int nb = 64;
  const int nblk = cdiv(N, nb);
  const size_t diag_smem = kDiagSmem;
  const size_t sm = smem_bytes<CholCfg>();
  hipEvent_t ev_panel = nullptr, ev_rest = nullptr;
  if (aux) {
    hipError_t err = hipEventCreateWithFlags(&ev_panel, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&ev_rest, hipEventDisableTiming);
    if (err != hipSuccess) {
      if (ev_panel) (void)hipEventDestroy(ev_panel);
      return err;
    }
  }
  hipError_t err = hipSuccess;
  bool rest_pending = false;
  for (int k = 0; k < nblk && err == hipSuccess; ++k) {
    hipLaunchKernelGGL(k_chol_diag<kDiagWaves>, dim3(1), dim3(64 * kDiagWaves), diag_smem, s, A, Li,
                       N, nb, k, lam, info);
    const int ntiles = nblk - 1;   // (nblk-k-1) panel + k inverse blocks
    if (ntiles > 0)
      hipLaunchKernelGGL(k_chol_panel, dim3(ntiles), dim3(256), sm, s, A, Li, N, k, (const int*)info);
    const int rem = nblk - k - 1;
    if (rem <= 0) break;
    if (!aux) {
      hipLaunchKernelGGL(k_chol_trailing, dim3(rem * (rem + 1) / 2 + rem * (k + 1)), dim3(256), sm, s,
                         A, Li, N, k, (const int*)info, 0);
      err = hipGetLastError();
      continue;
    }
    // part 2 of step k (aux) after step k's panel and after part 2 of step k-1
    if ((err = hipEventRecord(ev_panel, s)) != hipSuccess) break;
    if ((err = hipStreamWaitEvent(aux, ev_panel, 0)) != hipSuccess) break;
    // part 1 of step k (s) after part 2 of step k-1
    if (rest_pending && (err = hipStreamWaitEvent(s, ev_rest, 0)) != hipSuccess) break;
    hipLaunchKernelGGL(k_chol_trailing, dim3(rem + (k + 1)), dim3(256), sm, s, A, Li, N, k,
                       (const int*)info, 1);
    const int r2 = rem - 1;
    if (r2 > 0) {
      hipLaunchKernelGGL(k_chol_trailing, dim3(r2 * (r2 + 1) / 2 + r2 * (k + 1)), dim3(256), sm, aux,
                         A, Li, N, k, (const int*)info, 2);
      if ((err = hipEventRecord(ev_rest, aux)) != hipSuccess) break;
      rest_pending = true;
    } else {
      rest_pending = false;
    }
    err = hipGetLastError();
  }
  if (aux) {
    // everything after the factorisation on s sees the last part-2 updates
    if (err == hipSuccess && rest_pending) err = hipStreamWaitEvent(s, ev_rest, 0);
    (void)hipEventDestroy(ev_panel);
    (void)hipEventDestroy(ev_rest);
  }
  if (err != hipSuccess) return err;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_trmm_w(const EncDev<T>& e, const T* Li, T* W, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(e.N, Cfg::BM) * cdiv(e.M, Cfg::BN);
  return with_feat_al(enc_features(e), e.nx % Cfg::BK == 0, [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_trmm_w<Cfg, decltype(fc)::value, decltype(al)::value>), dim3(tiles),
                       dim3(256), smem_bytes<Cfg>(), s, e, Li, W);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_trmm_r(const T* Li, const T* W, T* R, int N, int M, hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(N, Cfg::BM) * cdiv(M, Cfg::BN);
  hipLaunchKernelGGL(k_trmm_r<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, Li, W, R, N, M);
  return hipGetLastError();
}

// The apply uses the same 128x64 3M tiles as the triangular products: with
// the raised wave priority over the matrix products, their occupancy of two
// workgroups per CU beats 128x128 at one (7.76 against 8.04 ms at 1000
// frames, N = 4096, M = 32768; without the priority raise 128x128 had been
// ahead, 8.1 against 8.3 ms).
template <typename T> struct ApplyCfgOf;
template <> struct ApplyCfgOf<float> { typedef F32Cfg type; };
template <> struct ApplyCfgOf<double> { typedef F64Cfg type; };
// FP32 applies of at most 32 frames run on 32x128 tiles: a 128-frame tile
// would spend most of its matrix products on padding rows.
typedef TileCfg<float, 32, 128, 8, true> F32FewFramesCfg;
constexpr int kFewFramesMaxF = 32;
// A grouped apply of few frames has few tiles, so its contraction may be split
// up to 16 ways (the other split launches stop at 4).
constexpr int kApplyMaxSplit = 16;

template <typename T>
int apply_tiles(int F, int N) {
  typedef typename ApplyCfgOf<T>::type Cfg;
  return cdiv(F, Cfg::BM) * cdiv(N, Cfg::BN);
}

// Grouped apply with per-item contraction splits: sets each item's split,
// tile range and partial-sum workspace, runs the tiles, then the reduction.
template <class Cfg>
static hipError_t run_apply(ApplyBatch b, hipStream_t s) {
  typedef typename Cfg::T T;
  const int slots = resident_blocks(k_apply<Cfg>, 256, smem_bytes<Cfg>());
  int tiles = 0, nsplit = 0;
  size_t work_elems = 0;
  for (int i = 0; i < b.n; ++i) {
    ApplyItemDev& it = b.it[i];
    const int nchunks = cdiv(it.M, Cfg::BK);
    it.ntile = cdiv(it.F, Cfg::BM) * cdiv(it.N, Cfg::BN);
    it.splits = pick_split(it.ntile, slots, nchunks, kApplyMaxSplit);
    it.kchunk = cdiv(nchunks, it.splits) * Cfg::BK;
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
    hipError_t err = hipMallocAsync(&work, work_elems * 2 * sizeof(T), s);
    if (err != hipSuccess) return err;
    size_t off = 0;
    for (int i = 0; i < b.n; ++i)
      if (b.it[i].splits > 1) {
        b.it[i].work = (cx<T>*)work + off;
        off += (size_t)b.it[i].splits * b.it[i].F * b.it[i].N;
      }
  }
  hipLaunchKernelGGL(k_apply<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, b);
  hipError_t err = hipGetLastError();
  if (nsplit) {
    if (err == hipSuccess) {
      hipLaunchKernelGGL(k_apply_reduce<T>, dim3(1024, b.n), dim3(256), 0, s, b);
      err = hipGetLastError();
    }
    const hipError_t ferr = hipFreeAsync(work, s);
    if (err == hipSuccess) err = ferr;
  }
  return err;
}

template <typename T>
hipError_t launch_apply(const ApplyBatch& b, int, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    // items go to the tile shape their own frame count selects, so an item's
    // result does not depend on the other items of the group
    ApplyBatch few, many;
    few.n = many.n = 0;
    for (int i = 0; i < b.n; ++i) {
      if (b.it[i].F <= kFewFramesMaxF)
        few.it[few.n++] = b.it[i];
      else
        many.it[many.n++] = b.it[i];
    }
    if (few.n) {
      const hipError_t err = run_apply<F32FewFramesCfg>(few, s);
      if (err != hipSuccess) return err;
    }
    return many.n ? run_apply<F32Cfg>(many, s) : hipSuccess;
  } else {
    return run_apply<typename ApplyCfgOf<T>::type>(b, s);
  }
}

template <typename T, typename SX, typename SD>
hipError_t launch_forward(const EncDev<T>& e, const SX* X, int F, const SD* Din, T* Dout,
                          hipStream_t s) {
  typedef typename PickCfg<T>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(e.M, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  return with_feat_al(enc_features(e), e.nx % Cfg::BK == 0, [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_forward<Cfg, decltype(fc)::value, SX, SD, decltype(al)::value>),
                       dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, X, F, Din, Dout);
    return hipGetLastError();
  });
}

template <typename T, typename SD, typename SX, typename SO>
hipError_t launch_adjoint(const EncDev<T>& e, const SD* D, int F, const SX* X, double lam, SO* Z,
                          hipStream_t s) {
  typedef typename std::conditional<std::is_same<T, double>::value, F64Cfg3, F32Cfg>::type Cfg;
  const int tiles = cdiv(F, Cfg::BM) * cdiv(e.N, Cfg::BN);
  if (tiles == 0) return hipSuccess;
  return with_feat_al(enc_features(e), e.K % Cfg::BK == 0, [&](auto fc, auto al) {
    auto kern = k_adjoint<Cfg, decltype(fc)::value, SD, SX, SO, decltype(al)::value>;
    // split the M contraction when one pass of the tile grid would leave the
    // GPU partly idle (the grid's last round is what the split fills)
    const int nchunks = cdiv(e.M, Cfg::BK);
    const int splits = pick_split(tiles, resident_blocks(kern, 256, smem_bytes<Cfg>()), nchunks);
    if (splits == 1) {
      hipLaunchKernelGGL(kern, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, D, F, X, lam, Z,
                         tiles, nchunks * Cfg::BK, (T*)nullptr);
      return hipGetLastError();
    }
    const int kchunk = cdiv(nchunks, splits) * Cfg::BK;
    const int64_t n = (int64_t)F * e.N;
    void* work = nullptr;
    hipError_t err = hipMallocAsync(&work, (size_t)splits * n * 2 * sizeof(T), s);
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
    const hipError_t ferr = hipFreeAsync(work, s);
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

hipError_t launch_herm_fill(double* G, int N, hipStream_t s) {
  dim3 grid(cdiv(N, 16), cdiv(N, 16));
  hipLaunchKernelGGL(k_herm_fill, grid, dim3(256), 0, s, G, N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_rows(const T* R, const T* D, T* X, int N, int M, int F, hipStream_t s) {
  if (F <= 0 || N <= 0) return hipSuccess;
  if (F > kRowApplyMaxF) return hipErrorInvalidValue;
  const bool vec = M % 2 == 0 && ((uintptr_t)R % 16) == 0 && ((uintptr_t)D % 16) == 0;
  auto go = [&](auto fm, auto rw) {
    constexpr int FM = decltype(fm)::value, RW = decltype(rw)::value;
    const dim3 grid(cdiv(N, 4 * RW)), block(256);
    if constexpr (sizeof(T) == 4) {
      if (vec) {
        hipLaunchKernelGGL((k_apply_rows<T, FM, RW, 2>), grid, block, 0, s, R, D, X, N, M, F);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_apply_rows<T, FM, RW, 1>), grid, block, 0, s, R, D, X, N, M, F);
    return hipGetLastError();
  };
  // rows per wave: as many as keep the accumulators (2 FM RW values) within
  // 64 registers
  using std::integral_constant;
  constexpr int W = sizeof(T) == 4 ? 4 : 2;
  if (F <= 1) return go(integral_constant<int, 1>(), integral_constant<int, 1>());
  if (F <= 2) return go(integral_constant<int, 2>(), integral_constant<int, W>());
  if (F <= 4) return go(integral_constant<int, 4>(), integral_constant<int, W>());
  return go(integral_constant<int, 8>(), integral_constant<int, W / 2 * 2 == 4 ? 4 : 2>());
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

// BF16x3 variants of the FP32-typed products (same kernels, split-precision mainloop)
hipError_t launch_trmm_w_b3(const EncDev<float>& e, const float* Li, float* W, hipStream_t s) {
  typedef B3Cfg Cfg;
  const int tiles = cdiv(e.N, Cfg::BM) * cdiv(e.M, Cfg::BN);
  return with_feat_al(enc_features(e), e.nx % Cfg::BK == 0, [&](auto fc, auto al) {
    auto kern = k_trmm_w<Cfg, decltype(fc)::value, decltype(al)::value>;
    // once per kernel (thread-safe static initialisation)
    static const hipError_t attr = allow_smem(kern, smem_bytes<Cfg>());
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, e, Li, W);
    return hipGetLastError();
  });
}

hipError_t launch_trmm_r_b3(const float* Li, const float* W, float* R, int N, int M, hipStream_t s) {
  typedef B3Cfg Cfg;
  static const hipError_t attr = allow_smem(k_trmm_r<Cfg>, smem_bytes<Cfg>());
  if (attr != hipSuccess) return attr;
  const int tiles = cdiv(N, Cfg::BM) * cdiv(M, Cfg::BN);
  hipLaunchKernelGGL(k_trmm_r<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), s, Li, W, R, N, M);
  return hipGetLastError();
}

int apply_tiles_b3(int F, int N) { return cdiv(F, B3Cfg::BM) * cdiv(N, B3Cfg::BN); }

hipError_t launch_apply_b3(const ApplyBatch& b, int, hipStream_t s) {
  typedef B3Cfg Cfg;
  static const hipError_t attr = allow_smem(k_apply<Cfg>, smem_bytes<Cfg>());
  if (attr != hipSuccess) return attr;
  return run_apply<Cfg>(b, s);
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
template hipError_t launch_gram<float>(const EncDev<float>&, double*, int, hipStream_t);
template hipError_t launch_gram<double>(const EncDev<double>&, double*, int, hipStream_t);
template hipError_t launch_gram_shared<float>(const EncDev<float>&, double*, hipStream_t);
template hipError_t launch_right_pinv<float>(const EncDev<float>&, const float*, float*, float*,
                                             float*, hipStream_t);
template hipError_t launch_right_pinv<double>(const EncDev<double>&, const double*, double*, double*,
                                              double*, hipStream_t);
template hipError_t launch_gram_shared<double>(const EncDev<double>&, double*, hipStream_t);
template hipError_t launch_trmm_w<float>(const EncDev<float>&, const float*, float*, hipStream_t);
template hipError_t launch_trmm_w<double>(const EncDev<double>&, const double*, double*, hipStream_t);
template hipError_t launch_trmm_r<float>(const float*, const float*, float*, int, int, hipStream_t);
template hipError_t launch_trmm_r<double>(const double*, const double*, double*, int, int, hipStream_t);
template int apply_tiles<float>(int, int);
template int apply_tiles<double>(int, int);
template hipError_t launch_apply<float>(const ApplyBatch&, int, hipStream_t);
template hipError_t launch_apply_rows<float>(const float*, const float*, float*, int, int, int,
                                             hipStream_t);
template hipError_t launch_apply_rows<double>(const double*, const double*, double*, int, int, int,
                                              hipStream_t);
template hipError_t launch_apply<double>(const ApplyBatch&, int, hipStream_t);
template hipError_t launch_forward<float, float, float>(const EncDev<float>&, const float*, int,
                                                        const float*, float*, hipStream_t);
template hipError_t launch_forward<double, double, double>(const EncDev<double>&, const double*, int,
                                                           const double*, double*, hipStream_t);
template hipError_t launch_forward<double, float, float>(const EncDev<double>&, const float*, int,
                                                         const float*, double*, hipStream_t);
template hipError_t launch_adjoint<double, double, float, float>(const EncDev<double>&, const double*,
                                                                int, const float*, double, float*,
                                                                hipStream_t);
template hipError_t launch_adjoint<double, double, double, double>(const EncDev<double>&,
                                                                   const double*, int,
                                                                   const double*, double, double*,
                                                                   hipStream_t);
template hipError_t launch_adjoint<double, float, float, double>(const EncDev<double>&, const float*,
                                                                 int, const float*, double,
                                                                 double*, hipStream_t);
template hipError_t launch_adjoint<double, float, float, float>(const EncDev<double>&, const float*,
                                                                int, const float*, double, float*,
                                                                hipStream_t);
template hipError_t launch_adjoint<float, float, float, float>(const EncDev<float>&, const float*, int,
                                                               const float*, double, float*,
                                                               hipStream_t);
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

}  // namespace pinv
