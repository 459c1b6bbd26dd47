// Blocked right-looking Cholesky of G + lam I in FP64 with L^-1 formed
// alongside (Eq. 6, Eq. 8; Sec. 2.3).
#include <type_traits>

#include "pinv_internal.h"

namespace pinv {

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

// Trailing update after steps kb .. k = kb + kn - 1 (kn = 1, or 2 for the
// two-level factorisation): A_ij -= sum_{l=kb..k} L_il L_jl^H for k < j <= i
// ("herk" tiles) and B_ij -= sum_{l=kb..k} L_il Y_lj for i > k, j <= k
// (inverse tiles), one contraction over the kn 64-column panels, which lie
// side by side in A's columns and in Li's rows (Y_lj for j > l is zero: Li
// starts zeroed and only its lower blocks are written).  `part` selects the
// tiles of one launch:
//   0  all of them;
//   1  the look-ahead set: block column k+1 of A and block row k+1 of B, all
//      that step k+1's diagonal block and panel read;
//   2  the rest (A columns >= k+2, B rows >= k+2), which can run beside
//      step k+1's diagonal and panel kernels.
// The accumulators start from -(old tile), loaded together with the first
// operand chunk, and the tile is stored negated: no read after the products.
template <class Cfg>
__global__ __launch_bounds__(256) void k_chol_trailing(double* __restrict__ A, double* __restrict__ Li,
                                                       int N, int kb, int kn,
                                                       const int* __restrict__ info, int part) {
  if (*info) return;
  const int nb = 64;
  const int k = kb + kn - 1;
  const int nblk = (N + nb - 1) / nb;
  const int rem = nblk - k - 1;
  const int t = blockIdx.x;
  const cx<double>* Ac = reinterpret_cast<const cx<double>*>(A);
  const cx<double>* Lc = reinterpret_cast<const cx<double>*>(Li);
  double* smem = smem_base<Cfg>();
  const int kw = min(N, (k + 1) * nb) - kb * nb;
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
  LoadDenseKC<Cfg, 64, Cfg::LDA, double, false> la;      // L_il[m][.] at A[(i*nb+m)*N + kb*nb + .]
  la.p = Ac + kb * nb;
  la.ld = N;
  la.o0 = r0;
  la.oend = N;
  if (herk) {
    LoadDenseKC<Cfg, 64, Cfg::LDB, double, true> lb;     // conj(L_jl[n][.])
    lb.p = Ac + kb * nb;
    lb.ld = N;
    lb.o0 = c0;
    lb.oend = N;
    mainloop<Cfg, false>(la, lb, 0, kw, acc, smem);
  } else {
    LoadDenseOC<Cfg, 64, Cfg::LDB, double, false> lb;    // Y_lj[.][n] at Li[(kb*nb+.)*N + j*nb + n]
    lb.p = Lc + (size_t)(kb * nb) * N;
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


// host launcher

// One factorisation step's trailing launches of step range kb .. kb + kn - 1
// over tiles `part`.
template <class Cfg>
static void trailing(double* A, double* Li, int N, int kb, int kn, int* info, int part,
                     hipStream_t st) {
  const int nblk = cdiv(N, 64);
  const int k = kb + kn - 1;
  const int rem = nblk - k - 1;
  int tiles;
  if (part == 1) {
    tiles = rem + (k + 1);
  } else {
    const int r = part == 2 ? rem - 1 : rem;
    tiles = r * (r + 1) / 2 + r * (k + 1);
  }
  if (tiles <= 0) return;
  hipLaunchKernelGGL(k_chol_trailing<Cfg>, dim3(tiles), dim3(256), smem_bytes<Cfg>(), st, A, Li, N,
                     kb, kn, (const int*)info, part);
}

// Blocked right-looking factorisation, 64-column steps.  nb = 64: every
// step updates the whole trailing matrix (rank 64).  nb = 128 (two-level):
// the first step of each pair updates only the next block column (and block
// row of the inverse), and after the second step one rank-128 update covers
// the rest, so the trailing matrix is read and written half as often and
// each tile runs twice the matrix products per load of its old value (at
// N = 16384: 238 against 260 ms).
//
// With an auxiliary stream `aux` the factorisation looks ahead: the trailing
// tiles the next step's diagonal block and panel read (part 1) run on s, the
// rest (part 2) on aux beside the next diagonal and panel kernels.  Events
// order part 2 after the panel it reads, and every later launch on s that
// touches its tiles after it.  Without aux everything runs on s in order.
template <class Cfg>
static hipError_t cholinv(double* A, double* Li, int N, double lam, int* info, hipStream_t s,
                          hipStream_t aux, int nb) {
  const int nblk = cdiv(N, 64);
  const int kn_max = nb / 64;
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
  auto wait_rest = [&]() {
    if (rest_pending) {
      err = hipStreamWaitEvent(s, ev_rest, 0);
      rest_pending = false;
    }
  };
  for (int kb = 0; kb < nblk && err == hipSuccess; kb += kn_max) {
    const int kn = std::min(kn_max, nblk - kb);
    for (int k = kb; k < kb + kn && err == hipSuccess; ++k) {
      hipLaunchKernelGGL(k_chol_diag<kDiagWaves>, dim3(1), dim3(64 * kDiagWaves), diag_smem, s, A, Li,
                         N, 64, k, lam, info);
      if (nblk - 1 > 0)   // (nblk-k-1) panel tiles + k inverse tiles
        hipLaunchKernelGGL(k_chol_panel, dim3(nblk - 1), dim3(256), sm, s, A, Li, N, k,
                           (const int*)info);
      if (k + 1 < kb + kn) {
        // inside a pair: the next step's block column and row from this step
        // alone (after the previous pair's part 2, which updated them)
        wait_rest();
        if (err != hipSuccess) break;
        trailing<Cfg>(A, Li, N, k, 1, info, 1, s);
      }
    }
    if (err != hipSuccess) break;
    const int last = kb + kn - 1;
    if (nblk - last - 1 <= 0) break;
    if (!aux) {
      trailing<Cfg>(A, Li, N, kb, kn, info, 0, s);
      err = hipGetLastError();
      continue;
    }
    // part 2 (aux) after this pair's last panel and after the previous part 2
    if ((err = hipEventRecord(ev_panel, s)) != hipSuccess) break;
    if ((err = hipStreamWaitEvent(aux, ev_panel, 0)) != hipSuccess) break;
    // part 1 (s) after the previous part 2
    wait_rest();
    if (err != hipSuccess) break;
    trailing<Cfg>(A, Li, N, kb, kn, info, 1, s);
    if (nblk - last - 2 > 0) {
      trailing<Cfg>(A, Li, N, kb, kn, info, 2, aux);
      if ((err = hipEventRecord(ev_rest, aux)) != hipSuccess) break;
      rest_pending = true;
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

// The trailing tiles run four real products per complex product: three (Gauss)
// took longer at N = 16384 (321 against 260 ms at nb = 64, 277 against 238
// at nb = 128), the third LDS plane and the extra accumulators (one wavefront
// per SIMD instead of two) outweighing the fewer matrix products.
hipError_t launch_cholinv(double* A, double* Li, int N, double lam, int* info, hipStream_t s,
                          hipStream_t aux, int nb) {
  if (nb != 64 && nb != 128) return hipErrorInvalidValue;
  return cholinv<CholCfg>(A, Li, N, lam, info, s, aux, nb);
}

}  // namespace pinv
