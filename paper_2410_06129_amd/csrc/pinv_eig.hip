// The eigenvalue route (Eq. 7) with truncation (Sec. 2.1, Eq. 4): the FP64
// Gram's Hermitian eigendecomposition E^H E = P Lambda P^H by the parallel
// cyclic Jacobi method, the eigenvalues sorted (largest first) and truncated
// by a condition number or an energy fraction, and the kept eigenpairs as the
// factor Q^H = diag(sqrt f) P_r^H (f_j = 1 / (mu_j + lam)) that the
// triangular-product kernels then apply densely: W = Q^H E^H, R = Q W.
//
// Jacobi: every step pairs all indices (the round-robin "circle" order: index
// 0 fixed, the others rotating one place per step, N - 1 steps a sweep) and
// applies the N/2 disjoint 2 x 2 unitary rotations that zero the paired
// off-diagonal entries, A <- U^H A U and V <- V U, in one elementwise pass.
// For a pair (p, q) with H = [[a, b], [conj b, d]]: with w = conj(b)/|b|,
// diag(1, w) makes the pair real symmetric, and the real rotation
// [[c, s], [-s, c]] with tau = (d - a) / (2|b|), t = sign(tau) / (|tau| +
// sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c diagonalises it, so
//   U[p][p] = c, U[q][p] = -s w, U[p][q] = s, U[q][q] = c w.
#include "../../include/pinv.h"
#include "pinv_internal.h"

namespace pinv {

__device__ __forceinline__ cx<double> cadd(cx<double> a, cx<double> b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cx<double> conjc(cx<double> a) { return {a.re, -a.im}; }

// Layout of the eigensolver's small workspace (bytes from its start).
struct EigWork {
  size_t sums, rank, part, us, up, order, total;
  EigWork(int N) {
    const size_t np = N + (N & 1);
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    sums = 0;
    rank = 256;
    part = 1024;
    us = al(part + 2 * 512 * sizeof(double));
    up = al(us + np * 2 * sizeof(double));
    order = al(up + np * 2 * sizeof(double));
    total = al(order + (size_t)N * sizeof(int));
  }
};

// Player at position `pos` of the circle at step `step` (np players, even).
__device__ __forceinline__ int circle_player(int pos, int step, int np) {
  return pos == 0 ? 0 : 1 + (pos - 1 + step) % (np - 1);
}

// Rotations of one step: for every index i the entries U[i][i] (us) and
// U[partner][i] (up) of the step's unitary U, the partner being the index
// paired with i in the step's circle order.
__global__ __launch_bounds__(256) void k_jac_rot(const double* __restrict__ A, int N, int np,
                                                 int step, double* __restrict__ us,
                                                 double* __restrict__ up) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np / 2) return;
  const int p = circle_player(k, step, np), q = circle_player(np - 1 - k, step, np);
  cx<double>* Us = reinterpret_cast<cx<double>*>(us);
  cx<double>* Up = reinterpret_cast<cx<double>*>(up);
  if (p >= N || q >= N) {   // paired with the padding index of an odd N
    const int r = p < N ? p : q;
    if (r < N) {
      Us[r] = cx<double>{1.0, 0.0};
      Up[r] = cx<double>{0.0, 0.0};
    }
    return;
  }
  const cx<double>* a = reinterpret_cast<const cx<double>*>(A);
  const double app = a[(size_t)p * N + p].re, aqq = a[(size_t)q * N + q].re;
  const cx<double> b = a[(size_t)p * N + q];
  const double ab = hypot(b.re, b.im);
  if (ab == 0.0) {
    Us[p] = Us[q] = cx<double>{1.0, 0.0};
    Up[p] = Up[q] = cx<double>{0.0, 0.0};
    return;
  }
  const double tau = (aqq - app) / (2.0 * ab);
  double t;
  if (fabs(tau) > 1e150)
    t = 0.5 / tau;
  else
    t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
  const cx<double> w{b.re / ab, -b.im / ab};   // conj(b) / |b|
  Us[p] = cx<double>{c, 0.0};
  Up[p] = cx<double>{-s * w.re, -s * w.im};
  Us[q] = cx<double>{c * w.re, c * w.im};
  Up[q] = cx<double>{s, 0.0};
}

// A2 = U^H A U (blockIdx.z = 0) and V2 = V U (blockIdx.z = 1) for the step's
// block-diagonal U.  A thread takes one pair (p', q') of the step's columns
// and, for A, one pair (p, q) of its rows: it reads the four entries
// A[p|q][p'|q'] once and writes their rotated values; for V it takes one row
// and the column pair.  With u_x = U[x][x] and v_x = U[partner x][x]:
//   (A U)[i][p'] = A[i][p'] u_p' + A[i][q'] v_p',  (A U)[i][q'] = A[i][q'] u_q' + A[i][p'] v_q'
//   A2[p][j] = conj(u_p) (A U)[p][j] + conj(v_p) (A U)[q][j]   (and p, q swapped)
// An index paired with the padding of an odd N keeps u = 1, v = 0 and its
// partner's entries count as zero.  Consecutive threads take consecutive
// column pairs, whose p' run up and q' run down the row: both coalesce.
// (Forming the rotations here instead of in k_jac_rot, each thread from the
// pair entries it needs, was slower: 10.5 against 6.1 s of Jacobi at
// N = 2304, the FP64 divides and square roots and the scattered diagonal
// reads outweighing the saved launch.)
__global__ __launch_bounds__(256) void k_jac_apply(const double* __restrict__ A, double* __restrict__ A2,
                                                   const double* __restrict__ V, double* __restrict__ V2,
                                                   int N, int np, int step,
                                                   const double* __restrict__ us,
                                                   const double* __restrict__ up) {
  const int l = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (l >= np / 2) return;
  const cx<double>* Us = reinterpret_cast<const cx<double>*>(us);
  const cx<double>* Up = reinterpret_cast<const cx<double>*>(up);
  const cx<double> zero{0.0, 0.0};
  const int jp = circle_player(l, step, np), jq = circle_player(np - 1 - l, step, np);
  const bool hjp = jp < N, hjq = jq < N;
  const cx<double> ujp = hjp ? Us[jp] : cx<double>{1.0, 0.0}, vjp = hjp ? Up[jp] : zero;
  const cx<double> ujq = hjq ? Us[jq] : cx<double>{1.0, 0.0}, vjq = hjq ? Up[jq] : zero;
  // a row's two entries of the column pair, times U
  auto cols = [&](const cx<double>* row, cx<double>& yp, cx<double>& yq) {
    const cx<double> xp = hjp ? row[jp] : zero, xq = hjq ? row[jq] : zero;
    yp = cadd(cmul(xp, ujp), cmul(xq, vjp));
    yq = cadd(cmul(xq, ujq), cmul(xp, vjq));
  };
  if (blockIdx.z == 0) {
    if (r >= np / 2) return;
    const int ip = circle_player(r, step, np), iq = circle_player(np - 1 - r, step, np);
    const bool hip_ = ip < N, hiq = iq < N;
    const cx<double>* a = reinterpret_cast<const cx<double>*>(A);
    cx<double> pp = zero, pq = zero, qp = zero, qq = zero;
    if (hip_) cols(a + (size_t)ip * N, pp, pq);
    if (hiq) cols(a + (size_t)iq * N, qp, qq);
    cx<double>* o = reinterpret_cast<cx<double>*>(A2);
    if (hip_) {
      const cx<double> u = conjc(Us[ip]), v = conjc(Up[ip]);
      if (hjp) o[(size_t)ip * N + jp] = cadd(cmul(u, pp), cmul(v, qp));
      if (hjq) o[(size_t)ip * N + jq] = cadd(cmul(u, pq), cmul(v, qq));
    }
    if (hiq) {
      const cx<double> u = conjc(Us[iq]), v = conjc(Up[iq]);
      if (hjp) o[(size_t)iq * N + jp] = cadd(cmul(u, qp), cmul(v, pp));
      if (hjq) o[(size_t)iq * N + jq] = cadd(cmul(u, qq), cmul(v, pq));
    }
  } else {
    if (r >= N) return;
    cx<double> yp, yq;
    cols(reinterpret_cast<const cx<double>*>(V) + (size_t)r * N, yp, yq);
    cx<double>* o = reinterpret_cast<cx<double>*>(V2) + (size_t)r * N;
    if (hjp) o[jp] = yp;
    if (hjq) o[jq] = yq;
  }
}

// V = I.
__global__ __launch_bounds__(256) void k_eye(double* __restrict__ V, int N) {
  cx<double>* v = reinterpret_cast<cx<double>*>(V);
  const size_t n = (size_t)N * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    v[e] = cx<double>{(e / N == e % N) ? 1.0 : 0.0, 0.0};
}

// Sums of |A_ij|^2 off and on the diagonal: per block into part[2b], part[2b+1]
// (grid-stride, fixed order), then k_sum_parts adds the blocks in order.
constexpr int kNormBlocks = 512;
__global__ __launch_bounds__(256) void k_jac_norms(const double* __restrict__ A, int N,
                                                   double* __restrict__ part) {
  const cx<double>* a = reinterpret_cast<const cx<double>*>(A);
  const size_t n = (size_t)N * N;
  double off = 0.0, dg = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> x = a[e];
    const double m = x.re * x.re + x.im * x.im;
    if (e / N == e % N) dg += m; else off += m;
  }
  __shared__ double so[256], sd[256];
  so[threadIdx.x] = off;
  sd[threadIdx.x] = dg;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      sd[threadIdx.x] += sd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = so[0];
    part[2 * blockIdx.x + 1] = sd[0];
  }
}

__global__ void k_sum_parts(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double o = 0.0, d = 0.0;
  for (int b = 0; b < nb; ++b) {
    o += part[2 * b];
    d += part[2 * b + 1];
  }
  out[0] = o;
  out[1] = d;
}

// Eigenvalues mu_j = Re A[j][j] sorted largest first (ties by index):
// spec[rank(j)] = mu_j, order[rank(j)] = j.
__global__ __launch_bounds__(256) void k_eig_rank(const double* __restrict__ A, int N,
                                                  double* __restrict__ spec, int* __restrict__ order) {
  const cx<double>* a = reinterpret_cast<const cx<double>*>(A);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  __shared__ double tile[256];
  const double mj = j < N ? a[(size_t)j * N + j].re : 0.0;
  int rank = 0;
  for (int k0 = 0; k0 < N; k0 += 256) {
    const int k = k0 + (int)threadIdx.x;
    tile[threadIdx.x] = k < N ? a[(size_t)k * N + k].re : 0.0;
    __syncthreads();
    const int kn = min(256, N - k0);
    for (int t = 0; t < kn; ++t) {
      const double mk = tile[t];
      rank += (mk > mj || (mk == mj && k0 + t < j)) ? 1 : 0;
    }
    __syncthreads();
  }
  if (j < N) {
    spec[rank] = mj;
    order[rank] = j;
  }
}

// The kept count r of the sorted eigenvalues (one workgroup): all, those with
// mu_j * kappa^2 >= mu_0 (sigma_0 / sigma_j <= kappa), or the fewest largest
// whose running sum reaches `value` of the total.  Each thread sums a
// contiguous chunk; the chunk sums are prefixed in order by thread 0.  Writes
// r to out[0] and, if a kept mu_j + lam is not > 0, j + 1 to info.
__global__ __launch_bounds__(1024) void k_eig_select(const double* __restrict__ spec, int N, int mode,
                                                      double value, double lam, int* __restrict__ out,
                                                      int* __restrict__ info) {
  __shared__ double part[1024];
  __shared__ int firsts[1024];
  __shared__ double total;
  __shared__ int kept;
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (N + nt - 1) / nt;
  const int b0 = min(N, t * per), b1 = min(N, b0 + per);
  double s = 0.0;
  int cnt = 0;
  for (int j = b0; j < b1; ++j) {
    s += spec[j];
    cnt += spec[j] * value * value >= spec[0] ? 1 : 0;
  }
  part[t] = mode == PINV_TRUNC_KAPPA ? (double)cnt : s;
  __syncthreads();
  if (t == 0) {
    double acc = 0.0;
    for (int u = 0; u < nt; ++u) {
      const double x = part[u];
      part[u] = acc;
      acc += x;
    }
    total = acc;
    kept = N;
  }
  __syncthreads();
  if (mode == PINV_TRUNC_ENERGY) {
    const double target = value * total;
    double acc = part[t];
    int first = N;
    for (int j = b0; j < b1; ++j) {
      acc += spec[j];
      if (acc >= target) {
        first = j;
        break;
      }
    }
    firsts[t] = first;
    __syncthreads();
    if (t == 0) {
      int f = N;
      for (int u = 0; u < nt; ++u) f = min(f, firsts[u]);
      kept = f < N ? f + 1 : N;
    }
    __syncthreads();
  }
  if (t == 0) {
    const int r = mode == PINV_TRUNC_KAPPA ? (int)total : kept;
    out[0] = r;
    for (int j = 0; j < r; ++j)
      if (!(spec[j] + lam > 0.0)) {
        atomicCAS(info, 0, j + 1);
        break;
      }
  }
}

// Qh[j][n] = sqrt(f_j) conj(V[n][order[j]]) for j < r, zero for j >= r,
// f_j = 1 / (mu_j + lam).
__global__ __launch_bounds__(256) void k_eig_q(const double* __restrict__ V, const double* __restrict__ spec,
                                               const int* __restrict__ order, const int* __restrict__ rank,
                                               int N, double lam, double* __restrict__ Qh) {
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (n >= N || j >= N) return;
  cx<double> q{0.0, 0.0};
  if (j < rank[0]) {
    const double mu = spec[j] + lam;
    const double g = mu > 0.0 ? sqrt(1.0 / mu) : 0.0;
    const cx<double> v = reinterpret_cast<const cx<double>*>(V)[(size_t)n * N + order[j]];
    q = cx<double>{g * v.re, -g * v.im};
  }
  reinterpret_cast<cx<double>*>(Qh)[(size_t)j * N + n] = q;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
size_t eig_work_bytes(int N) { return EigWork(N).total; }

hipError_t launch_jacobi_eig(double* A, double* A2, double* V, double* V2, int N, void* work,
                             int max_sweeps, hipStream_t s, int* sweeps, double** A_out,
                             double** V_out) {
  const int np = N + (N & 1);
  const EigWork L(N);
  char* w = (char*)work;
  double* sums = (double*)(w + L.sums);
  double* part = (double*)(w + L.part);
  double* us = (double*)(w + L.us);
  double* up = (double*)(w + L.up);
  hipLaunchKernelGGL(k_eye, dim3(1024), dim3(256), 0, s, V, N);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  // column pairs across, row pairs (A) or rows (V) down
  const dim3 agrid(cdiv(np / 2, 64), cdiv(N, 4), 2);
  double prev = -1.0;
  *sweeps = -1;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int st = 0; st < np - 1; ++st) {
      hipLaunchKernelGGL(k_jac_rot, dim3(cdiv(np / 2, 256)), dim3(256), 0, s, (const double*)A, N, np, st,
                         us, up);
      hipLaunchKernelGGL(k_jac_apply, agrid, dim3(256), 0, s, (const double*)A, A2, (const double*)V, V2,
                         N, np, st, (const double*)us, (const double*)up);
      std::swap(A, A2);
      std::swap(V, V2);
    }
    hipLaunchKernelGGL(k_jac_norms, dim3(kNormBlocks), dim3(256), 0, s, (const double*)A, N, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (const double*)part, kNormBlocks, sums);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    double h[2] = {0.0, 0.0};
    if ((err = hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) return err;
    if ((err = hipStreamSynchronize(s)) != hipSuccess) return err;
    const double off = sqrt(h[0]), tot = sqrt(h[0] + h[1]);
    // converged once the off-diagonal part is at the level of FP64 rounding,
    // or once it stops shrinking (quadratic convergence has reached that floor)
    const bool floor = off <= 1e-15 * tot;
    const bool stalled = prev >= 0.0 && off <= 1e-12 * tot && off > 0.25 * prev;
    prev = off;
    if (floor || stalled || tot == 0.0) {
      *sweeps = sw + 1;
      break;
    }
  }
  *A_out = A;
  *V_out = V;
  return hipSuccess;
}

hipError_t launch_eig_select(const double* A, const double* V, int N, int mode, double value,
                             double lam, double* spec, double* Qh, int* info, void* work, int* rank,
                             hipStream_t s) {
  const EigWork L(N);
  char* w = (char*)work;
  int* rdev = (int*)(w + L.rank);
  int* order = (int*)(w + L.order);
  hipLaunchKernelGGL(k_eig_rank, dim3(cdiv(N, 256)), dim3(256), 0, s, A, N, spec, order);
  hipLaunchKernelGGL(k_eig_select, dim3(1), dim3(1024), 0, s, (const double*)spec, N, mode, value, lam,
                     rdev, info);
  hipLaunchKernelGGL(k_eig_q, dim3(cdiv(N, 64), cdiv(N, 4)), dim3(256), 0, s, V, (const double*)spec,
                     (const int*)order, (const int*)rdev, N, lam, Qh);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if ((err = hipMemcpyAsync(rank, rdev, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return err;
  return hipStreamSynchronize(s);
}

}  // namespace pinv
