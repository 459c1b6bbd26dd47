// Gram kernels: G = E^H E with E generated per tile (Sec. 2.2; Eq. 11), the
// samples' Gram E E^H for the right pseudoinverse (Sec. 2.2), and the
// Hermitian fill of the kept FP64 Gram.
#include <type_traits>

#include "pinv_internal.h"

namespace pinv {

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
// Gram through the point-spread function (Toeplitz form).  Without an
// off-resonance map, and with every coil on one trajectory (E_c = F diag(C_c),
// Eq. 11), each Fourier factor of F depends on two voxels only through their
// offset r_b - r_a, so
//   G[a][b] = S[a][b] * P[s_a][s_b](ix_b - ix_a, iy_b - iy_a)
//   S[a][b] = sum_c conj(C_c(v_a)) C_c(v_b)                   (coil cross-products)
//   P[sa][sb](dx, dy) = sum_i exp(-i 2 pi (kx_i dx/nx + ky_i dy/ny + (f_sb - f_sa) t_i))
// k_psf forms P for every species pair on the (2nx-1) x (2ny-1) offset grid
// (FP64, the sum over samples split into partial grids that k_psf_reduce adds
// in split order), and k_psf_expand writes G.  The offset factors come from the
// build's own tables: exp(-i 2 pi kx dx/nx) = Px[i][dx] conj(Px[i][0]) for
// dx >= 0 and Px[i][0] conj(Px[i][-dx]) for dx < 0 (likewise for y), and the
// species factor is conj(Q[i][sa]) Q[i][sb].
// ---------------------------------------------------------------------------
constexpr int kPsfTile = 64;     // offsets per side of a workgroup's tile
constexpr int kPsfChunk = 16;    // samples staged in LDS per step

// Offset factor exp(-i 2 pi k d / n) for d = u - (n - 1), u in [0, 2n - 1).
__device__ __forceinline__ cx<double> psf_factor(const cx<double>* tab, int n, int u) {
  const int d = u - (n - 1);
  const cx<double> a = d >= 0 ? tab[d] : tab[0];
  const cx<double> b = d >= 0 ? tab[0] : tab[-d];
  return cx<double>{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};   // a conj(b)
}

// part[split][pair][uy][ux] = sum over this split's samples.  Grid: x = offset
// tiles (ux fastest), y = species pair, z = split.  Thread (tx, ty) owns the
// 4 x 4 offsets (ux0 + tx + 16 a, uy0 + ty + 16 b).
__global__ __launch_bounds__(256) void k_psf(EncDev<double> e, int kchunk, double* __restrict__ part) {
  const int W = 2 * e.nx - 1, H = 2 * e.ny - 1;
  const int ntx = (W + kPsfTile - 1) / kPsfTile;
  const int ux0 = (blockIdx.x % ntx) * kPsfTile, uy0 = (blockIdx.x / ntx) * kPsfTile;
  const int pair = blockIdx.y, sa = pair / e.S, sb = pair - sa * e.S;
  const int i0 = blockIdx.z * kchunk, i1 = min(e.K, i0 + kchunk);
  __shared__ cx<double> sx[kPsfChunk][kPsfTile];
  __shared__ cx<double> sy[kPsfChunk][kPsfTile];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const cx<double>* px = reinterpret_cast<const cx<double>*>(e.px);
  const cx<double>* py = reinterpret_cast<const cx<double>*>(e.py);
  const cx<double>* q = reinterpret_cast<const cx<double>*>(e.q);
  double ar[4][4], ai[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) ar[a][b] = ai[a][b] = 0.0;
  for (int ic = i0; ic < i1; ic += kPsfChunk) {
    // stage kPsfChunk samples x 64 offsets of each factor (4 entries per thread each)
    for (int idx = threadIdx.x; idx < kPsfChunk * kPsfTile; idx += 256) {
      const int r = idx / kPsfTile, u = idx - r * kPsfTile;
      const int i = ic + r;
      cx<double> fx{0.0, 0.0}, fy{0.0, 0.0};
      if (i < i1) {
        if (ux0 + u < W) fx = psf_factor(px + (size_t)i * e.nx, e.nx, ux0 + u);
        if (uy0 + u < H) {
          fy = psf_factor(py + (size_t)i * e.ny, e.ny, uy0 + u);
          if (q) {   // conj(Q[i][sa]) Q[i][sb]
            const cx<double> qa = q[(size_t)i * e.S + sa], qb = q[(size_t)i * e.S + sb];
            const cx<double> w{qa.re * qb.re + qa.im * qb.im, qa.re * qb.im - qa.im * qb.re};
            fy = cmul(fy, w);
          }
        }
      }
      sx[r][u] = fx;
      sy[r][u] = fy;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kPsfChunk; ++r) {
      cx<double> xv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = sx[r][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) yv[b] = sy[r][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          ar[a][b] += xv[a].re * yv[b].re - xv[a].im * yv[b].im;
          ai[a][b] += xv[a].re * yv[b].im + xv[a].im * yv[b].re;
        }
    }
    __syncthreads();
  }
  cx<double>* out = reinterpret_cast<cx<double>*>(part) +
                    ((size_t)blockIdx.z * gridDim.y + pair) * (size_t)W * H;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int ux = ux0 + tx + 16 * a, uy = uy0 + ty + 16 * b;
      if (ux < W && uy < H) out[(size_t)uy * W + ux] = cx<double>{ar[a][b], ai[a][b]};
    }
}

// psf[i] = sum_s part[s][i] in split order (n complex values per split).
__global__ __launch_bounds__(256) void k_psf_reduce(const double* __restrict__ part, int splits,
                                                    int64_t n, double* __restrict__ psf) {
  const cx<double>* pp = reinterpret_cast<const cx<double>*>(part);
  cx<double>* o = reinterpret_cast<cx<double>*>(psf);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double zr = pp[i].re, zi = pp[i].im;
    for (int s = 1; s < splits; ++s) {
      zr += pp[(int64_t)s * n + i].re;
      zi += pp[(int64_t)s * n + i].im;
    }
    o[i] = cx<double>{zr, zi};
  }
}

// G[a][b] = S[a][b] P[s_a][s_b](ix_b - ix_a, iy_b - iy_a) for a 64 x 64 tile,
// written to G (the factorisation's workspace) and to Gk (the Gram the plan
// keeps), both full N x N.  Thread t owns column b = b0 + t % 64 and rows
// a = a0 + t / 64 + 4 r; the coil values of the tile's rows are staged in LDS
// 16 coils at a time, its column's in registers.
__global__ __launch_bounds__(256) void k_psf_expand(EncDev<double> e, const double* __restrict__ psf,
                                                    double* __restrict__ G, double* __restrict__ Gk) {
  constexpr int CC = 16;
  const int N = e.N, V = e.V, W = 2 * e.nx - 1, H = 2 * e.ny - 1;
  const int nbt = (N + 63) / 64;
  const int a0 = (blockIdx.x / nbt) * 64, b0 = (blockIdx.x % nbt) * 64;
  const int lb = threadIdx.x & 63, la = threadIdx.x >> 6;
  const int b = b0 + lb;
  const bool bok = b < N;
  const int bb = bok ? b : 0;
  const int sb = bb / V, jb = bb - sb * V;
  int ixb, iyb;
  voxel_xy(e, jb, &ixb, &iyb);
  __shared__ cx<double> ca[CC][64];
  const cx<double>* coil = reinterpret_cast<const cx<double>*>(e.coil);
  const cx<double>* P = reinterpret_cast<const cx<double>*>(psf);
  double sr[16], si[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) sr[r] = coil ? 0.0 : 1.0, si[r] = 0.0;
  if (coil) {
    for (int c0 = 0; c0 < e.C; c0 += CC) {
      const int nc = min(CC, e.C - c0);
      for (int idx = threadIdx.x; idx < nc * 64; idx += 256) {
        const int c = idx / 64, o = idx - c * 64;
        const int a = a0 + o;
        ca[c][o] = a < N ? coil[(size_t)(c0 + c) * V + (a % V)] : cx<double>{0.0, 0.0};
      }
      __syncthreads();
      cx<double> cb[CC];
#pragma unroll
      for (int c = 0; c < CC; ++c)
        cb[c] = c < nc ? coil[(size_t)(c0 + c) * V + jb] : cx<double>{0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int al = la + 4 * r;
#pragma unroll
        for (int c = 0; c < CC; ++c) {   // conj(C_c(v_a)) C_c(v_b)
          const cx<double> x = ca[c][al];
          if (c < nc) {
            sr[r] += x.re * cb[c].re + x.im * cb[c].im;
            si[r] += x.re * cb[c].im - x.im * cb[c].re;
          }
        }
      }
      __syncthreads();
    }
  }
  cx<double>* g = reinterpret_cast<cx<double>*>(G);
  cx<double>* gk = reinterpret_cast<cx<double>*>(Gk);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int a = a0 + la + 4 * r;
    if (a >= N || !bok) continue;
    const int sa = a / V, ja = a - sa * V;
    int ixa, iya;
    voxel_xy(e, ja, &ixa, &iya);
    const cx<double> p =
        P[((size_t)(sa * e.S + sb) * H + (iyb - iya + e.ny - 1)) * W + (ixb - ixa + e.nx - 1)];
    const cx<double> v{p.re * sr[r] - p.im * si[r], p.re * si[r] + p.im * sr[r]};
    g[(size_t)a * N + b] = v;
    gk[(size_t)a * N + b] = v;
  }
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


// host launchers
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
  return with_feat_al(enc_features(e), row_aligned(e, Cfg::BK), [&](auto fc, auto al) {
    hipLaunchKernelGGL((k_gram_rows<Cfg, decltype(fc)::value, decltype(al)::value>), dim3(tiles),
                       dim3(256), smem_bytes<Cfg>(), s, e, G);
    return hipGetLastError();
  });
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

size_t psf_work_bytes(const EncDev<double>& e, int* splits) {
  const int W = 2 * e.nx - 1, H = 2 * e.ny - 1;
  const int tiles = cdiv(W, kPsfTile) * cdiv(H, kPsfTile);
  const int pairs = e.S * e.S;
  // enough workgroups to fill the device, at least 256 samples per split
  int sp = std::max(1, std::min(e.K / 256, cdiv(2048, (long)tiles * pairs)));
  sp = std::min(sp, 256);
  if (splits) *splits = sp;
  const size_t grid = (size_t)pairs * W * H * 16;
  return grid * (size_t)(sp + 1);   // partial grids, then the summed grid
}

hipError_t launch_psf_gram(const EncDev<double>& e, void* work, double* G, double* Gk,
                           hipStream_t s) {
  int splits = 1;
  (void)psf_work_bytes(e, &splits);
  const int W = 2 * e.nx - 1, H = 2 * e.ny - 1;
  const int tiles = cdiv(W, kPsfTile) * cdiv(H, kPsfTile);
  const int pairs = e.S * e.S;
  const int kchunk = cdiv(cdiv(e.K, splits), kPsfChunk) * kPsfChunk;
  splits = cdiv(e.K, kchunk);
  double* part = (double*)work;
  const int64_t n = (int64_t)pairs * W * H;
  double* psf = part + 2 * (size_t)splits * n;
  hipLaunchKernelGGL(k_psf, dim3(tiles, pairs, splits), dim3(256), 0, s, e, kchunk, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_psf_reduce, dim3(blocks), dim3(256), 0, s, (const double*)part, splits, n, psf);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const int nbt = cdiv(e.N, 64);
  hipLaunchKernelGGL(k_psf_expand, dim3((unsigned)nbt * nbt), dim3(256), 0, s, e, (const double*)psf,
                     G, Gk);
  return hipGetLastError();
}

hipError_t launch_herm_fill(double* G, int N, hipStream_t s) {
  dim3 grid(cdiv(N, 16), cdiv(N, 16));
  hipLaunchKernelGGL(k_herm_fill, grid, dim3(256), 0, s, G, N);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_gram<float>(const EncDev<float>&, double*, int, hipStream_t);
template hipError_t launch_gram<double>(const EncDev<double>&, double*, int, hipStream_t);
template hipError_t launch_gram_shared<float>(const EncDev<float>&, double*, hipStream_t);
template hipError_t launch_gram_shared<double>(const EncDev<double>&, double*, hipStream_t);

}  // namespace pinv
