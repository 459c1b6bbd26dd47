// C-ABI of libpinv: contexts, plan cache with HBM admission, encoding tables,
// and the build / apply / forward pipelines.  Every arithmetic step of the
// path runs in the kernels of pinv_gram.hip, pinv_chol.hip, pinv_trmm.hip,
// pinv_apply.hip, pinv_solve.hip and pinv_metrics.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pinv.h"
#include "pinv_internal.h"

using namespace pinv;

static thread_local std::string g_last_error;

// Records the message and clears the thread's pending HIP error, so that the
// error of a failed call is not read again by the next call's launch checks.
static pinv_status fail(pinv_status s, const std::string& msg) {
  g_last_error = msg;
  (void)hipGetLastError();
  return s;
}

// Entry of a call that launches work: the device made current, and a HIP
// error left pending by earlier calls on this thread (the caller's or a
// failed one's) cleared, so that launch checks report this call's own.
static hipError_t enter_device(int device) {
  (void)hipGetLastError();
  return hipSetDevice(device);
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess)                                                            \
      return fail(_e == hipErrorOutOfMemory ? PINV_ERR_NOMEM : PINV_ERR_DEVICE,      \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                \
  } while (0)

// ---------------------------------------------------------------------------
// objects
// ---------------------------------------------------------------------------
struct pinv_plan {
  pinv_context* ctx = nullptr;
  std::atomic<int> refs{0};
  bool cached = false;
  uint64_t key = 0;
  int prec = PINV_FP32;
  int N = 0, M = 0, K = 0, C = 0, S = 0, V = 0, nx = 0, ny = 0;
  double lam = 0.0;
  // device memory held for the plan's lifetime
  void* tab32 = nullptr;
  void* tab64 = nullptr;
  EncDev<float> e32{};
  EncDev<double> e64{};
  void* R = nullptr;
  void* Linv = nullptr;      // complex64 for FP32/BF16X3 plans, complex128 for FP64
  void* gram = nullptr;      // full Hermitian E^H E in FP64 (refinement residuals)
  bool gram_exact = true;    // false when the Gram was formed over M rows in FP32
  bool no_r = false;         // factor-only plan: no W, no R (applies solve with L^-1)
  bool right = false;        // M < N: Gram, factor and L^-1 are the samples' (M x M)
  int G = 0;                 // order of the Gram and the factor: N, or M when right
  bool m3 = true;            // W, R and apply with three real products per complex product
  int gram_form = PINV_GRAM_SHARED;   // how the Gram was formed
  bool r_fp64 = false;       // FP32 plan whose W and R were formed in FP64
  int route = PINV_ROUTE_CHOLESKY;
  int rank = 0;              // eigenvalues kept (eigenvalue route; N otherwise)
  int sweeps = 0;            // Jacobi sweeps (eigenvalue route)
  void* spec = nullptr;      // eigenvalues of E^H E, largest first (eigenvalue route)
  int* info = nullptr;
  bool pooled = false;             // device buffers from the context's plan pool
  size_t bytes = 0;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // One event per use of the plan that may still be in flight (applies,
  // metrics, copies on any stream).  A release orders the frees after the
  // build and after all of them, so it never waits on the host.
  std::mutex use_mu;
  std::vector<hipEvent_t> uses;
  bool waited = false;
  pinv_status status = PINV_OK;
  int info_host = 0;
  float stage_ms[4] = {0, 0, 0, 0};
  std::list<pinv_plan*>::iterator lru_it;
};

struct pinv_context {
  int device = 0;
  hipStream_t aux_nb = nullptr;   // the factorisation's look-ahead stream (non-blocking)
  // Buffers of released plans whose last uses may still run: freed into the
  // plan pool once all their events have completed (see free_plan_memory).
  struct PendingFree {
    std::vector<void*> bufs;
    std::vector<hipEvent_t> evs;
  };
  std::mutex free_mu;
  std::vector<PendingFree> pending;
  hipMemPool_t build_pool = nullptr;   // build workspaces (Gram, FP64 factor, W)
  hipMemPool_t plan_pool = nullptr;    // plan buffers (R, L^-1, Gram, tables)
  // pinned staging for table uploads, reused by every build of the context:
  // stage_ev marks the completion of the last copies out of it
  std::mutex stage_mu;
  void* stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  size_t budget = 0;
  size_t used = 0;
  std::mutex mu;
  std::unordered_map<uint64_t, pinv_plan*> cache;
  std::list<pinv_plan*> lru;   // front = most recently used
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

// FNV-1a 64-bit hash (Fowler, Noll, Vo) over raw bytes.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  }
  template <typename X> void add(const X& x) { add(&x, sizeof(X)); }
};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct Dims {
  int nx, ny, V, S, C, K, N, M;
  int Vg;          // grid voxels nx*ny (V = Vg without a mask, nvox with one)
  bool has_q, has_coil, has_b0, masked;
};

pinv_status validate(const pinv_encoding* e, Dims* d) {
  if (!e) return fail(PINV_ERR_INVALID, "encoding is NULL");
  if (e->nx < 1 || e->ny < 1) return fail(PINV_ERR_INVALID, "nx and ny must be >= 1");
  if (e->nk < 1) return fail(PINV_ERR_INVALID, "nk must be >= 1");
  if (!e->k) return fail(PINV_ERR_INVALID, "k is NULL");
  if (e->ncoil < 1) return fail(PINV_ERR_INVALID, "ncoil must be >= 1");
  if (e->nspecies < 1) return fail(PINV_ERR_INVALID, "nspecies must be >= 1");
  if (e->ncoil > 1 && !e->coil) return fail(PINV_ERR_INVALID, "ncoil > 1 needs coil maps");
  if (e->nspecies > 1 && !e->species_hz)
    return fail(PINV_ERR_INVALID, "nspecies > 1 needs species_hz");
  const bool need_t = e->nspecies > 1 || e->species_hz != nullptr || e->b0_hz != nullptr;
  if (need_t && !e->t) return fail(PINV_ERR_INVALID, "sample times t are required with species or B0");
  const long long Vg = (long long)e->nx * e->ny;
  if (e->nx > 32767 || e->ny > 32767) return fail(PINV_ERR_UNSUPPORTED, "nx and ny above 32767");
  long long V = Vg;
  if (e->voxels) {
    if (e->nvox < 1) return fail(PINV_ERR_INVALID, "a voxel mask needs nvox >= 1");
    for (int j = 0; j < e->nvox; ++j) {
      if (e->voxels[j] < 0 || e->voxels[j] >= Vg)
        return fail(PINV_ERR_INVALID, "voxel index " + std::to_string(e->voxels[j]) +
                                          " outside the grid");
      if (j > 0 && e->voxels[j] <= e->voxels[j - 1])
        return fail(PINV_ERR_INVALID, "voxel mask must be strictly ascending");
    }
    V = e->nvox;
  }
  const long long N = V * e->nspecies;
  const long long M = (long long)e->ncoil * e->nk;
  if (N > 65536) return fail(PINV_ERR_UNSUPPORTED, "N = S*nx*ny above 65536");
  if (M > (1LL << 30)) return fail(PINV_ERR_UNSUPPORTED, "M = C*nk above 2^30");
  d->nx = e->nx;
  d->ny = e->ny;
  d->V = (int)V;
  d->Vg = (int)Vg;
  d->masked = e->voxels != nullptr;
  d->S = e->nspecies;
  d->C = e->ncoil;
  d->K = (int)e->nk;
  d->N = (int)N;
  d->M = (int)M;
  bool q = false;
  if (e->species_hz)
    for (int s = 0; s < e->nspecies; ++s) q = q || e->species_hz[s] != 0.0;
  d->has_q = q || e->nspecies > 1;
  d->has_coil = e->coil != nullptr;
  d->has_b0 = e->b0_hz != nullptr;
  for (long long i = 0; i < 2 * (long long)e->nk; ++i)
    if (!isfinite(e->k[i])) return fail(PINV_ERR_INVALID, "non-finite k");
  return PINV_OK;
}

uint64_t plan_key(const pinv_encoding* e, const Dims& d, double lam, int prec, int form_bits,
                  double trunc_value) {
  Fnv f;
  f.add(d.nx);
  f.add(d.ny);
  f.add(d.K);
  f.add(d.C);
  f.add(d.S);
  f.add(e->k, sizeof(double) * 2 * d.K);
  f.add(uint8_t(e->t != nullptr));
  if (e->t) f.add(e->t, sizeof(double) * d.K);
  f.add(uint8_t(e->coil != nullptr));
  if (e->coil) f.add(e->coil, sizeof(double) * 2 * (size_t)d.C * d.Vg);
  f.add(uint8_t(e->b0_hz != nullptr));
  if (e->b0_hz) f.add(e->b0_hz, sizeof(double) * d.Vg);
  f.add(uint8_t(d.masked));
  if (d.masked) f.add(e->voxels, sizeof(int32_t) * d.V);
  f.add(uint8_t(e->species_hz != nullptr));
  if (e->species_hz) f.add(e->species_hz, sizeof(double) * d.S);
  f.add(lam);
  f.add(prec);
  f.add(form_bits);
  f.add(trunc_value);
  return f.h;
}

// exp(-i 2 pi turns) with the turn count reduced to (-1/2, 1/2] first.
inline void phasor(double turns, double* re, double* im) {
  const double f = turns - nearbyint(turns);
  *re = cos(2.0 * M_PI * f);
  *im = -sin(2.0 * M_PI * f);
}

// Host FP64 tables (Px, Py, Q, coil, b0, t), laid out contiguously.
struct HostTables {
  std::vector<double> px, py, q, coil, b0, t;
  std::vector<int32_t> vxy;   // (iy << 16) | ix of each unknown voxel (masked encodings only)
};

void build_tables(const pinv_encoding* e, const Dims& d, HostTables* h) {
  h->px.resize(2 * (size_t)d.K * d.nx);
  h->py.resize(2 * (size_t)d.K * d.ny);
  for (int i = 0; i < d.K; ++i) {
    const double kx = e->k[2 * i], ky = e->k[2 * i + 1];
    for (int ix = 0; ix < d.nx; ++ix) {
      const double x = (ix - d.nx / 2.0) / d.nx;
      phasor(kx * x, &h->px[2 * ((size_t)i * d.nx + ix)], &h->px[2 * ((size_t)i * d.nx + ix) + 1]);
    }
    for (int iy = 0; iy < d.ny; ++iy) {
      const double y = (iy - d.ny / 2.0) / d.ny;
      phasor(ky * y, &h->py[2 * ((size_t)i * d.ny + iy)], &h->py[2 * ((size_t)i * d.ny + iy) + 1]);
    }
  }
  if (d.has_q) {
    h->q.resize(2 * (size_t)d.K * d.S);
    for (int i = 0; i < d.K; ++i)
      for (int s = 0; s < d.S; ++s) {
        const double f = e->species_hz ? e->species_hz[s] : 0.0;
        phasor(f * e->t[i], &h->q[2 * ((size_t)i * d.S + s)], &h->q[2 * ((size_t)i * d.S + s) + 1]);
      }
  }
  // coil maps and the off-resonance map at the unknown voxels only
  auto grid_voxel = [&](int j) { return d.masked ? (size_t)e->voxels[j] : (size_t)j; };
  if (d.has_coil) {
    h->coil.resize(2 * (size_t)d.C * d.V);
    for (int c = 0; c < d.C; ++c)
      for (int j = 0; j < d.V; ++j) {
        const size_t src = 2 * ((size_t)c * d.Vg + grid_voxel(j)), dst = 2 * ((size_t)c * d.V + j);
        h->coil[dst] = e->coil[src];
        h->coil[dst + 1] = e->coil[src + 1];
      }
  }
  if (d.has_b0) {
    h->b0.resize(d.V);
    for (int j = 0; j < d.V; ++j) h->b0[j] = e->b0_hz[grid_voxel(j)];
    h->t.assign(e->t, e->t + d.K);
  }
  if (d.masked) {
    h->vxy.resize(d.V);
    for (int j = 0; j < d.V; ++j) {
      const int v = e->voxels[j], iy = v / d.nx, ix = v - iy * d.nx;
      h->vxy[j] = (iy << 16) | ix;
    }
  }
}

// Bytes of the tables as type T in one device buffer (each table 256-aligned).
template <typename T>
size_t tables_bytes(const HostTables& h) {
  size_t tot = 0;
  for (size_t n : {h.px.size(), h.py.size(), h.q.size(), h.coil.size(), h.b0.size(), h.t.size()})
    tot += align256(n * sizeof(T));
  return tot + align256(h.vxy.size() * sizeof(int32_t));
}

// Converts the tables to T into `host` (pinned staging, tables_bytes<T> long)
// and copies them to `dev` on s.
template <typename T>
pinv_status upload_tables(const HostTables& h, const Dims& d, hipStream_t s, void* host, void* dev,
                          EncDev<T>* ev) {
  const size_t n_px = h.px.size(), n_py = h.py.size(), n_q = h.q.size(), n_c = h.coil.size(),
               n_b = h.b0.size(), n_t = h.t.size();
  size_t off[6], tot = 0;
  const size_t ns[6] = {n_px, n_py, n_q, n_c, n_b, n_t};
  for (int i = 0; i < 6; ++i) {
    off[i] = tot;
    tot += align256(ns[i] * sizeof(T));
  }
  const std::vector<double>* src[6] = {&h.px, &h.py, &h.q, &h.coil, &h.b0, &h.t};
  for (int i = 0; i < 6; ++i) {
    T* dst = (T*)((char*)host + off[i]);
    for (size_t j = 0; j < ns[i]; ++j) dst[j] = (T)(*src[i])[j];
  }
  const size_t off_vxy = tot;
  if (!h.vxy.empty()) {
    memcpy((char*)host + off_vxy, h.vxy.data(), h.vxy.size() * sizeof(int32_t));
    tot += align256(h.vxy.size() * sizeof(int32_t));
  }
  HIPCHK(hipMemcpyAsync(dev, host, tot, hipMemcpyHostToDevice, s));
  char* b = (char*)dev;
  ev->px = (const T*)(b + off[0]);
  ev->py = (const T*)(b + off[1]);
  ev->q = n_q ? (const T*)(b + off[2]) : nullptr;
  ev->coil = n_c ? (const T*)(b + off[3]) : nullptr;
  ev->b0 = n_b ? (const T*)(b + off[4]) : nullptr;
  ev->t = n_t ? (const T*)(b + off[5]) : nullptr;
  ev->vxy = h.vxy.empty() ? nullptr : (const int*)(b + off_vxy);
  ev->nx = d.nx;
  ev->ny = d.ny;
  ev->S = d.S;
  ev->C = d.C;
  ev->K = d.K;
  ev->V = d.V;
  ev->M = d.M;
  ev->N = d.N;
  return PINV_OK;
}

// Record that work just enqueued on `s` reads the plan.  Events whose work
// has finished are re-recorded; one still pending is never overwritten, so a
// stream handle that was destroyed and handed out again cannot hide work.
hipError_t note_use(const pinv_plan* pc, hipStream_t s) {
  pinv_plan* p = (pinv_plan*)pc;
  std::lock_guard<std::mutex> g(p->use_mu);
  hipEvent_t ev = nullptr;
  for (hipEvent_t e : p->uses)
    if (hipEventQuery(e) == hipSuccess) {
      ev = e;
      break;
    }
  (void)hipGetLastError();
  if (!ev) {
    const hipError_t r = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (r != hipSuccess) return r;
    p->uses.push_back(ev);
  }
  return hipEventRecord(ev, s);
}

// Return a plan's buffers.  Pooled buffers, with the build's and every
// recorded use's events, go on the context's pending list without waiting on
// the host or on any stream; drain_frees hands them to the plan pool once
// those events have completed, on the stream of the allocation that needs
// the memory, where the pool can reuse it at once.  No stream waits on the
// events: with few hardware queues per process a wait would also hold back
// unrelated work sharing the waiting stream's queue.  Buffers from hipMalloc
// (no plan pool) are freed after the device has finished with them.
void free_plan_memory(pinv_plan* p) {
  pinv_context* c = p->ctx;
  void* const bufs[] = {p->tab32, p->tab64, p->R, p->Linv, p->gram, (void*)p->info, p->spec};
  if (p->pooled) {
    pinv_context::PendingFree f;
    for (void* q : bufs)
      if (q) f.bufs.push_back(q);
    for (hipEvent_t& e : p->ev)
      if (e) f.evs.push_back(e), e = nullptr;
    for (hipEvent_t e : p->uses) f.evs.push_back(e);
    p->uses.clear();
    std::lock_guard<std::mutex> g(c->free_mu);
    c->pending.push_back(std::move(f));
    return;
  }
  (void)hipDeviceSynchronize();
  for (void* q : bufs)
    if (q) (void)hipFree(q);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->uses) (void)hipEventDestroy(e);
  p->uses.clear();
}

// Free the pending buffers whose events have all completed (all of them, after
// waiting on the host, with `wait`) into the plan pool, stream-ordered on s.
void drain_frees(pinv_context* c, hipStream_t s, bool wait) {
  std::lock_guard<std::mutex> g(c->free_mu);
  for (size_t i = 0; i < c->pending.size();) {
    pinv_context::PendingFree& f = c->pending[i];
    bool done = true;
    for (hipEvent_t e : f.evs) {
      if (wait) {
        (void)hipEventSynchronize(e);
      } else if (hipEventQuery(e) != hipSuccess) {
        done = false;
        break;
      }
    }
    (void)hipGetLastError();
    if (!done) {
      ++i;
      continue;
    }
    for (void* q : f.bufs) (void)hipFreeAsync(q, s);
    for (hipEvent_t e : f.evs) (void)hipEventDestroy(e);
    c->pending.erase(c->pending.begin() + i);
  }
}

// Build options after defaults: the complex-product form of W, R and the
// apply, the Gram form, and whether W and R are formed in FP64.
// Factorisation block size when the options leave it at 0.
constexpr int kDefaultNb = 128;

struct BuildForm {
  bool m3 = true;
  int nb = kDefaultNb;
  int gram = PINV_GRAM_SHARED;
  bool r_fp64 = false;
  bool no_r = false;
  int route = PINV_ROUTE_CHOLESKY;
  int trunc = PINV_TRUNC_NONE;
  double trunc_value = 0.0;
};

// Sweep cap of the Jacobi eigensolver.  Its Grams are ill conditioned with
// clustered small eigenvalues, so the off-diagonal mass falls only a few times
// per sweep until it is below their gaps: 29 sweeps at N = 1024, 35 at 2304.
constexpr int kMaxJacobiSweeps = 60;

// Device bytes a build needs at its peak: plan buffers plus build workspaces.
size_t plan_footprint(const Dims& d, int prec, const BuildForm& f) {
  const size_t N = d.N, M = d.M;
  const bool right = d.M < d.N;
  const size_t Gd = right ? M : N;   // order of the Gram and the factor
  const size_t cs = prec == PINV_FP64 ? 16 : 8;
  const size_t ws = f.r_fp64 ? 16 : cs;   // W (and Z) element size
  size_t b = 0;
  b += 16 * Gd * Gd;            // Gram / factor workspace (FP64)
  b += 16 * Gd * Gd;            // L^-1 in FP64 during the factorisation
  b += cs * Gd * Gd;            // L^-1 kept
  if (!f.no_r && prec == PINV_BF16X3) {
    // split-packed L^-1 and L^-H, W^T and R (rows padded to 32 columns), and
    // a slab of conj(E) during the W product
    const size_t Np = sp_cols(N), Mp = sp_cols(M);
    b += 2 * 8 * N * Np + 8 * M * Np + 8 * N * Mp + 8 * Np * (size_t)e_slab_rows(N, M);
  } else if (!f.no_r) {
    b += ws * N * M;            // W (and Z for the right pseudoinverse)
    if (right) b += ws * N * M;
    b += cs * N * M;            // R
  }
  b += 16 * Gd * Gd;            // the Gram kept
  if (f.route == PINV_ROUTE_EIGEN)
    b += 3 * 16 * N * N + eig_work_bytes((int)N) + 8 * N;   // Jacobi copies, eigenvalues
  if (f.gram == PINV_GRAM_PSF) {
    EncDev<double> e{};
    e.nx = d.nx;
    e.ny = d.ny;
    e.S = d.S;
    e.K = d.K;
    b += psf_work_bytes(e, nullptr);
  }
  b += 64ull << 20;             // tables and slack
  return b;
}

size_t plan_resident(const Dims& d, int prec, bool no_r) {
  const size_t N = d.N, M = d.M;
  const size_t Gd = d.M < d.N ? M : N;
  const size_t cs = prec == PINV_FP64 ? 16 : 8;
  const size_t r = no_r ? 0 : prec == PINV_BF16X3 ? 8 * N * sp_cols(M) : cs * N * M;
  return r + cs * Gd * Gd + 16 * Gd * Gd + 8 * Gd + (16ull << 20);
}

// Evict LRU plans held only by the cache until `need` bytes fit.  ctx->mu held.
bool make_room(pinv_context* c, size_t need) {
  if (c->used + need <= c->budget) return true;
  for (auto it = c->lru.end(); it != c->lru.begin();) {
    --it;
    pinv_plan* p = *it;
    if (p->refs.load() == 1 && p->cached) {   // only the cache holds it
      c->cache.erase(p->key);
      it = c->lru.erase(it);
      c->used -= p->bytes;
      free_plan_memory(p);
      delete p;
      if (c->used + need <= c->budget) return true;
    }
  }
  return c->used + need <= c->budget;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* pinv_status_string(pinv_status s) {
  switch (s) {
    case PINV_OK: return "ok";
    case PINV_ERR_INVALID: return "invalid argument";
    case PINV_ERR_NOMEM: return "out of device memory or budget";
    case PINV_ERR_NOT_PD: return "shifted Gram matrix is not positive definite";
    case PINV_ERR_DEVICE: return "device error";
    case PINV_ERR_BUSY: return "busy";
    case PINV_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* pinv_last_error(void) { return g_last_error.c_str(); }

// Streams the library creates for itself, one set per device, kept for the
// life of the process.  HIP maps streams onto a few hardware queues per
// process (four by default); streams created and destroyed with every context
// or server landed on different queues each time, and a server whose build
// and apply streams ended up sharing one queue served half as fast.  Created
// once, in a fixed order, the mapping stays put.
//  * aux_nb: non-blocking: the factorisation's look-ahead stream (the bulk of
//    each trailing update beside the next diagonal block and panel), the
//    serving loop's build stream, and frees with no allocating stream.  (A
//    stream kept off the last 32 CUs, leaving them to the one-workgroup
//    diagonal kernel, gained nothing with rank-128 trailing updates: 262
//    against 238 ms at N = 16384, where only every second diagonal block runs
//    beside a trailing update.)
//  * apply: the serving loop's apply stream.
struct DeviceStreams {
  hipStream_t aux_nb = nullptr, apply = nullptr;
};

static std::mutex g_streams_mu;
static std::unordered_map<int, DeviceStreams>* g_streams = nullptr;

// Process exit: hand the streams back before the HIP runtime tears down (the
// handler is registered after the runtime has initialised, so it runs first).
static void destroy_device_streams() {
  std::lock_guard<std::mutex> g(g_streams_mu);
  if (!g_streams) return;
  for (auto& kv : *g_streams) {
    (void)hipSetDevice(kv.first);
    (void)hipStreamDestroy(kv.second.aux_nb);
    (void)hipStreamDestroy(kv.second.apply);
  }
  g_streams->clear();
}

static bool device_streams(int device, DeviceStreams* out) {
  std::lock_guard<std::mutex> g(g_streams_mu);
  if (!g_streams) {
    g_streams = new std::unordered_map<int, DeviceStreams>();
    std::atexit(destroy_device_streams);
  }
  auto& streams = *g_streams;
  auto it = streams.find(device);
  if (it != streams.end()) {
    *out = it->second;
    return true;
  }
  DeviceStreams d;
  if (hipStreamCreateWithFlags(&d.aux_nb, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipStreamCreateWithFlags(&d.apply, hipStreamNonBlocking) != hipSuccess) return false;
  streams[device] = d;
  *out = d;
  return true;
}

// Record a failure's detail for pinv_last_error (library-internal).
extern "C++" pinv_status pinv_fail(pinv_status s, const std::string& msg) { return fail(s, msg); }

// The device a context runs on (library-internal).
extern "C++" int pinv_context_device(const pinv_context* c) { return c->device; }

// The serving loop's build and apply streams on `device` (library-internal).
extern "C++" bool pinv_serving_streams(int device, hipStream_t* build, hipStream_t* apply) {
  DeviceStreams d;
  if (!device_streams(device, &d)) return false;
  *build = d.aux_nb;
  *apply = d.apply;
  return true;
}

pinv_status pinv_context_create(int device, size_t budget, pinv_context** out) {
  if (!out) return fail(PINV_ERR_INVALID, "out is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(PINV_ERR_INVALID, "no such device");
  HIPCHK(enter_device(device));
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  pinv_context* c = new pinv_context();
  c->device = device;
  c->budget = budget ? budget : (size_t)(0.9 * (double)fr);
  DeviceStreams ds;
  if (!device_streams(device, &ds)) {
    pinv_context_destroy(c);
    return fail(PINV_ERR_DEVICE, "cannot create the library's streams");
  }
  c->aux_nb = ds.aux_nb;
  // Keep freed stream-ordered allocations (build workspaces, scratch) mapped
  // across synchronisations: the pool's default release threshold of 0 hands
  // them back at every synchronising call, and the next build then pays for
  // mapping W afresh inside its first kernel.  Memory goes back to the device
  // only through the explicit trims (pinv_plan_wait, pinv_context_trim).
  hipMemPool_t pool;
  uint64_t keep = UINT64_MAX;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess)
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  // Build workspaces come from a pool of their own, so the per-call scratch of
  // applies and refinement (default pool) cannot split a freed multi-GB
  // workspace and force the next build to map a new one.
  hipMemPoolProps props;
  memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  props.maxSize = tot;
  if (hipMemPoolCreate(&c->build_pool, &props) == hipSuccess)
    (void)hipMemPoolSetAttribute(c->build_pool, hipMemPoolAttrReleaseThreshold, &keep);
  else
    c->build_pool = nullptr, (void)hipGetLastError();
  if (hipMemPoolCreate(&c->plan_pool, &props) == hipSuccess)
    (void)hipMemPoolSetAttribute(c->plan_pool, hipMemPoolAttrReleaseThreshold, &keep);
  else
    c->plan_pool = nullptr, (void)hipGetLastError();
  if (hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming) != hipSuccess) {
    pinv_context_destroy(c);
    return fail(PINV_ERR_DEVICE, "cannot create the staging event");
  }
  *out = c;
  return PINV_OK;
}

pinv_status pinv_context_destroy(pinv_context* c) {
  if (!c) return fail(PINV_ERR_INVALID, "context is NULL");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> g(c->mu);
    for (pinv_plan* p : c->lru) {
      free_plan_memory(p);
      delete p;
    }
    c->lru.clear();
    c->cache.clear();
  }
  if (c->aux_nb) {
    drain_frees(c, c->aux_nb, true);
    (void)hipStreamSynchronize(c->aux_nb);
  }
  if (c->build_pool) (void)hipMemPoolDestroy(c->build_pool);
  if (c->plan_pool) (void)hipMemPoolDestroy(c->plan_pool);
  if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
  if (c->stage) (void)hipHostFree(c->stage);
  delete c;   // the library's streams stay for the next context
  return PINV_OK;
}

// Validate a build request and derive the absolute shift, the cache key and
// the resolved options.
static pinv_status check_build(const pinv_encoding* e, const pinv_build_opts* o, Dims* d,
                               double* lam_out, uint64_t* key_out, BuildForm* form) {
  if (!o) return fail(PINV_ERR_INVALID, "NULL options");
  pinv_status st = validate(e, d);
  if (st != PINV_OK) return st;
  if (o->prec != PINV_FP64 && o->prec != PINV_FP32 && o->prec != PINV_BF16X3)
    return fail(PINV_ERR_INVALID, "unknown precision");
  if (o->flags & ~(PINV_FLAG_KEEP_GRAM | PINV_FLAG_UNCACHED | PINV_FLAG_GRAM_FULL | PINV_FLAG_NO_R |
                   PINV_FLAG_R_FP64))
    return fail(PINV_ERR_INVALID, "unknown flag bits");
  if (o->cprod < PINV_CPROD_AUTO || o->cprod > PINV_CPROD_4M)
    return fail(PINV_ERR_INVALID, "unknown cprod");
  if (o->nb != 0 && o->nb != 64 && o->nb != 128)
    return fail(PINV_ERR_UNSUPPORTED, "nb must be 0, 64 or 128: the factorisation steps 64 columns "
                                      "at a time (its diagonal block holds one column per lane of "
                                      "a wavefront) and updates the trailing matrix every 64 or "
                                      "128 columns");
  if (o->gram < PINV_GRAM_AUTO || o->gram > PINV_GRAM_FULL)
    return fail(PINV_ERR_INVALID, "unknown gram form");
  if (!(o->lambda >= 0.0) || !isfinite(o->lambda)) return fail(PINV_ERR_INVALID, "lambda must be finite and >= 0");
  double lam = o->lambda;
  if (o->lambda_mode == PINV_LAMBDA_REL_MEAN_DIAG) {
    // trace(E^H E) = K * S * sum_v sum_c |C_c(v)|^2 over the unknown voxels, since
    // every phase factor has modulus 1
    double cp = 0.0;
    if (e->coil) {
      for (int c = 0; c < d->C; ++c)
        for (int j = 0; j < d->V; ++j) {
          const size_t i = (size_t)c * d->Vg + (d->masked ? (size_t)e->voxels[j] : (size_t)j);
          cp += e->coil[2 * i] * e->coil[2 * i] + e->coil[2 * i + 1] * e->coil[2 * i + 1];
        }
    } else {
      cp = (double)d->V;
    }
    lam = o->lambda * (double)d->K * d->S * cp / (double)d->N;
  } else if (o->lambda_mode != PINV_LAMBDA_ABS) {
    return fail(PINV_ERR_INVALID, "unknown lambda_mode");
  }
  const bool no_r = (o->flags & PINV_FLAG_NO_R) != 0;
  const bool r_fp64 = (o->flags & PINV_FLAG_R_FP64) != 0;
  if (o->route != PINV_ROUTE_CHOLESKY && o->route != PINV_ROUTE_EIGEN)
    return fail(PINV_ERR_INVALID, "unknown route");
  if (o->trunc < PINV_TRUNC_NONE || o->trunc > PINV_TRUNC_ENERGY)
    return fail(PINV_ERR_INVALID, "unknown truncation mode");
  if (o->route == PINV_ROUTE_CHOLESKY && o->trunc != PINV_TRUNC_NONE)
    return fail(PINV_ERR_INVALID, "truncation needs PINV_ROUTE_EIGEN");
  if (o->trunc == PINV_TRUNC_KAPPA && !(o->trunc_value >= 1.0 && isfinite(o->trunc_value)))
    return fail(PINV_ERR_INVALID, "PINV_TRUNC_KAPPA needs trunc_value >= 1");
  if (o->trunc == PINV_TRUNC_ENERGY && !(o->trunc_value > 0.0 && o->trunc_value <= 1.0))
    return fail(PINV_ERR_INVALID, "PINV_TRUNC_ENERGY needs trunc_value in (0, 1]");
  if (o->route == PINV_ROUTE_EIGEN) {
    if (o->prec == PINV_BF16X3)
      return fail(PINV_ERR_UNSUPPORTED, "PINV_ROUTE_EIGEN with PINV_BF16X3");
    if (no_r) return fail(PINV_ERR_INVALID, "PINV_ROUTE_EIGEN forms R; PINV_FLAG_NO_R refused");
    if (d->M < d->N)
      return fail(PINV_ERR_UNSUPPORTED, "PINV_ROUTE_EIGEN needs M >= N (the unknowns' Gram)");
  }
  int gram = o->gram;
  if (o->flags & PINV_FLAG_GRAM_FULL) {
    if (gram != PINV_GRAM_AUTO && gram != PINV_GRAM_FULL)
      return fail(PINV_ERR_INVALID, "PINV_FLAG_GRAM_FULL with another gram form");
    gram = PINV_GRAM_FULL;
  }
  if (no_r && o->prec == PINV_BF16X3)
    return fail(PINV_ERR_INVALID, "PINV_FLAG_NO_R with PINV_BF16X3: the split products only form W and R");
  if (o->prec == PINV_BF16X3 && o->cprod != PINV_CPROD_AUTO)
    return fail(PINV_ERR_INVALID, "PINV_BF16X3 plans take cprod = PINV_CPROD_AUTO");
  if (r_fp64 && o->prec != PINV_FP32)
    return fail(PINV_ERR_INVALID, "PINV_FLAG_R_FP64 is for PINV_FP32 plans");
  if (r_fp64 && no_r) return fail(PINV_ERR_INVALID, "PINV_FLAG_R_FP64 with PINV_FLAG_NO_R: no R");
  if (d->M < d->N) {   // right pseudoinverse through the samples' Gram
    if (no_r) return fail(PINV_ERR_INVALID, "PINV_FLAG_NO_R needs M >= N (the unknowns' Gram)");
    if (o->prec == PINV_BF16X3)
      return fail(PINV_ERR_UNSUPPORTED, "PINV_BF16X3 with M < N (right pseudoinverse)");
    if (gram != PINV_GRAM_AUTO)
      return fail(PINV_ERR_INVALID, "M < N forms the samples' Gram; gram must be PINV_GRAM_AUTO");
    gram = PINV_GRAM_SHARED;
  } else if (gram == PINV_GRAM_AUTO) {
    gram = d->has_b0 ? PINV_GRAM_SHARED : PINV_GRAM_PSF;
  } else if (gram == PINV_GRAM_PSF && d->has_b0) {
    return fail(PINV_ERR_INVALID, "PINV_GRAM_PSF needs an encoding without an off-resonance map");
  }
  form->gram = gram;
  form->no_r = no_r;
  form->r_fp64 = r_fp64;
  form->route = o->route;
  form->trunc = o->route == PINV_ROUTE_EIGEN ? o->trunc : PINV_TRUNC_NONE;
  form->trunc_value = form->trunc == PINV_TRUNC_NONE ? 0.0 : o->trunc_value;
  // AUTO: 3M for the FP32 products; 4M for FP64 products, where 3M saved no
  // time (W at N = 16384: 6.97 s on 3M against 4.74 s on 4M, the FP64 element
  // generation and the third LDS plane outweighing the fewer matrix products)
  form->m3 = o->cprod == PINV_CPROD_3M   ? true
             : o->cprod == PINV_CPROD_4M ? false
                                         : o->prec != PINV_FP64 && !r_fp64;
  form->nb = o->nb == 0 ? kDefaultNb : o->nb;
  *lam_out = lam;
  const int bits = (form->m3 ? 1 : 0) | (gram << 1) | (r_fp64 ? 16 : 0) | (no_r ? 32 : 0) |
                   (form->route << 6) | (form->trunc << 7) | (form->nb == 128 ? 1 << 9 : 0);
  *key_out = plan_key(e, *d, lam, o->prec, bits, form->trunc_value);
  return PINV_OK;
}

pinv_status pinv_encoding_key(const pinv_encoding* e, const pinv_build_opts* o, uint64_t* key,
                              size_t* plan_bytes) {
  Dims d;
  double lam;
  uint64_t k;
  BuildForm form;
  pinv_status st = check_build(e, o, &d, &lam, &k, &form);
  if (st != PINV_OK) return st;
  if (key) *key = k;
  if (plan_bytes) *plan_bytes = plan_footprint(d, o->prec, form);
  return PINV_OK;
}

// Return memory that stream-ordered frees left in the pools to the device, so
// that allocations outside them (the caller's tensors) can use it: per-call
// scratch (the device's default pool) and build workspaces (the build pool),
// and with `plans` also freed plan buffers (the plan pool).  Unforced, only
// when less than a quarter of the device is free: re-mapping a freed multi-GB
// buffer costs the next build milliseconds inside its first kernel and slows
// whatever else runs meanwhile.  Plan memory is handed back only on request or
// when a plan or workspace allocation fails, so later plans reuse it.
static void trim_pool(pinv_context* c, bool force, bool plans) {
  size_t fr = 0, tot = 0;
  if (!force && hipMemGetInfo(&fr, &tot) == hipSuccess && fr >= tot / 4) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  if (c->build_pool) (void)hipMemPoolTrimTo(c->build_pool, 0);
  if (plans && c->plan_pool) {
    // released plans whose work has finished go back as well
    drain_frees(c, c->aux_nb, false);
    (void)hipStreamSynchronize(c->aux_nb);
    (void)hipMemPoolTrimTo(c->plan_pool, 0);
  }
}

// Scratch and workspaces back to the device under memory pressure (the
// serving loop calls this after each batch).
extern "C++" void pinv_context_trim_scratch(pinv_context* c) { trim_pool(c, false, false); }

// Scratch reclaim for calls that allocate from the default pool: the stream's
// own frees complete, then every pool of the context hands its unused memory
// (build workspaces and released plans included) back to the device.
static void reclaim_pools(void* arg, hipStream_t s) {
  (void)hipStreamSynchronize(s);
  trim_pool((pinv_context*)arg, true, true);
}

// A stream-ordered allocation from the default pool for a call's own
// temporaries, tried once more after reclaim_pools when memory is short.
static hipError_t pool_alloc(pinv_context* c, void** ptr, size_t bytes, hipStream_t s) {
  hipError_t e = hipMallocAsync(ptr, bytes, s);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    reclaim_pools(c, s);
    e = hipMallocAsync(ptr, bytes, s);
  }
  return e;
}

// A build workspace, stream-ordered on s, from the context's build pool.
static hipError_t workspace_alloc(void** ptr, size_t bytes, pinv_context* c, hipStream_t s) {
  auto once = [&]() {
    return c->build_pool ? hipMallocFromPoolAsync(ptr, bytes, c->build_pool, s)
                         : hipMallocAsync(ptr, bytes, s);
  };
  hipError_t e = once();
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    trim_pool(c, true, true);
    e = once();
  }
  return e;
}

// A plan buffer, stream-ordered on s from the context's plan pool (plain
// hipMalloc if the pool could not be created); when the device is out of
// memory, freed pool memory is handed back and the allocation tried once more.
static hipError_t plan_malloc(void** ptr, size_t bytes, pinv_context* c, hipStream_t s) {
  auto once = [&]() {
    return c->plan_pool ? hipMallocFromPoolAsync(ptr, bytes, c->plan_pool, s) : hipMalloc(ptr, bytes);
  };
  drain_frees(c, s, false);   // released plans' memory, reusable on s at once
  hipError_t e = once();
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s);
    drain_frees(c, s, true);
    (void)hipStreamSynchronize(s);
    trim_pool(c, true, true);
    e = once();
  }
  return e;
}

pinv_status pinv_build(pinv_context* c, const pinv_encoding* e, const pinv_build_opts* o,
                       void* stream, pinv_plan** out) {
  if (!c || !o || !out) return fail(PINV_ERR_INVALID, "NULL argument");
  Dims d;
  double lam;
  uint64_t key;
  BuildForm form;
  pinv_status st = check_build(e, o, &d, &lam, &key, &form);
  if (st != PINV_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(c->device));

  const bool uncached = (o->flags & PINV_FLAG_UNCACHED) != 0;
  std::lock_guard<std::mutex> g(c->mu);
  auto hit = uncached ? c->cache.end() : c->cache.find(key);
  if (hit != c->cache.end()) {
    pinv_plan* p = hit->second;
    p->refs++;
    c->lru.erase(p->lru_it);
    c->lru.push_front(p);
    p->lru_it = c->lru.begin();
    *out = p;
    return PINV_OK;
  }
  const bool no_r = form.no_r;
  const size_t foot = plan_footprint(d, o->prec, form);
  if (!make_room(c, foot))
    return fail(PINV_ERR_NOMEM, "plan footprint " + std::to_string(foot) +
                                    " B exceeds the free budget");

  pinv_plan* p = new pinv_plan();
  p->ctx = c;
  p->key = key;
  p->prec = o->prec;
  p->N = d.N;
  p->M = d.M;
  p->K = d.K;
  p->C = d.C;
  p->S = d.S;
  p->V = d.V;
  p->nx = d.nx;
  p->ny = d.ny;
  p->lam = lam;
  p->no_r = no_r;
  p->right = d.M < d.N;
  p->G = p->right ? d.M : d.N;
  p->m3 = form.m3;
  p->gram_form = form.gram;
  p->r_fp64 = form.r_fp64;
  p->route = form.route;
  p->rank = (int)d.N;
  auto cleanup = [&](pinv_status rs) {
    (void)hipStreamSynchronize(s);
    free_plan_memory(p);
    delete p;
    return rs;
  };

  HostTables ht;
  build_tables(e, d, &ht);
  const size_t N = d.N, M = d.M;
  const bool f64 = o->prec == PINV_FP64;
  const size_t cs = f64 ? 16 : 8;
  const size_t ws = form.r_fp64 ? 16 : cs;   // W and Z element size
  void *G = nullptr, *L64 = nullptr, *W = nullptr, *Z = nullptr, *PW = nullptr;
  void *LS = nullptr, *LHS = nullptr, *ES = nullptr;   // split-packed L^-1, L^-H, conj(E) slab (BF16X3)
  const bool b3 = o->prec == PINV_BF16X3;
  const size_t Gd = p->G;   // order of the Gram and the factor
  hipError_t he;
#define BCHK(expr)                                                                    \
  do {                                                                                \
    he = (expr);                                                                      \
    if (he != hipSuccess) {                                                           \
      fail(he == hipErrorOutOfMemory ? PINV_ERR_NOMEM : PINV_ERR_DEVICE,              \
           std::string(#expr) + ": " + hipGetErrorString(he));                        \
      if (G) (void)hipFreeAsync(G, s);                                                \
      if (L64 && L64 != p->Linv) (void)hipFreeAsync(L64, s);                          \
      if (W) (void)hipFreeAsync(W, s);                                                \
      if (Z) (void)hipFreeAsync(Z, s);                                                \
      if (PW) (void)hipFreeAsync(PW, s);                                              \
      if (LS) (void)hipFreeAsync(LS, s);                                              \
      if (LHS) (void)hipFreeAsync(LHS, s);                                            \
      if (ES) (void)hipFreeAsync(ES, s);                                              \
      return cleanup(he == hipErrorOutOfMemory ? PINV_ERR_NOMEM : PINV_ERR_DEVICE);   \
    }                                                                                 \
  } while (0)

  // Plan buffers come stream-ordered from the context's plan pool and the
  // tables are staged through its reusable pinned buffer: a build in steady
  // state maps no new memory while earlier work still runs on the device.
  p->pooled = c->plan_pool != nullptr;
  const size_t b64 = tables_bytes<double>(ht), b32 = f64 ? 0 : tables_bytes<float>(ht);
  BCHK(plan_malloc(&p->tab64, b64, c, s));
  if (!f64) BCHK(plan_malloc(&p->tab32, b32, c, s));
  {
    std::lock_guard<std::mutex> g(c->stage_mu);
    BCHK(hipEventSynchronize(c->stage_ev));   // earlier copies out of the staging buffer are done
    if (c->stage_bytes < b64 + b32) {
      if (c->stage) (void)hipHostFree(c->stage);
      c->stage = nullptr;
      c->stage_bytes = 0;
      BCHK(hipHostMalloc(&c->stage, b64 + b32, hipHostMallocDefault));
      c->stage_bytes = b64 + b32;
    }
    st = upload_tables<double>(ht, d, s, c->stage, p->tab64, &p->e64);
    if (st == PINV_OK && !f64)
      st = upload_tables<float>(ht, d, s, (char*)c->stage + b64, p->tab32, &p->e32);
    if (st == PINV_OK) BCHK(hipEventRecord(c->stage_ev, s));
  }
  if (st != PINV_OK) return cleanup(st);
  for (auto& ev : p->ev) BCHK(hipEventCreate(&ev));
  BCHK(plan_malloc((void**)&p->info, sizeof(int), c, s));
  BCHK(hipMemsetAsync(p->info, 0, sizeof(int), s));
  // a BF16X3 plan keeps R split-packed (rows n, sp_cols(M) columns)
  if (!no_r) BCHK(plan_malloc(&p->R, b3 ? 8 * N * sp_cols(M) : cs * N * M, c, s));
  BCHK(plan_malloc(&p->Linv, cs * Gd * Gd, c, s));
  BCHK(plan_malloc(&p->gram, 16 * Gd * Gd, c, s));
  if (form.route == PINV_ROUTE_EIGEN) BCHK(plan_malloc(&p->spec, 8 * Gd, c, s));
  p->gram_exact = !(form.gram == PINV_GRAM_FULL && !f64);
  BCHK(workspace_alloc(&G, 16 * Gd * Gd, c, s));
  if (f64) {
    L64 = p->Linv;
  } else {
    BCHK(workspace_alloc(&L64, 16 * Gd * Gd, c, s));
  }
  BCHK(hipMemsetAsync(L64, 0, 16 * Gd * Gd, s));
  if (!no_r) BCHK(workspace_alloc(&W, b3 ? 8 * M * sp_cols(N) : ws * N * M, c, s));
  int64_t slab = 0;
  if (b3 && !no_r && !p->right && form.route == PINV_ROUTE_CHOLESKY) {
    // split-packed L^-1 and L^-H rows and the conj(E) slab, mapped before the
    // first stage so no stage's interval includes growing the pool
    const size_t Np = sp_cols(N);
    slab = e_slab_rows(N, M);
    BCHK(workspace_alloc(&LS, 8 * N * Np, c, s));
    BCHK(workspace_alloc(&LHS, 8 * N * Np, c, s));
    BCHK(workspace_alloc(&ES, 8 * (size_t)slab * Np, c, s));
  }
  if (p->right) BCHK(workspace_alloc(&Z, ws * N * M, c, s));
  if (form.gram == PINV_GRAM_PSF) BCHK(workspace_alloc(&PW, psf_work_bytes(p->e64, nullptr), c, s));

  // 1. Gram (a3) with E generated per tile (a2), or through the PSF
  BCHK(hipEventRecord(p->ev[0], s));
  if (form.gram == PINV_GRAM_PSF) {
    // offset-grid PSF times the coil cross-products, written to the workspace
    // and the kept Gram (both full Hermitian)
    BCHK(launch_psf_gram(p->e64, PW, (double*)G, (double*)p->gram, s));
    BCHK(hipFreeAsync(PW, s));
    PW = nullptr;
  } else {
    if (p->right)
      BCHK(launch_gram_rows(p->e64, (double*)G, s));   // FP64 E E^H over the N unknowns
    else if (form.gram == PINV_GRAM_SHARED)
      BCHK(launch_gram_shared<double>(p->e64, (double*)G, s));   // FP64 F^H F, coil products (Eq. 11)
    else if (f64)
      BCHK(launch_gram<double>(p->e64, (double*)G, 0, s));
    else
      BCHK(launch_gram<float>(p->e32, (double*)G, 2048, s));
    BCHK(hipMemcpyAsync(p->gram, G, 16 * Gd * Gd, hipMemcpyDeviceToDevice, s));
    BCHK(launch_herm_fill((double*)p->gram, (int)Gd, s));
    // the eigendecomposition works on the whole Hermitian matrix
    if (form.route == PINV_ROUTE_EIGEN) BCHK(launch_herm_fill((double*)G, (int)Gd, s));
  }
  BCHK(hipEventRecord(p->ev[1], s));
  if (form.route == PINV_ROUTE_EIGEN) {
    // 2. the Gram's eigendecomposition (Jacobi, FP64; synchronous), the
    // truncation, and Q^H = diag(1/sqrt(mu_j + lam)) P_r^H into L64
    void *A2 = nullptr, *V = nullptr, *V2 = nullptr, *EW = nullptr;
    auto eig = [&]() -> hipError_t {
      hipError_t r = workspace_alloc(&A2, 16 * N * N, c, s);
      if (r == hipSuccess) r = workspace_alloc(&V, 16 * N * N, c, s);
      if (r == hipSuccess) r = workspace_alloc(&V2, 16 * N * N, c, s);
      if (r == hipSuccess) r = workspace_alloc(&EW, eig_work_bytes((int)N), c, s);
      double *Af = nullptr, *Vf = nullptr;
      if (r == hipSuccess)
        r = launch_jacobi_eig((double*)G, (double*)A2, (double*)V, (double*)V2, (int)N, EW,
                              kMaxJacobiSweeps, s, &p->sweeps, &Af, &Vf);
      if (r == hipSuccess && p->sweeps > 0)
        r = launch_eig_select(Af, Vf, (int)N, form.trunc, form.trunc_value, lam, (double*)p->spec,
                              (double*)L64, p->info, EW, &p->rank, s);
      for (void* q : {EW, V2, V, A2})
        if (q) (void)hipFreeAsync(q, s);
      return r;
    };
    BCHK(eig());
    if (p->sweeps < 0) {
      fail(PINV_ERR_UNSUPPORTED, "the Jacobi eigendecomposition did not converge in " +
                                     std::to_string(kMaxJacobiSweeps) + " sweeps");
      (void)hipFreeAsync(G, s);
      if (!f64) (void)hipFreeAsync(L64, s);
      if (W) (void)hipFreeAsync(W, s);
      return cleanup(PINV_ERR_UNSUPPORTED);
    }
    if (!f64) BCHK(launch_to_f32((const double*)L64, (float*)p->Linv, Gd * Gd, s));
    BCHK(hipEventRecord(p->ev[2], s));
    // 3. W = Q^H E^H (rank rows), R = Q W
    const int r = p->rank;
    if (f64) {
      BCHK(launch_trmm_w<double>(p->e64, (const double*)p->Linv, (double*)W, form.m3, s, r));
      BCHK(hipEventRecord(p->ev[3], s));
      BCHK((launch_trmm_r<double, double>((const double*)p->Linv, (const double*)W, (double*)p->R,
                                          d.N, d.M, form.m3, s, r)));
    } else if (form.r_fp64) {
      BCHK(launch_trmm_w<double>(p->e64, (const double*)L64, (double*)W, form.m3, s, r));
      BCHK(hipEventRecord(p->ev[3], s));
      BCHK((launch_trmm_r<double, float>((const double*)L64, (const double*)W, (float*)p->R, d.N,
                                         d.M, form.m3, s, r)));
    } else {
      BCHK(launch_trmm_w<float>(p->e32, (const float*)p->Linv, (float*)W, form.m3, s, r));
      BCHK(hipEventRecord(p->ev[3], s));
      BCHK((launch_trmm_r<float, float>((const float*)p->Linv, (const float*)W, (float*)p->R, d.N,
                                        d.M, form.m3, s, r)));
    }
  } else {
  // 2. shift + blocked Cholesky with L^-1 (a4), FP64
  BCHK(launch_cholinv((double*)G, (double*)L64, (int)Gd, lam, p->info, s,
                      p->ctx->aux_nb, form.nb));
  if (!f64) BCHK(launch_to_f32((const double*)L64, (float*)p->Linv, Gd * Gd, s));
  BCHK(hipEventRecord(p->ev[2], s));
  // 3. W = L^-1 E^H, R = L^-H W (a5); a factor-only plan stops at L^-1.  With
  // fewer samples than unknowns, W' = L'^-1 E, Z = L'^-H W' and R = Z^H.
  // An FP32 plan with FP64-formed R runs both products in FP64 from the FP64
  // factor and tables and rounds R once to complex64.
  const bool m3 = form.m3;
  if (no_r) {
    BCHK(hipEventRecord(p->ev[3], s));
  } else if (p->right) {
    BCHK(hipEventRecord(p->ev[3], s));
    if (f64)
      BCHK((launch_right_pinv<double, double>(p->e64, (const double*)p->Linv, (double*)W, (double*)Z,
                                              (double*)p->R, m3, s)));
    else if (form.r_fp64)
      BCHK((launch_right_pinv<double, float>(p->e64, (const double*)L64, (double*)W, (double*)Z,
                                             (float*)p->R, m3, s)));
    else
      BCHK((launch_right_pinv<float, float>(p->e32, (const float*)p->Linv, (float*)W, (float*)Z,
                                            (float*)p->R, m3, s)));
  } else if (f64) {
    BCHK(launch_trmm_w<double>(p->e64, (const double*)p->Linv, (double*)W, m3, s));
    BCHK(hipEventRecord(p->ev[3], s));
    BCHK((launch_trmm_r<double, double>((const double*)p->Linv, (const double*)W, (double*)p->R, d.N,
                                        d.M, m3, s)));
  } else if (form.r_fp64) {
    BCHK(launch_trmm_w<double>(p->e64, (const double*)L64, (double*)W, m3, s));
    BCHK(hipEventRecord(p->ev[3], s));
    BCHK((launch_trmm_r<double, float>((const double*)L64, (const double*)W, (float*)p->R, d.N, d.M,
                                       m3, s)));
  } else if (b3) {
    // the factor split once into bf16 hi/lo planes, as rows of L^-1 and of
    // L^-H; the products write W^T and R split-packed
    BCHK(launch_sp_pack<double>((const double*)L64, (int64_t)N, d.N, d.N, false, false, LS, s));
    BCHK(launch_sp_pack<double>((const double*)L64, (int64_t)N, d.N, d.N, true, true, LHS, s));
    BCHK(launch_trmm_w_sp(p->e32, LS, W, ES, slab, s));
    BCHK(hipFreeAsync(ES, s));
    ES = nullptr;
    BCHK(hipEventRecord(p->ev[3], s));
    BCHK(launch_trmm_r_sp(W, LHS, p->R, d.N, d.M, s));
    BCHK(hipFreeAsync(LHS, s));
    LHS = nullptr;
    BCHK(hipFreeAsync(LS, s));
    LS = nullptr;
  } else {
    BCHK(launch_trmm_w<float>(p->e32, (const float*)p->Linv, (float*)W, m3, s));
    BCHK(hipEventRecord(p->ev[3], s));
    BCHK((launch_trmm_r<float, float>((const float*)p->Linv, (const float*)W, (float*)p->R, d.N, d.M,
                                      m3, s)));
  }
  }   // route
  BCHK(hipEventRecord(p->ev[4], s));
  if (W) BCHK(hipFreeAsync(W, s));
  W = nullptr;
  if (Z) BCHK(hipFreeAsync(Z, s));
  Z = nullptr;
  BCHK(hipFreeAsync(G, s));
  G = nullptr;
  if (!f64) {
    BCHK(hipFreeAsync(L64, s));
  }
  L64 = nullptr;
#undef BCHK
  // the pinned staging buffers stay with the plan until its build has finished

  p->bytes = plan_resident(d, o->prec, no_r);
  c->used += p->bytes;
  if (uncached) {
    p->refs = 1;   // the caller only
    p->cached = false;
  } else {
    p->refs = 2;   // the cache and the caller
    p->cached = true;
    c->cache[key] = p;
    c->lru.push_front(p);
    p->lru_it = c->lru.begin();
  }
  *out = p;
  return PINV_OK;
}

extern "C" pinv_status pinv_context_trim(pinv_context* c) {
  if (!c) return fail(PINV_ERR_INVALID, "context is NULL");
  HIPCHK(enter_device(c->device));
  trim_pool(c, true, true);
  return PINV_OK;
}

pinv_status pinv_plan_wait(pinv_plan* p) {
  if (!p) return fail(PINV_ERR_INVALID, "plan is NULL");
  if (!p->waited) {
    HIPCHK(enter_device(p->ctx->device));
    HIPCHK(hipEventSynchronize(p->ev[4]));
    trim_pool(p->ctx, false, false);
    HIPCHK(hipMemcpy(&p->info_host, p->info, sizeof(int), hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) HIPCHK(hipEventElapsedTime(&p->stage_ms[i], p->ev[i], p->ev[i + 1]));
    if (p->no_r) p->stage_ms[2] = p->stage_ms[3] = 0.f;   // no W or R was formed
    p->status = p->info_host ? PINV_ERR_NOT_PD : PINV_OK;
    p->waited = true;
  }
  if (p->status == PINV_ERR_NOT_PD)
    return fail(PINV_ERR_NOT_PD, "Cholesky pivot <= 0 or NaN at column " +
                                     std::to_string(p->info_host - 1));
  return p->status;
}

pinv_status pinv_plan_query(pinv_plan* p) {
  if (!p) return fail(PINV_ERR_INVALID, "plan is NULL");
  if (p->waited) return p->status == PINV_OK ? PINV_OK : pinv_plan_wait(p);
  hipError_t q = hipEventQuery(p->ev[4]);
  if (q == hipErrorNotReady) return PINV_ERR_BUSY;
  if (q != hipSuccess) return fail(PINV_ERR_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
  return pinv_plan_wait(p);
}

// Iterative refinement on the normal equations (Eq. 6) for one item:
//   r = E^H d - (G + lam I) x   in FP64  (b = E^H d formed once, E regenerated in FP64)
//   x += L^-H L^-1 r            (the plan's factor)
// When the plan's Gram is not exact to FP64 (FP32 Gram over all rows) the
// residual is formed as E^H (d - E x) - lam x instead.  Scratch: r and t
// (F x N of TS), and b (F x N FP64) or d - E x (F x M FP64), plus the
// adjoint's split partials.
extern "C++" {
template <typename TS>   // storage type of data/images and of the plan's L^-1
static pinv_status refine_item(pinv_plan* p, const void* data, int F, void* image, int steps,
                               Scratch& sc, hipStream_t s) {
  if (steps <= 0 || F <= 0) return PINV_OK;
  const size_t N = p->N, M = p->M;
  const TS* d = (const TS*)data;
  TS* x = (TS*)image;
  void *b = nullptr, *rd = nullptr, *r = nullptr, *t = nullptr;
  hipError_t e = sc.get(&r, 2 * sizeof(TS) * (size_t)F * N, s);
  if (e == hipSuccess) e = sc.get(&t, 2 * sizeof(TS) * (size_t)F * N, s);
  if (e == hipSuccess) {
    if (p->gram_exact) {
      e = sc.get(&b, 16 * (size_t)F * N, s);
      if (e == hipSuccess)
        e = launch_adjoint<double, TS, TS, double>(p->e64, d, F, (const TS*)nullptr, 0.0, (double*)b,
                                                   sc, s);
    } else {
      e = sc.get(&rd, 16 * (size_t)F * M, s);
    }
  }
  for (int it = 0; it < steps && e == hipSuccess; ++it) {
    if (p->gram_exact) {
      e = launch_resid<TS, TS>((const double*)p->gram, (const double*)b, x, F, p->N, p->lam, (TS*)r, s);
    } else {
      e = launch_forward<double, TS, TS>(p->e64, x, F, d, (double*)rd, s);
      if (e == hipSuccess)
        e = launch_adjoint<double, double, TS, TS>(p->e64, (const double*)rd, F, x, p->lam, (TS*)r,
                                                   sc, s);
    }
    if (e == hipSuccess) e = launch_tri_frames<TS, 0, TS>((const TS*)p->Linv, (const TS*)r, F, p->N, (TS*)t, s);
    if (e == hipSuccess) e = launch_tri_frames<TS, 1, TS>((const TS*)p->Linv, (const TS*)t, F, p->N, x, s);
  }
  for (void* q : {rd, b, t, r})   // most recent first (the fixed-region scratch is a stack)
    if (q) (void)sc.put(q, s);
  HIPCHK(e);
  return PINV_OK;
}

// Factor-only plans solve the normal equations per frame without R:
//   b = E^H d = sum_c E_c^H d_c   (E generated per tile in the plan's precision)
//   x = L^-H (L^-1 b)
// b is formed in `image`, L^-1 b in a scratch array, L^-H (L^-1 b) back in `image`.
template <typename TS>
static pinv_status solve_item(pinv_plan* p, const void* data, int F, void* image, Scratch& sc,
                              hipStream_t s) {
  const size_t N = p->N;
  TS* x = (TS*)image;
  void* t = nullptr;
  HIPCHK(sc.get(&t, 2 * sizeof(TS) * (size_t)F * N, s));
  hipError_t e;
  if constexpr (sizeof(TS) == 8)
    e = launch_adjoint<double, double, double, double>(p->e64, (const double*)data, F, nullptr, 0.0,
                                                       x, sc, s);
  else
    e = launch_adjoint<float, float, float, float>(p->e32, (const float*)data, F, nullptr, 0.0, x,
                                                   sc, s);
  if (e == hipSuccess) e = launch_tri_frames<TS, 0, TS>((const TS*)p->Linv, x, F, p->N, (TS*)t, s);
  if (e == hipSuccess) e = launch_tri_frames<TS, 2, TS>((const TS*)p->Linv, (const TS*)t, F, p->N, x, s);
  const hipError_t f = sc.put(t, s);
  HIPCHK(e);
  HIPCHK(f);
  return PINV_OK;
}

// Right-pseudoinverse plans (M < N) refine on the sample side: with
// G' = E E^H + lam I = L' L'^H and x = E^H y,
//   y = L'^-H L'^-1 d,   then per step   r = d - G' y (FP64 G', FP64 d),
//   y += L'^-H L'^-1 r,  and finally     x = E^H y (E regenerated in FP64).
// y is kept in FP64 (the triangular products accumulate into it), so the
// final product does not amplify a rounded y.
template <typename TS>
static pinv_status solve_right_item(pinv_plan* p, const void* data, int F, void* image, int steps,
                                    Scratch& sc, hipStream_t s) {
  const size_t M = p->M;
  const TS* d = (const TS*)data;
  const TS* Li = (const TS*)p->Linv;
  void *y = nullptr, *t = nullptr, *r = nullptr, *d64 = nullptr;
  hipError_t e = sc.get(&y, 16 * (size_t)F * M, s);
  if (e == hipSuccess) e = sc.get(&t, 2 * sizeof(TS) * (size_t)F * M, s);
  if (e == hipSuccess) e = sc.get(&r, 2 * sizeof(TS) * (size_t)F * M, s);
  if (e == hipSuccess && sizeof(TS) == 4) e = sc.get(&d64, 16 * (size_t)F * M, s);
  if (e == hipSuccess) e = launch_tri_frames<TS, 0, TS>(Li, d, F, p->M, (TS*)t, s);
  if (e == hipSuccess) e = launch_tri_frames<TS, 2, double>(Li, (const TS*)t, F, p->M, (double*)y, s);
  const double* b = nullptr;
  if constexpr (sizeof(TS) == 4) {
    if (e == hipSuccess) e = launch_to_f64((const float*)d, (double*)d64, (size_t)F * M, s);
    b = (const double*)d64;
  } else {
    b = (const double*)d;
  }
  for (int it = 0; it < steps && e == hipSuccess; ++it) {
    e = launch_resid<double, TS>((const double*)p->gram, b, (const double*)y, F, p->M, p->lam,
                                 (TS*)r, s);
    if (e == hipSuccess) e = launch_tri_frames<TS, 0, TS>(Li, (const TS*)r, F, p->M, (TS*)t, s);
    if (e == hipSuccess)
      e = launch_tri_frames<TS, 1, double>(Li, (const TS*)t, F, p->M, (double*)y, s);
  }
  if (e == hipSuccess)
    e = launch_adjoint<double, double, TS, TS>(p->e64, (const double*)y, F, nullptr, 0.0,
                                               (TS*)image, sc, s);
  for (void* q : {d64, r, t, y})
    if (q) (void)sc.put(q, s);
  HIPCHK(e);
  return PINV_OK;
}

// Scratch bytes one item's apply takes from a fixed region (the stack peak of
// the steps apply_items runs for it).
size_t item_scratch_bytes(const pinv_plan* p, int F, int steps) {
  if (F <= 0) return 0;
  auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t N = p->N, M = p->M;
  const size_t ts = p->prec == PINV_FP64 ? 8 : 4;
  size_t peak = 0;
  const int rows_max = row_apply_max_frames(p->prec != PINV_FP64);
  const bool tiles = F > rows_max && !p->no_r && !(p->right && steps > 0);
  if (F <= rows_max && !p->no_r && !(p->right && steps > 0)) {
    // the row apply's per-slice partial images
    peak = p->prec == PINV_FP64 ? apply_rows_scratch_bytes<double>(F, (int)N, (int)M)
                                : apply_rows_scratch_bytes<float>(F, (int)N, (int)M);
  }
  if (tiles) {
    // a BF16X3 item's data is split-packed first (F x sp_cols(M), 8 bytes each)
    const size_t Mp = sp_cols(M);
    peak = p->prec == PINV_FP64 ? apply_scratch_bytes<double>(F, (int)N, (int)M, p->m3, false)
           : p->prec == PINV_BF16X3
               ? al(8 * F * Mp) + (F <= kStreamMaxF ? apply_stream_scratch_bytes(F, (int)N, (int)Mp)
                                                    : apply_scratch_bytes_b3(F, (int)N, (int)Mp))
               : apply_scratch_bytes<float>(F, (int)N, (int)M, p->m3, p->r_fp64);
  }
  if (p->no_r) {
    const size_t adj = p->prec == PINV_FP64
                           ? adjoint_scratch_bytes<double, double, double, double>(p->e64, F)
                           : adjoint_scratch_bytes<float, float, float, float>(p->e32, F);
    peak = std::max(peak, al(2 * ts * F * N) + adj);
  }
  if (steps > 0 && p->right) {
    const size_t adj = p->prec == PINV_FP64
                           ? adjoint_scratch_bytes<double, double, double, double>(p->e64, F)
                           : adjoint_scratch_bytes<double, double, float, float>(p->e64, F);
    peak = std::max(peak, al(16 * F * M) + 2 * al(2 * ts * F * M) + (ts == 4 ? al(16 * F * M) : 0) + adj);
  } else if (steps > 0) {
    size_t refine = 2 * al(2 * ts * F * N);
    if (p->gram_exact)
      refine += al(16 * F * N) + (p->prec == PINV_FP64
                                      ? adjoint_scratch_bytes<double, double, double, double>(p->e64, F)
                                      : adjoint_scratch_bytes<double, float, float, double>(p->e64, F));
    else
      refine += al(16 * F * M) + (p->prec == PINV_FP64
                                      ? adjoint_scratch_bytes<double, double, double, double>(p->e64, F)
                                      : adjoint_scratch_bytes<double, double, float, float>(p->e64, F));
    peak = std::max(peak, refine);
  }
  return peak;
}
}  // extern "C++"

// The apply pipeline of pinv_apply_grouped with its scratch from `sc`.
extern "C++" pinv_status apply_items(pinv_context* c, int32_t n, const pinv_apply_item* items,
                                     int32_t refine_steps, Scratch& sc, hipStream_t s) {
  for (int i = 0; i < n; ++i) {
    const pinv_plan* p = (const pinv_plan*)items[i].plan;
    if (!p || p->ctx != c) return fail(PINV_ERR_INVALID, "item " + std::to_string(i) + ": bad plan");
    if (refine_steps > 0 && p->route == PINV_ROUTE_EIGEN)
      return fail(PINV_ERR_INVALID, "item " + std::to_string(i) +
                                        ": eigenvalue-route plans take no refinement (a truncated "
                                        "R is not the normal equations' solution)");
    if (items[i].F < 0 || items[i].F > (1 << 24))
      return fail(PINV_ERR_INVALID, "item " + std::to_string(i) + ": F out of range");
    if (items[i].F > 0 && (!items[i].data || !items[i].image))
      return fail(PINV_ERR_INVALID, "item " + std::to_string(i) + ": NULL buffer");
  }
  for (int i = 0; i < n; ++i) HIPCHK(hipStreamWaitEvent(s, ((const pinv_plan*)items[i].plan)->ev[4], 0));
  // grouped launches over runs of equal precision and product form, up to
  // kMaxGroup items each
  int i = 0;
  while (i < n) {
    const pinv_plan* p0 = (const pinv_plan*)items[i].plan;
    const int prec = p0->prec;
    const bool m3 = p0->m3, seg = p0->r_fp64;
    ApplyBatch b;
    b.n = 0;
    while (i < n && b.n < kMaxGroup && ((const pinv_plan*)items[i].plan)->prec == prec &&
           ((const pinv_plan*)items[i].plan)->m3 == m3 &&
           ((const pinv_plan*)items[i].plan)->r_fp64 == seg) {
      const pinv_plan* p = (const pinv_plan*)items[i].plan;
      if (items[i].F > row_apply_max_frames(p->prec != PINV_FP64) && !p->no_r &&
          !(p->right && refine_steps > 0)) {
        ApplyItemDev& it = b.it[b.n++];
        it.D = items[i].data;
        it.R = p->R;
        it.X = items[i].image;
        it.F = (int)items[i].F;
        it.N = p->N;
        it.M = p->M;
      }
      ++i;
    }
    if (b.n == 0) continue;
    if (prec == PINV_FP64) {
      HIPCHK(launch_apply<double>(b, m3, false, sc, s));
    } else if (prec == PINV_BF16X3) {
      // each item's data split-packed once; the tiles then only move bf16 planes
      void* packed[kMaxGroup] = {};
      hipError_t e = hipSuccess;
      int got = 0;
      for (; got < b.n && e == hipSuccess; ++got) {
        ApplyItemDev& it = b.it[got];
        const int64_t Mp = sp_cols(it.M);
        e = sc.get(&packed[got], (size_t)8 * it.F * Mp, s);
        if (e != hipSuccess) break;
        e = launch_sp_pack<float>((const float*)it.D, it.M, it.F, it.M, false, false, packed[got], s);
        it.D = packed[got];
        it.M = (int)Mp;
      }
      // up to kStreamMaxF frames stream R; more run as tiles
      ApplyBatch tiles;
      tiles.n = 0;
      for (int t = 0; t < b.n && e == hipSuccess; ++t) {
        const ApplyItemDev& it = b.it[t];
        if (it.F <= kStreamMaxF)
          e = launch_apply_stream_sp(it.R, it.D, (float*)it.X, it.N, it.M, it.F, sc, s);
        else
          tiles.it[tiles.n++] = it;
      }
      if (e == hipSuccess && tiles.n) e = launch_apply_b3(tiles, sc, s);
      for (int j = got - 1; j >= 0; --j)   // most recent first (the fixed-region scratch is a stack)
        if (packed[j]) {
          const hipError_t f = sc.put(packed[j], s);
          if (e == hipSuccess) e = f;
        }
      HIPCHK(e);
    } else {
      HIPCHK(launch_apply<float>(b, m3, seg, sc, s));
    }
  }
  // a few frames: stream R row by row (bound by HBM bandwidth, not MFMA)
  for (int j = 0; j < n; ++j) {
    const pinv_plan* p = (const pinv_plan*)items[j].plan;
    const int F = (int)items[j].F;
    if (p->no_r || F <= 0 || F > row_apply_max_frames(p->prec != PINV_FP64) || (p->right && refine_steps > 0))
      continue;
    if (p->prec == PINV_FP64)
      HIPCHK(launch_apply_rows<double>((const double*)p->R, (const double*)items[j].data,
                                       (double*)items[j].image, p->N, p->M, F, sc, s));
    else if (p->prec == PINV_BF16X3)
      HIPCHK(launch_apply_rows_sp(p->R, (const float*)items[j].data, (float*)items[j].image, p->N,
                                  p->M, F, sc, s));
    else
      HIPCHK(launch_apply_rows<float>((const float*)p->R, (const float*)items[j].data,
                                      (float*)items[j].image, p->N, p->M, F, sc, s));
  }
  for (int j = 0; j < n; ++j) {
    pinv_plan* p = (pinv_plan*)items[j].plan;
    if (!p->no_r || items[j].F <= 0) continue;
    const pinv_status st =
        p->prec == PINV_FP64
            ? solve_item<double>(p, items[j].data, (int)items[j].F, items[j].image, sc, s)
            : solve_item<float>(p, items[j].data, (int)items[j].F, items[j].image, sc, s);
    if (st != PINV_OK) return st;
  }
  if (refine_steps > 0) {
    for (int j = 0; j < n; ++j) {
      pinv_plan* p = (pinv_plan*)items[j].plan;
      if (items[j].F <= 0) continue;
      pinv_status st;
      if (p->right)
        st = p->prec == PINV_FP64
                 ? solve_right_item<double>(p, items[j].data, (int)items[j].F, items[j].image,
                                            refine_steps, sc, s)
                 : solve_right_item<float>(p, items[j].data, (int)items[j].F, items[j].image,
                                           refine_steps, sc, s);
      else
        st = p->prec == PINV_FP64
                 ? refine_item<double>(p, items[j].data, (int)items[j].F, items[j].image, refine_steps,
                                       sc, s)
                 : refine_item<float>(p, items[j].data, (int)items[j].F, items[j].image, refine_steps,
                                      sc, s);
      if (st != PINV_OK) return st;
    }
  }
  return PINV_OK;
}

pinv_status pinv_apply_grouped(pinv_context* c, int32_t n, const pinv_apply_item* items,
                               int32_t refine_steps, void* stream) {
  if (!c || (n > 0 && !items) || n < 0) return fail(PINV_ERR_INVALID, "bad arguments");
  if (refine_steps < 0 || refine_steps > 4) return fail(PINV_ERR_INVALID, "refine_steps in 0..4");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(c->device));
  Scratch sc;   // stream-ordered allocations from the default pool
  sc.reclaim = reclaim_pools;
  sc.reclaim_arg = c;
  const pinv_status st = apply_items(c, n, items, refine_steps, sc, s);
  if (st != PINV_OK) return st;
  for (int j = 0; j < n; ++j)
    if (items[j].F > 0) HIPCHK(note_use((const pinv_plan*)items[j].plan, s));
  return PINV_OK;
}

pinv_status pinv_apply(pinv_context* c, const pinv_plan* p, const void* data, int64_t F, void* image,
                       int32_t refine_steps, void* stream) {
  pinv_apply_item it{p, data, image, F};
  return pinv_apply_grouped(c, 1, &it, refine_steps, stream);
}

pinv_status pinv_forward(pinv_context* c, const pinv_plan* pc, const void* image, int64_t F,
                         void* data, void* stream) {
  if (!c || !pc || F < 0 || (F > 0 && (!image || !data))) return fail(PINV_ERR_INVALID, "bad arguments");
  pinv_plan* p = (pinv_plan*)pc;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(c->device));
  if (F == 0) return PINV_OK;
  HIPCHK(hipStreamWaitEvent(s, p->ev[0], 0));   // the tables are on the device
  if (p->prec == PINV_FP64) {
    HIPCHK((launch_forward<double, double, double>(p->e64, (const double*)image, (int)F, nullptr,
                                                   (double*)data, s)));
  } else {
    HIPCHK((launch_forward<float, float, float>(p->e32, (const float*)image, (int)F, nullptr,
                                                (float*)data, s)));
  }
  HIPCHK(note_use(p, s));
  return PINV_OK;
}

extern "C++" {
// Coil noise covariance factor Psi_c = Lc Lc^H (C x C, complex, row-major
// interleaved, Lc lower).  False unless Psi_c is Hermitian positive definite.
static bool coil_cholesky(const double* psi, int C, std::vector<double>& L) {
  double amax = 0.0;
  for (int i = 0; i < 2 * C * C; ++i) amax = std::max(amax, std::fabs(psi[i]));
  if (!(amax > 0.0) || !std::isfinite(amax)) return false;
  for (int a = 0; a < C; ++a)
    for (int b = 0; b < C; ++b) {
      const double dr = psi[2 * (a * C + b)] - psi[2 * (b * C + a)];
      const double di = psi[2 * (a * C + b) + 1] + psi[2 * (b * C + a) + 1];
      if (std::hypot(dr, di) > 1e-12 * amax) return false;
    }
  L.assign(2 * C * C, 0.0);
  for (int j = 0; j < C; ++j) {
    double d = psi[2 * (j * C + j)];
    for (int k = 0; k < j; ++k)
      d -= L[2 * (j * C + k)] * L[2 * (j * C + k)] + L[2 * (j * C + k) + 1] * L[2 * (j * C + k) + 1];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[2 * (j * C + j)] = ljj;
    for (int i = j + 1; i < C; ++i) {
      double sr = psi[2 * (i * C + j)], si = psi[2 * (i * C + j) + 1];
      for (int k = 0; k < j; ++k) {   // s -= L[i][k] conj(L[j][k])
        const double ar = L[2 * (i * C + k)], ai = L[2 * (i * C + k) + 1];
        const double br = L[2 * (j * C + k)], bi = L[2 * (j * C + k) + 1];
        sr -= ar * br + ai * bi;
        si -= ai * br - ar * bi;
      }
      L[2 * (i * C + j)] = sr / ljj;
      L[2 * (i * C + j) + 1] = si / ljj;
    }
  }
  return true;
}

// The plan's R as a dense complex matrix of its storage type: p->R itself, or
// for BF16X3 plans (R kept split-packed) an unpacked complex64 copy in *tmp,
// which the caller frees stream-ordered.
static hipError_t dense_r(const pinv_plan* p, hipStream_t s, const void** R, void** tmp) {
  *tmp = nullptr;
  *R = p->R;
  if (p->prec != PINV_BF16X3) return hipSuccess;
  hipError_t e = pool_alloc(p->ctx, tmp, (size_t)8 * p->N * p->M, s);
  if (e == hipSuccess) e = launch_sp_unpack(p->R, p->N, p->M, (float*)*tmp, s);
  *R = *tmp;
  return e;
}

static pinv_status metric_args(pinv_context* c, const pinv_plan* p, int32_t mode, void* out) {
  if (!c || !p || !out) return fail(PINV_ERR_INVALID, "NULL argument");
  if (p->ctx != c) return fail(PINV_ERR_INVALID, "plan belongs to another context");
  if (mode != PINV_METRIC_DIAG && mode != PINV_METRIC_FULL)
    return fail(PINV_ERR_INVALID, "mode must be PINV_METRIC_DIAG or PINV_METRIC_FULL");
  if (p->no_r) return fail(PINV_ERR_UNSUPPORTED, "the plan was built without R (PINV_FLAG_NO_R)");
  return PINV_OK;
}
}  // extern "C++"

pinv_status pinv_srf(pinv_context* c, const pinv_plan* pc, int32_t mode, void* out, void* stream) {
  const pinv_status st = metric_args(c, pc, mode, out);
  if (st != PINV_OK) return st;
  const pinv_plan* p = pc;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(c->device));
  HIPCHK(hipStreamWaitEvent(s, p->ev[4], 0));
  const void* R = nullptr;
  void* tmp = nullptr;
  hipError_t e = dense_r(p, s, &R, &tmp);
  if (e == hipSuccess) {
    if (p->prec == PINV_FP64)
      e = mode == PINV_METRIC_DIAG ? launch_srf_diag<double>(p->e64, (const double*)R, (double*)out, s)
                                   : launch_srf_full<double>(p->e64, (const double*)R, (double*)out, s);
    else
      e = mode == PINV_METRIC_DIAG ? launch_srf_diag<float>(p->e32, (const float*)R, (float*)out, s)
                                   : launch_srf_full<float>(p->e32, (const float*)R, (float*)out, s);
  }
  if (tmp) {
    const hipError_t f = hipFreeAsync(tmp, s);
    if (e == hipSuccess) e = f;
  }
  HIPCHK(e);
  HIPCHK(note_use(p, s));
  return PINV_OK;
}

extern "C++" {
namespace {
template <typename T>
pinv_status noise_impl(const pinv_plan* p, const T* R, const T* Lc, int32_t mode, T* out,
                       hipStream_t s) {
  if (mode == PINV_METRIC_DIAG) {
    HIPCHK(launch_noise_diag<T>(R, p->N, p->K, p->C, Lc, out, s));
    return PINV_OK;
  }
  if (!Lc) {
    HIPCHK(launch_noise_full<T>(R, p->N, p->M, out, s));
    return PINV_OK;
  }
  void* Rt = nullptr;
  HIPCHK(pool_alloc(p->ctx, &Rt, (size_t)p->N * p->M * 2 * sizeof(T), s));
  hipError_t e = launch_noise_mix<T>(R, p->N, p->K, p->C, Lc, (T*)Rt, s);
  if (e == hipSuccess) e = launch_noise_full<T>((const T*)Rt, p->N, p->M, out, s);
  const hipError_t f = hipFreeAsync(Rt, s);
  HIPCHK(e);
  HIPCHK(f);
  return PINV_OK;
}
}  // namespace
}  // extern "C++"

pinv_status pinv_noise(pinv_context* c, const pinv_plan* pc, const double* coil_cov, int32_t mode,
                       void* out, void* stream) {
  const pinv_status st = metric_args(c, pc, mode, out);
  if (st != PINV_OK) return st;
  const pinv_plan* p = pc;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(c->device));
  HIPCHK(hipStreamWaitEvent(s, p->ev[4], 0));
  const bool f64 = p->prec == PINV_FP64;
  const size_t rs = f64 ? 8 : 4;
  void* dL = nullptr;
  if (coil_cov) {
    std::vector<double> L;
    if (!coil_cholesky(coil_cov, p->C, L))
      return fail(PINV_ERR_INVALID, "coil_cov is not Hermitian positive definite");
    const size_t bytes = L.size() * rs;
    void* host = nullptr;
    HIPCHK(hipHostMalloc(&host, bytes, hipHostMallocDefault));
    for (size_t i = 0; i < L.size(); ++i) {
      if (f64) ((double*)host)[i] = L[i];
      else ((float*)host)[i] = (float)L[i];
    }
    hipError_t e = hipMallocAsync(&dL, bytes, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dL, host, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the staging buffer is freed next
    (void)hipHostFree(host);
    if (e != hipSuccess && dL) (void)hipFreeAsync(dL, s);
    HIPCHK(e);
  }
  const void* R = nullptr;
  void* tmp = nullptr;
  const hipError_t re = dense_r(p, s, &R, &tmp);
  pinv_status r = PINV_ERR_DEVICE;
  if (re == hipSuccess)
    r = f64 ? noise_impl<double>(p, (const double*)R, (const double*)dL, mode, (double*)out, s)
            : noise_impl<float>(p, (const float*)R, (const float*)dL, mode, (float*)out, s);
  if (tmp) (void)hipFreeAsync(tmp, s);
  if (dL) HIPCHK(hipFreeAsync(dL, s));
  HIPCHK(re);
  if (r == PINV_OK) HIPCHK(note_use(p, s));
  return r;
}

pinv_status pinv_plan_info_get(const pinv_plan* p, pinv_plan_info* out) {
  if (!p || !out) return fail(PINV_ERR_INVALID, "NULL argument");
  out->N = p->N;
  out->M = p->M;
  out->lambda_abs = p->lam;
  out->prec = p->prec;
  out->ready = p->waited && p->status == PINV_OK;
  out->key = p->key;
  out->device_bytes = p->bytes;
  for (int i = 0; i < 4; ++i) out->stage_ms[i] = p->waited ? p->stage_ms[i] : 0.f;
  out->has_r = p->no_r ? 0 : 1;
  out->gram_order = p->G;
  out->ncoil = p->C;
  out->cprod = p->m3 ? PINV_CPROD_3M : PINV_CPROD_4M;
  out->nk = p->K;
  out->gram_form = p->gram_form;
  out->r_fp64 = p->r_fp64 ? 1 : 0;
  out->route = p->route;
  out->rank = p->rank;
  out->sweeps = p->sweeps;
  out->reserved = 0;
  return PINV_OK;
}

pinv_status pinv_spectrum(pinv_context* c, const pinv_plan* p, double* out, void* stream) {
  if (!c || !p || !out) return fail(PINV_ERR_INVALID, "NULL argument");
  if (p->ctx != c) return fail(PINV_ERR_INVALID, "plan belongs to another context");
  if (p->route != PINV_ROUTE_EIGEN || !p->spec)
    return fail(PINV_ERR_INVALID, "the plan was not built with PINV_ROUTE_EIGEN");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(c->device));
  HIPCHK(hipStreamWaitEvent(s, p->ev[4], 0));
  HIPCHK(hipMemcpyAsync(out, p->spec, sizeof(double) * (size_t)p->G, hipMemcpyDeviceToDevice, s));
  HIPCHK(note_use(p, s));
  return PINV_OK;
}

pinv_status pinv_plan_buffers(const pinv_plan* p, void** R, void** Linv, void** gram) {
  if (!p) return fail(PINV_ERR_INVALID, "plan is NULL");
  if (R) *R = p->R;
  if (Linv) *Linv = p->Linv;
  if (gram) *gram = p->gram;
  return PINV_OK;
}

pinv_status pinv_plan_copy_buffer(const pinv_plan* p, int32_t which, void* dst, size_t bytes,
                                  void* stream) {
  if (!p || !dst) return fail(PINV_ERR_INVALID, "NULL argument");
  const size_t cs = p->prec == PINV_FP64 ? 16 : 8;
  const void* src = nullptr;
  size_t want = 0;
  if (which == 0) {
    src = p->R;
    want = cs * (size_t)p->N * p->M;
  } else if (which == 1) {
    src = p->Linv;
    want = cs * (size_t)p->G * p->G;
  } else if (which == 2) {
    src = p->gram;
    want = 16 * (size_t)p->G * p->G;
  } else {
    return fail(PINV_ERR_INVALID, "which must be 0, 1 or 2");
  }
  if (!src) return fail(PINV_ERR_INVALID, "buffer not held by this plan");
  if (bytes != want) return fail(PINV_ERR_INVALID, "size mismatch: want " + std::to_string(want));
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(enter_device(p->ctx->device));
  HIPCHK(hipStreamWaitEvent(s, p->ev[4], 0));
  if (which == 0 && p->prec == PINV_BF16X3)   // R is kept split-packed
    HIPCHK(launch_sp_unpack(p->R, p->N, p->M, (float*)dst, s));
  else
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(note_use(p, s));
  return PINV_OK;
}

pinv_status pinv_plan_release(pinv_plan* p) {
  if (!p) return fail(PINV_ERR_INVALID, "plan is NULL");
  pinv_context* c = p->ctx;
  std::lock_guard<std::mutex> g(c->mu);
  const int left = --p->refs;
  if (left <= 0) {
    (void)hipSetDevice(c->device);
    if (p->cached) {
      c->cache.erase(p->key);
      c->lru.erase(p->lru_it);
    }
    c->used -= p->bytes;
    free_plan_memory(p);
    delete p;
  }
  return PINV_OK;
}

pinv_status pinv_cache_trim(pinv_context* c, size_t* freed) {
  if (!c) return fail(PINV_ERR_INVALID, "context is NULL");
  HIPCHK(enter_device(c->device));
  std::lock_guard<std::mutex> g(c->mu);
  const size_t before = c->used;
  make_room(c, (size_t)-1 / 2);
  if (freed) *freed = before - c->used;
  return PINV_OK;
}

pinv_status pinv_context_usage(const pinv_context* c, size_t* used, size_t* budget, int32_t* n) {
  if (!c) return fail(PINV_ERR_INVALID, "context is NULL");
  if (used) *used = c->used;
  if (budget) *budget = c->budget;
  if (n) *n = (int32_t)c->cache.size();
  return PINV_OK;
}

}  // extern "C"
