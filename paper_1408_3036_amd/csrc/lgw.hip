// Host side of the lgw library: context set-up, batched Sternheimer solves,
// chi0 application, Lanczos and projection (C ABI in include/lgw.h).
#include "lgw.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <thread>
#include <exception>
#include <functional>
#include <mutex>
#include <condition_variable>
#include <deque>
#include <vector>

#include "herm_eig.h"
#include "kernels.h"

// lgw_lanczos_project: Lanczos vectors per projection chunk, and the number
// of chunks projected at once (each on its own stream)
#ifndef LGW_PROJECT_CHUNK
#define LGW_PROJECT_CHUNK 8
#endif
#ifndef LGW_PROJECT_WORKERS
#define LGW_PROJECT_WORKERS 2
#endif
// chunk with the multi-shift solver: its recursion is latency-bound for a few
// systems, so it takes more vectors at a time
#ifndef LGW_MAX_GRAPHS
#define LGW_MAX_GRAPHS 64
#endif
#ifndef LGW_PROJECT_CHUNK_MS
#define LGW_PROJECT_CHUNK_MS 16
#endif

using namespace lgw;

// ---- device scratch of the no-allocation entry point (lgw_hpsi_noalloc) ----
// The column intermediates of an H application (and, in single precision, the
// converted operands) live in this fixed array instead of workspace the
// library allocates.  Every device the library runs on holds its own copy
// until the process ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returned on that device: the array's name is a host-side
// stand-in, not a device address.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];


namespace {

struct Fail {
  lgw_status st;
  std::string msg;
};

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      throw Fail{e_ == hipErrorOutOfMemory ? LGW_ENOMEM : LGW_EDEVICE,                     \
                 std::string(#x) + ": " + hipGetErrorString(e_)};                          \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void ensure(size_t bytes) {
    if (bytes <= n && p) return;
    release();
    HIPCHK(hipMalloc(&p, bytes < 256 ? 256 : bytes));
    n = bytes < 256 ? 256 : bytes;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

enum Kind { K_CGLIN = 0, K_CGSQ = 1, K_SQMR = 2 };

}  // namespace

struct lgw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lgw_opts opts{};
  double L[3] = {0, 0, 0};
  int N = 0;
  long n3 = 0;
  double ecut = 0, omega = 0, dV = 0;
  int nv = 0, npw = 0, ncols = 0, hx = 0, hy = 0;
  std::vector<int> m, col_start, col_h, col_pos;
  std::vector<double> kin, eps;
  DevBuf d_col_start, d_col_h, d_col_pos, d_col_of, d_kin, d_Vt, d_Vt32, d_sqrtv, d_tw64, d_tw32, d_psi, d_u, d_Phi,
      d_Phi32;
  // kinetic preconditioner (opts.precond = 1): diagonal scalings of the
  // linear / SQMR systems (|K|^2/2 + shift)^(-1/2) and of the squared form
  // (|K|^2/2 + shift)^(-1), in both precisions, and min/max of each
  DevBuf d_pre64[2], d_pre32[2];
  double pre_ratio[2] = {1.0, 1.0};
  Geom geom{};
  std::map<std::string, DevBuf> ws;
  std::vector<int> st_iters, st_flags, st_sweeps;
  std::vector<double> st_res;
  long long tot_iters = 0, tot_h = 0;
  std::string err;
  std::string scratch_err;   // why this device has no scratch address (lgw_hpsi_noalloc)
  // the self-energy's resolvents of H run without the conduction projector
  // (every proj() is then the identity; set only by a scope guard)
  bool no_proj = false;
  // frequency of the operator eps(z) - 1 of the Lanczos recursion (0: static)
  z64 lz_z{0.0, 0.0};
  bool ones_ready = false;
  // opt-in per-kernel timing with HIP events on the context stream
  bool prof = false;
  struct Timed {
    int kernel;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> pool;
  double kt_ms[2 * LGW_K_FP32] = {0};
  double kt_bytes[2 * LGW_K_FP32] = {0};
  long long kt_launches[2 * LGW_K_FP32] = {0};
  // further contexts on the same system, each with its own stream and copies
  // of the read-only data, created on first use by calls that overlap
  // independent streams of work (lgw_lanczos_project)
  std::vector<std::unique_ptr<lgw_ctx>> twins;
  // pinned staging ring for small host->device uploads on the context stream
  // (h2d_async); a slot is written again only after a stream synchronisation
  static constexpr size_t kPinBytes = size_t(1) << 20;
  char* pin = nullptr;
  size_t pin_off = 0;
  // pinned host buffer for large uploads: its user rewrites it only after a
  // stream synchronisation; growing it synchronises first
  char* pinb = nullptr;
  size_t pinb_n = 0;
  void* pinned(size_t bytes) {
    if (bytes > pinb_n) {
      if (pinb) {
        HIPCHK(hipStreamSynchronize(stream));
        (void)hipHostFree(pinb);
        pinb = nullptr;
        pinb_n = 0;
      }
      HIPCHK(hipHostMalloc((void**)&pinb, bytes, hipHostMallocDefault));
      pinb_n = bytes;
    }
    return pinb;
  }
  // pinned host buffer for device->host readbacks (readback): a copy into
  // pageable memory waits for its own completion, so several of them in a row
  // cost a host round trip each; into pinned memory they queue behind one wait
  char* rdb = nullptr;
  size_t rdb_n = 0;
  char* readback_buf(size_t bytes) {
    if (bytes > rdb_n) {
      if (rdb) {
        HIPCHK(hipStreamSynchronize(stream));
        (void)hipHostFree(rdb);
        rdb = nullptr;
        rdb_n = 0;
      }
      HIPCHK(hipHostMalloc((void**)&rdb, bytes, hipHostMallocDefault));
      rdb_n = bytes;
    }
    return rdb;
  }
  // instantiated graphs of small-batch Krylov chunks, kept across solves and
  // keyed by every pointer and size their capture bakes in; all are dropped
  // before any workspace buffer is reallocated
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
  std::map<std::vector<uintptr_t>, long long> graph_h;   // H applications one replay of a graph performs
  // frequency recycling: per-step copies of the band right-hand sides and the
  // static solutions of the recursion's chi0 applications (off while null)
  z64* keep_b = nullptr;
  z64* keep_f = nullptr;
  int keep_n = 0, keep_cap = 0;
  // iterations the last small-batch solve of each (kind, precision, pass of
  // the refinement) took: the next one runs that many before its first
  // convergence poll
  std::map<std::tuple<int, int, int>, int> it_hint;
  // last contents uploaded by h2d_param per destination: small parameter
  // arrays (system lists, shifts) that no kernel writes are uploaded only when
  // they change.  Cleared whenever a workspace buffer is (re)allocated, so an
  // address never outlives the buffer it was recorded for.
  std::map<const void*, std::vector<char>> up_cache;
  void drop_graphs() {
    if (graphs.empty()) return;
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
    graph_h.clear();
  }

  template <class T>
  T* buf(const std::string& name, size_t count) {
    DevBuf& b = ws[name];
    if (!(count * sizeof(T) <= b.n && b.p)) {
      drop_graphs();
      up_cache.clear();
      b.ensure(count * sizeof(T));
      if (poison_workspace()) HIPCHK(hipMemsetAsync(b.p, 0xFF, b.n, stream));
    }
    return b.as<T>();
  }
  // LGW_POISON=1 (read once per process): every workspace buffer starts
  // filled with 0xFF bytes, a NaN in every floating-point type, so that a
  // kernel reading workspace it never wrote turns its results into NaN
  static bool poison_workspace() {
    static const bool on = [] {
      const char* e = std::getenv("LGW_POISON");
      return e && std::atoi(e) != 0;
    }();
    return on;
  }
  void sync() {
    HIPCHK(hipStreamSynchronize(stream));
    pin_off = 0;
    harvest();
  }
  void check_launch() { HIPCHK(hipGetLastError()); }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    // timing only, read after a stream synchronisation: no system-scope fence
    // (its cache writeback and invalidation would be timed with the kernel)
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
  }
  // bracket one launch: call begin() before it and end() after it.  Only
  // batched launches (more than kTimedMin systems) are timed: small launch-
  // bound batches run as replayed graphs.
  static constexpr int kTimedMin = 64;
  bool time_all = false;   // set by solvers that capture no graphs (multi-shift)
  hipEvent_t begin(int nsys) {
    if (!prof || (nsys <= kTimedMin && !time_all)) return nullptr;
    hipEvent_t a = ev();
    HIPCHK(hipEventRecord(a, stream));
    return a;
  }
  void end(hipEvent_t a, int kernel, double bytes) {
    if (!a) return;
    hipEvent_t b = ev();
    HIPCHK(hipEventRecord(b, stream));
    pending.push_back({kernel, bytes, a, b});
  }
  // after a stream synchronisation: accumulate the elapsed times
  void harvest() {
    for (const Timed& t : pending) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
      kt_ms[t.kernel] += ms;
      kt_bytes[t.kernel] += t.bytes;
      kt_launches[t.kernel] += 1;
      pool.push_back(t.a);
      pool.push_back(t.b);
    }
    pending.clear();
  }
  ~lgw_ctx() {
    for (auto& t : twins) {
      if (!t) continue;   // a twin whose creation failed
      hipStream_t ts = t->own_stream ? t->stream : nullptr;
      t.reset();
      if (ts) (void)hipStreamDestroy(ts);
    }
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graphs();
    if (pin) (void)hipHostFree(pin);
    if (pinb) (void)hipHostFree(pinb);
    if (rdb) (void)hipHostFree(rdb);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    for (const Timed& t : pending) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
  }
};

namespace {

// ---------------------------------------------------------------- helpers
template <class T>
const cplx<T>* tw_of(lgw_ctx* c);
template <> const z64* tw_of<double>(lgw_ctx* c) { return c->d_tw64.as<z64>(); }
template <> const z32* tw_of<float>(lgw_ctx* c) { return c->d_tw32.as<z32>(); }
template <class T>
const T* vt_of(lgw_ctx* c);
template <> const double* vt_of<double>(lgw_ctx* c) { return c->d_Vt.as<double>(); }
template <> const float* vt_of<float>(lgw_ctx* c) { return c->d_Vt32.as<float>(); }
template <class T>
const cplx<T>* phi_of(lgw_ctx* c);
template <> const z64* phi_of<double>(lgw_ctx* c) { return c->d_Phi.as<z64>(); }
template <> const z32* phi_of<float>(lgw_ctx* c) { return c->d_Phi32.as<z32>(); }
// preconditioner scaling for a system kind (null without preconditioning)
template <class T>
const T* pre_of(lgw_ctx* c, int kind);
template <> const double* pre_of<double>(lgw_ctx* c, int kind) {
  return c->opts.precond == 1 ? c->d_pre64[kind == K_CGSQ ? 1 : 0].as<double>() : nullptr;
}
template <> const float* pre_of<float>(lgw_ctx* c, int kind) {
  return c->opts.precond == 1 ? c->d_pre32[kind == K_CGSQ ? 1 : 0].as<float>() : nullptr;
}
double pre_ratio(const lgw_ctx* c, int kind) {
  return c->opts.precond == 1 ? c->pre_ratio[kind == K_CGSQ ? 1 : 0] : 1.0;
}

// host -> device copy that has finished reading the host buffer on return
void h2d(lgw_ctx* c, void* dst, const void* src, size_t bytes) {
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// host -> device copy of a small block, ordered on the context stream without
// waiting for it: the host data are staged in the pinned ring first, so the
// caller may reuse its buffer on return.  The ring is reused from its start
// after a stream synchronisation (every earlier copy has then read its slot).
void h2d_async(lgw_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  if (bytes > lgw_ctx::kPinBytes / 4) {
    h2d(c, dst, src, bytes);
    return;
  }
  if (!c->pin) HIPCHK(hipHostMalloc((void**)&c->pin, lgw_ctx::kPinBytes, hipHostMallocDefault));
  const size_t n = (bytes + 255) & ~size_t(255);
  if (c->pin_off + n > lgw_ctx::kPinBytes) c->sync();
  std::memcpy(c->pin + c->pin_off, src, bytes);
  HIPCHK(hipMemcpyAsync(dst, c->pin + c->pin_off, bytes, hipMemcpyHostToDevice, c->stream));
  c->pin_off += n;
}

// h2d_async for a parameter array that no kernel, copy or fill writes (system
// lists, shifts, index maps): skipped when the destination already holds
// these bytes from an earlier upload.  Every upload to such a destination goes
// through here, so the record is the device contents in stream order.
void h2d_param(lgw_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  auto it = c->up_cache.find(dst);
  const char* p = static_cast<const char*>(src);
  if (it != c->up_cache.end() && it->second.size() == bytes && std::memcmp(it->second.data(), p, bytes) == 0)
    return;
  h2d_async(c, dst, src, bytes);
  c->up_cache[dst].assign(p, p + bytes);
}

// Device arrays to host memory after the work queued on the context stream:
// the copies go through the pinned readback buffer and share one wait.
struct Rd {
  void* dst;
  const void* src;
  size_t bytes;
};
void readback(lgw_ctx* c, std::initializer_list<Rd> parts) {
  size_t tot = 0;
  for (const Rd& r : parts) tot += (r.bytes + 255) & ~size_t(255);
  char* h = c->readback_buf(std::max<size_t>(tot, 256));
  size_t off = 0;
  for (const Rd& r : parts) {
    if (r.bytes) HIPCHK(hipMemcpyAsync(h + off, r.src, r.bytes, hipMemcpyDeviceToHost, c->stream));
    off += (r.bytes + 255) & ~size_t(255);
  }
  c->sync();
  off = 0;
  for (const Rd& r : parts) {
    if (r.bytes) std::memcpy(r.dst, h + off, r.bytes);
    off += (r.bytes + 255) & ~size_t(255);
  }
}

template <class T>
void upload(lgw_ctx* c, DevBuf& b, const std::vector<T>& h) {
  b.ensure(h.size() * sizeof(T));
  h2d(c, b.p, h.data(), h.size() * sizeof(T));
}

// ---- plane-pass autotuner ---------------------------------------------------
// The plane pass has tile variants (threads per workgroup, row layout; the
// same transform, equal to rounding).  The best one per (grid, precision,
// batch-size bucket) is measured once per process, at the first set-up of a
// context with that grid, on a zero-filled column buffer of a representative
// batch, and kept in this table; with LGW_TUNE_CACHE set to a file name the
// measurements are also read from and appended to that file.
struct PlaneTune {
  int best = -1;
  double us[4] = {0, 0, 0, 0};
  int rep = 0;   // systems of the timed batch
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, PlaneTune> g_tune;   // (N, single precision, bucket)
bool g_tune_file_read = false;
constexpr int kTuneBuckets = 4;
constexpr int kTuneRep[kTuneBuckets] = {4, 64, 512, 2048};

int tune_bucket(int nsys) { return nsys <= 8 ? 0 : (nsys <= 64 ? 1 : (nsys <= 512 ? 2 : 3)); }

// the variant used without tuning (opts.autotune = 0, or no entry yet)
int plane_default_variant() { return 0; }

int plane_variant_for(int N, bool f32, int nsys, bool autotune) {
  if (!autotune) return plane_default_variant();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(N, f32 ? 1 : 0, tune_bucket(nsys)));
  return it == g_tune.end() || it->second.best < 0 ? plane_default_variant() : it->second.best;
}

// y = (H - shift) x [+ ecoef E] for nsys systems (device per-system arrays).
// With fed: x = P (fed->pre .* D) is formed by the first transform from the
// direction D and the CG kernels' partial sums, and stored to Xw (X == Xw).
template <class T>
void happly(lgw_ctx* c, const cplx<T>* X, long ldx, cplx<T>* Y, long ldy, const cplx<T>* shift,
            const cplx<T>* E, long lde, const T* ecoef, cplx<T>* Tb, const int* act, int nsys,
            const T* dout = nullptr, const ProjFeed<T>* fed = nullptr, const cplx<T>* D = nullptr,
            cplx<T>* Xw = nullptr, const CgDot<T>* cd = nullptr, const ProjPart<T>* pp = nullptr) {
  const long ldt = (long)c->N * c->ncols;
  const double e = 2.0 * sizeof(T);   // bytes of one complex value
  const double cols = (double)nsys * c->N * c->ncols, sph = (double)nsys * c->npw;
  // the fed transform reads the direction once, as p when it updates it
  if (fed && fed->r && D != fed->p) throw Fail{LGW_EINVAL, "internal: fed direction is not the CG direction"};
  hipEvent_t t0 = c->begin(nsys);
  if (fed)
    launch_zinv_fed<T>(c->geom, tw_of<T>(c), *fed, D, Xw, ldx, Tb, ldt, act, nsys, c->stream);
  else
    launch_zinv<T>(c->geom, tw_of<T>(c), X, ldx, Tb, ldt, T(1), act, nsys, c->stream);
  const int pk = sizeof(T) == 4 ? LGW_K_FP32 : 0;
  c->end(t0, pk + LGW_K_ZINV, e * (sph + cols));
  hipEvent_t t1 = c->begin(nsys);
  launch_plane_hv<T>(c->geom, tw_of<T>(c), Tb, ldt, vt_of<T>(c), act, nsys, c->stream,
                     plane_variant_for(c->N, sizeof(T) == 4, nsys, c->opts.autotune != 0));
  c->end(t1, pk + LGW_K_PLANE_HV, e * 2.0 * cols + sizeof(T) * (double)c->n3);
  hipEvent_t t2 = c->begin(nsys);
  launch_zfwd<T>(c->geom, tw_of<T>(c), Tb, ldt, T(1.0 / (double)c->n3), X, ldx, shift, E, lde, ecoef, Y, ldy,
                 act, nsys, c->stream, dout, cd ? *cd : CgDot<T>{}, pp);
  c->end(t2, pk + LGW_K_ZFWD, e * (cols + (E ? 3.0 : 2.0) * sph));
  c->tot_h += nsys;
}

// Y = dpost .* P (dpre .* X) for the listed systems (X may be Y)
template <class T>
void proj(lgw_ctx* c, const cplx<T>* X, cplx<T>* Y, long ldy, const int* act, int nsys, const T* dpre = nullptr,
          const T* dpost = nullptr) {
  if (c->no_proj) {
    // only the unscaled in-place form occurs there (no preconditioner)
    if (X != Y || dpre || dpost) throw Fail{LGW_EINVAL, "internal: scaled projection without a projector"};
    return;
  }
  const int ks = proj_ksplit<T>(c->npw, nsys);
  cplx<T>* part = c->buf<cplx<T>>(sizeof(T) == 8 ? "proj.part64" : "proj.part32", (size_t)ks * nsys * c->nv);
  hipEvent_t t0 = c->begin(nsys);
  launch_proj_mfma<T>(phi_of<T>(c), c->npw, c->nv, c->npw, X, Y, ldy, act, nsys, part, dpre, dpost, c->stream);
  // Y read once and written once; the valence block is read once per launch
  c->end(t0, (sizeof(T) == 4 ? LGW_K_FP32 : 0) + LGW_K_PROJ,
         2.0 * sizeof(T) * ((3.0 * nsys + c->nv) * c->npw));
}
template <class T>
void proj(lgw_ctx* c, cplx<T>* Y, long ldy, const int* act, int nsys) {
  proj<T>(c, Y, Y, ldy, act, nsys);
}

// Replays a fixed, launch-bound sequence of kernels on the context stream as
// a HIP graph kept by the context, instantiated at the first call with this
// key.  The sequence may enqueue kernels only (no copy, fill, host wait or
// timing event) and must find every workspace buffer it uses already sized;
// key holds every pointer, size and by-value argument the launches bake in
// (tag: which sequence).  The H applications the sequence counts are counted
// again at every replay.  Batches above kTimedMin systems, profiled solvers
// and contexts without graphs launch the sequence directly.  Captures are
// relaxed: other host threads (projection workers, other contexts) may
// allocate, copy or synchronise their own streams while one is open, and the
// captured sequences make no such call themselves.
template <class F>
void replay(lgw_ctx* c, uintptr_t tag, int nsys, std::vector<uintptr_t> key, F&& launch) {
  if (!c->opts.use_graph || c->time_all || nsys > lgw_ctx::kTimedMin) {
    launch();
    return;
  }
  key.insert(key.begin(), {tag, (uintptr_t)nsys});
  auto f = c->graphs.find(key);
  if (f == c->graphs.end()) {
    if (c->graphs.size() >= LGW_MAX_GRAPHS) c->drop_graphs();
    const long long h0 = c->tot_h;
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    try {
      launch();
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(c->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(c->stream, &gr));
    hipGraphExec_t gx = nullptr;
    const hipError_t ie = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIPCHK(ie);
    f = c->graphs.emplace(key, gx).first;
    c->graph_h[key] = c->tot_h - h0;
    c->tot_h = h0;
  }
  HIPCHK(hipGraphLaunch(f->second, c->stream));
  c->tot_h += c->graph_h[key];
}

// Y = A X for the projected operator of the given kind (X is in range(P_c)).
// With a preconditioner scaling S (pre != null): Y = S P A P S X, with P S X
// staged in ptmp (formed by the first transform from the CG kernels' partial
// sums when fed).  In single precision the outer P is left out and S is
// applied by the transform's store: A maps range(P) into itself up to the
// valence orbitals' eigen-residual (1e-13 relative at the workloads), far
// below FP32 rounding, and the FP64 refinement projects every correction.
// cd: the last transform also leaves p^H A p (CgDot).
template <class T>
void apply_op(lgw_ctx* c, int kind, const cplx<T>* X, cplx<T>* Y, cplx<T>* tmp, cplx<T>* Tb, long ld,
              const cplx<T>* shift, const T* w2, const int* act, int nsys, const T* pre = nullptr,
              cplx<T>* ptmp = nullptr, const ProjFeed<T>* fed = nullptr, const CgDot<T>* cd = nullptr) {
  const bool fold = pre && sizeof(T) == 4;
  const cplx<T>* D = nullptr;
  if (pre) {
    // ptmp = P S X; fed: formed by the first transform from the CG kernels' sums
    if (fed) D = X;
    else proj<T>(c, X, ptmp, ld, act, nsys, pre, nullptr);
    X = ptmp;
  }
  if (!D) fed = nullptr;
  const T* dout = fold ? pre : nullptr;
  if (kind == K_CGSQ) {
    happly<T>(c, X, ld, tmp, ld, shift, nullptr, 0, nullptr, Tb, act, nsys, nullptr, fed, D, ptmp);
    proj<T>(c, tmp, ld, act, nsys);
    happly<T>(c, tmp, ld, Y, ld, shift, X, ld, w2, Tb, act, nsys, dout, nullptr, nullptr, nullptr, cd);
  } else {
    happly<T>(c, X, ld, Y, ld, shift, nullptr, 0, nullptr, Tb, act, nsys, dout, fed, D, ptmp, cd);
  }
  if (!fold) proj<T>(c, Y, Y, ld, act, nsys, nullptr, pre);   // Y = S P Y (S = 1 without preconditioner)
}

// Batched Krylov state for one precision.
template <class T>
struct Batch {
  int kind = 0, nsys = 0;
  long ld = 0;
  SolveVecs<T> v{};
  cplx<T>* tmp = nullptr;
  cplx<T>* Tb = nullptr;
  cplx<T>* shift = nullptr;
  T* w2 = nullptr;
  int* act = nullptr;
  size_t poll_off = 0;         // byte offset of v.rr behind v.flag and v.iters
  int nsplit = 1;
  T* split_part = nullptr;
  const T* pre = nullptr;      // preconditioner scaling or null
  cplx<T>* ptmp = nullptr;
  cplx<T>* fpart = nullptr;    // CG with a preconditioner: projector partial sums (ProjFeed)
  T* dot_part = nullptr;       // CG with a preconditioner: p^H A p partials of the last transform (CgDot)
  cplx<T>* cp = nullptr;       // ... and the projector coefficients of the current and the next direction
  cplx<T>* cn = nullptr;
  std::vector<int> h_iters, h_flags;
  Batch() = default;
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  Batch(Batch&& o) noexcept { *this = std::move(o); }
  Batch& operator=(Batch&& o) noexcept {
    kind = o.kind; nsys = o.nsys; ld = o.ld; v = o.v; tmp = o.tmp; Tb = o.Tb; shift = o.shift; w2 = o.w2;
    act = o.act; poll_off = o.poll_off; nsplit = o.nsplit; split_part = o.split_part; pre = o.pre; ptmp = o.ptmp; fpart = o.fpart; dot_part = o.dot_part; cp = o.cp; cn = o.cn;
    h_iters = std::move(o.h_iters); h_flags = std::move(o.h_flags);
    return *this;
  }
};

template <class T>
Batch<T> make_batch(lgw_ctx* c, const char* tag, int kind, int nsys, const std::vector<cplx<T>>& shift,
                    const std::vector<T>& w2) {
  Batch<T> b;
  b.kind = kind;
  b.nsys = nsys;
  b.ld = c->npw;
  const size_t nv = (size_t)nsys * b.ld;
  const std::string t(tag);
  b.v.x = c->buf<cplx<T>>(t + ".x", nv);
  b.v.r = c->buf<cplx<T>>(t + ".r", nv);
  b.v.p = c->buf<cplx<T>>(t + ".p", nv);
  b.v.Ap = c->buf<cplx<T>>(t + ".Ap", nv);
  b.v.d = kind == K_SQMR ? c->buf<cplx<T>>(t + ".d", nv) : nullptr;
  b.tmp = kind == K_CGSQ ? c->buf<cplx<T>>(t + ".tmp", nv) : nullptr;
  b.pre = pre_of<T>(c, kind);
  b.ptmp = b.pre ? c->buf<cplx<T>>(t + ".ptmp", nv) : nullptr;
  b.Tb = c->buf<cplx<T>>(t + ".Tb", (size_t)nsys * c->N * c->ncols);
  b.v.ld = b.ld;
  // flags, iteration counts and residual estimates in one allocation, so a
  // convergence poll reads them back with one copy
  b.poll_off = ((size_t)2 * nsys * sizeof(int) + 15) & ~size_t(15);
  char* poll = c->buf<char>(t + ".poll", b.poll_off + (size_t)nsys * sizeof(T));
  b.v.flag = reinterpret_cast<int*>(poll);
  b.v.iters = b.v.flag + nsys;
  b.v.rr = reinterpret_cast<T*>(poll + b.poll_off);
  b.v.bb = c->buf<T>(t + ".bb", nsys);
  b.v.theta = c->buf<T>(t + ".th", nsys);
  b.v.rho = c->buf<cplx<T>>(t + ".rho", nsys);
  b.shift = c->buf<cplx<T>>(t + ".shift", nsys);
  b.w2 = c->buf<T>(t + ".w2", nsys);
  b.act = c->buf<int>(t + ".act", nsys);
  b.nsplit = std::max(1, std::min(64, c->npw / 1024));
  b.split_part = c->buf<T>(t + ".split", (size_t)2 * std::min(nsys, lgw_ctx::kTimedMin) * b.nsplit);
  b.fpart = b.pre && kind != K_SQMR && c->nv > 0 ? c->buf<cplx<T>>(t + ".fpart", (size_t)b.nsplit * nsys * c->nv)
                                                 : nullptr;
  if (b.fpart) {
    b.dot_part = c->buf<T>(t + ".dots", (size_t)std::min(nsys, lgw_ctx::kTimedMin) * zcol_blocks(c->geom));
    b.cp = c->buf<cplx<T>>(t + ".cp", (size_t)nsys * c->nv);
    b.cn = c->buf<cplx<T>>(t + ".cn", (size_t)nsys * c->nv);
    // ticket counters of the fed CG kernels: zero here, and every ticketed
    // launch leaves them zero
    b.v.cnt = c->buf<int>(t + ".cnt", nsys);
    HIPCHK(hipMemsetAsync(b.v.cnt, 0, nsys * sizeof(int), c->stream));
  }
  {
    size_t cap = 0;
    for (int n = 1; n <= nsys; n += (n < 64 ? 1 : 16)) cap = std::max(cap, (size_t)proj_ksplit<T>(c->npw, n) * n);
    cap = std::max(cap, (size_t)proj_ksplit<T>(c->npw, nsys) * nsys) + 64;
    (void)c->buf<cplx<T>>(sizeof(T) == 8 ? "proj.part64" : "proj.part32", cap * c->nv);
  }
  h2d_param(c, b.shift, shift.data(), nsys * sizeof(cplx<T>));
  std::vector<T> w(w2);
  w.resize(nsys, T(0));
  h2d_param(c, b.w2, w.data(), nsys * sizeof(T));
  b.h_iters.assign(nsys, 0);
  b.h_flags.assign(nsys, 0);
  return b;
}

// Iterate the listed systems of a batch from (re)initialisation with rhs B[bidx]
// until every one is converged, broken down or at max_iter.
// stall > 0: a system whose residual estimate (CG |r|, SQMR tau) has not
// halved within `stall` iterations ends (flag FLAG_MAXIT); used for the
// single-precision inner solves, whose attainable accuracy can sit above the
// inner tolerance for nearly resonant real-axis systems.
template <class T>
void run_batch(lgw_ctx* c, Batch<T>& b, const cplx<T>* B, long ldb, const int* bidx_dev, bool keep_x, double tol,
               const std::vector<int>& start, int stall = 0, int pass = 0) {
  std::vector<int> act(start);
  if (act.empty()) return;
  const int npw = c->npw;
  h2d_param(c, b.act, act.data(), act.size() * sizeof(int));
  // Small preconditioned CG batches: the CG kernels leave the projector's
  // slice sums of the residual (of b at the initialisation), the first
  // transform updates the direction and forms P S p from them (coefficients
  // by C(p) = C(r) + beta C(p_old)), and the last one leaves p^H A p, so a
  // step is the operator application plus one x/r launch.  In single
  // precision that transform stores A p itself (S folded in); in double
  // precision the outer projection follows it, and p^H S P Y = (P S p)^H Y
  // takes the projected input it was given instead.  Decided once per run.
  ProjFeed<T> feed;
  CgDot<T> cdot;
  const bool fed = b.fpart && (int)act.size() <= lgw_ctx::kTimedMin;
  if (fed) {
    feed.Phi = phi_of<T>(c);
    feed.ldphi = c->npw;
    feed.nv = c->nv;
    feed.pre = b.pre;
    feed.part = b.fpart;
    feed.ntot = b.nsys;
    feed.nsplit = b.nsplit;
    feed.r = b.v.r;
    feed.p = b.v.p;
    feed.rr = b.v.rr;
    feed.theta = b.v.theta;
    feed.Cp = b.cp;
    feed.Cn = b.cn;
    cdot.p = sizeof(T) == 4 ? b.v.p : b.ptmp;
    cdot.ldp = b.ld;
    cdot.part = b.dot_part;
    cdot.rr = b.v.rr;
    cdot.theta = b.v.theta;
    cdot.Cp = b.cp;
    cdot.Cn = b.cn;
    cdot.nv = c->nv;
  }
  const int nblk = zcol_blocks(c->geom);
  if (b.kind == K_SQMR)
    launch_sqmr_init<T>(b.v, B, ldb, bidx_dev, npw, (int)act.size(), keep_x, b.act, c->stream);
  else
    launch_cg_init<T>(b.v, B, ldb, bidx_dev, npw, (int)act.size(), keep_x, b.act, c->stream, feed, b.split_part);
  c->check_launch();
  const int check = std::max(1, c->opts.check_every);
  const int maxit = std::max(1, c->opts.max_iter);
  // Small, launch-bound batches replay their chunks as HIP graphs; their first
  // chunk is as long as the last solve of the same kind took (consecutive
  // solves of a recursion need similar counts), then a poll follows every
  // iteration for a while, since a poll costs less than a wasted iteration.
  const bool small = c->opts.use_graph && (int)act.size() <= lgw_ctx::kTimedMin && !c->time_all;
  int& hint = c->it_hint[{b.kind, (int)sizeof(T), std::min(pass, 3)}];
  std::vector<int> flags(b.nsys), iters(b.nsys);
  std::vector<T> est(b.nsys);
  std::vector<char> hpoll(b.poll_off + (size_t)b.nsys * sizeof(T));
  std::vector<double> best(b.nsys, 0.0);
  std::vector<int> best_it(b.nsys, -1);
  int it = 0;
  while (true) {
    // after each chunk: drop converged (or broken-down) systems.  The step
    // kernels skip flagged systems, so the first chunk runs without a poll
    // (initialisation flags only zero right-hand sides).
    if (it > 0) {
      const size_t ni = (size_t)b.nsys * sizeof(int);
      readback(c, {{hpoll.data(), b.v.flag, stall > 0 ? hpoll.size() : 2 * ni}});
      std::memcpy(flags.data(), hpoll.data(), ni);
      std::memcpy(iters.data(), hpoll.data() + ni, ni);
      if (stall > 0) std::memcpy(est.data(), hpoll.data() + b.poll_off, b.nsys * sizeof(T));
      std::vector<int> next, stalled;
      for (int s : act) {
        if (flags[s]) continue;
        if (stall > 0) {
          const double e = b.kind == K_SQMR ? (double)est[s] : std::sqrt((double)est[s]);
          if (best_it[s] < 0 || e < 0.5 * best[s]) {
            best[s] = e;
            best_it[s] = it;
          } else if (it - best_it[s] >= stall) {
            stalled.push_back(s);
            continue;
          }
        }
        next.push_back(s);
      }
      for (int s : stalled) b.h_flags[s] = FLAG_MAXIT;
      const int fl = FLAG_MAXIT;
      for (int s : stalled) h2d_async(c, b.v.flag + s, &fl, sizeof(int));
      act.swap(next);
      if (act.empty() || it >= maxit) break;
      h2d_param(c, b.act, act.data(), act.size() * sizeof(int));
    }
    int chunk = std::min(check, maxit - it);
    if (small && hint > 0) {
      if (it == 0) chunk = std::min(hint, maxit);
      else if (it < hint + check) chunk = std::min(1, maxit - it);
    }
    const int na = (int)act.size();
    auto iterate = [&](int n_it) {
      for (int k = 0; k < n_it; ++k) {
        apply_op<T>(c, b.kind, b.v.p, b.v.Ap, b.tmp, b.Tb, b.ld, b.shift, b.w2, b.act, na, b.pre, b.ptmp,
                    fed ? &feed : nullptr, fed ? &cdot : nullptr);
        hipEvent_t t0 = c->begin(na);
        if (b.kind == K_SQMR) {
          launch_sqmr_step<T>(b.v, npw, T(tol), b.act, na, c->stream);
          // reads q, t, r, d, x (q and r twice), writes r, d, x, q
          c->end(t0, (sizeof(T) == 4 ? LGW_K_FP32 : 0) + LGW_K_SQMR, 2.0 * sizeof(T) * 11.0 * na * npw);
        } else if (na <= lgw_ctx::kTimedMin) {
          // small batch: spread each system over several workgroups
          if (fed)
            launch_cg_step_fed<T>(b.v, npw, T(tol * tol), b.act, na, b.nsplit, b.split_part, b.dot_part, nblk, feed,
                                  c->stream);
          else
            launch_cg_step_split<T>(b.v, npw, T(tol * tol), b.act, na, b.nsplit, b.split_part, c->stream);
        } else {
          launch_cg_step<T>(b.v, npw, T(tol * tol), b.act, na, c->stream);
          // reads p, Ap (twice), x, r (twice), p; writes x, r, p
          c->end(t0, (sizeof(T) == 4 ? LGW_K_FP32 : 0) + LGW_K_CG, 2.0 * sizeof(T) * 10.0 * na * npw);
        }
      }
    };
    // Graphs are instantiated once per key and kept by the context (the active
    // list is read from device memory, so only its length is baked in).  The
    // projector's partial sums are sized for this batch before a capture, so
    // that nothing allocates inside it.
    hipGraphExec_t gx = nullptr;
    if (small && na <= lgw_ctx::kTimedMin) {
      uint64_t tb;
      std::memcpy(&tb, &tol, sizeof tb);
      const std::vector<uintptr_t> key = {
          (uintptr_t)b.kind, sizeof(T), (uintptr_t)na, (uintptr_t)chunk, (uintptr_t)tb, (uintptr_t)b.nsplit,
          (uintptr_t)npw, (uintptr_t)b.ld, (uintptr_t)b.v.x, (uintptr_t)b.v.r, (uintptr_t)b.v.p,
          (uintptr_t)b.v.Ap, (uintptr_t)b.v.d, (uintptr_t)b.v.rr, (uintptr_t)b.v.bb, (uintptr_t)b.v.theta,
          (uintptr_t)b.v.rho, (uintptr_t)b.v.flag, (uintptr_t)b.v.iters, (uintptr_t)b.tmp, (uintptr_t)b.Tb,
          (uintptr_t)b.shift, (uintptr_t)b.w2, (uintptr_t)b.act, (uintptr_t)b.split_part, (uintptr_t)b.pre,
          (uintptr_t)b.ptmp, (uintptr_t)b.fpart, (uintptr_t)fed, (uintptr_t)b.dot_part,
          (uintptr_t)b.cp, (uintptr_t)b.cn, (uintptr_t)b.v.cnt};
      auto f = c->graphs.find(key);
      if (f != c->graphs.end()) {
        gx = f->second;
      } else {
        if (c->graphs.size() >= LGW_MAX_GRAPHS) c->drop_graphs();
        (void)c->buf<cplx<T>>(sizeof(T) == 8 ? "proj.part64" : "proj.part32",
                              (size_t)proj_ksplit<T>(c->npw, na) * na * c->nv);
        const long long h0 = c->tot_h;
        hipGraph_t gr = nullptr;
        // relaxed, as in replay(): other threads' calls stay permitted
        HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        iterate(chunk);
        HIPCHK(hipStreamEndCapture(c->stream, &gr));
        const hipError_t ie = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        HIPCHK(ie);
        c->graphs.emplace(key, gx);
        c->tot_h = h0;
      }
    }
    if (gx) {
      HIPCHK(hipGraphLaunch(gx, c->stream));
      c->tot_h += (long long)chunk * na * (b.kind == K_CGSQ ? 2 : 1);
    } else {
      iterate(chunk);
    }
    c->check_launch();
    it += chunk;
  }
  // the loop ends at a poll, after the last launch: flags and iters are final
  int most = 0;
  for (int s : start) {
    b.h_flags[s] = flags[s] ? flags[s] : FLAG_MAXIT;
    b.h_iters[s] = iters[s];
    most = std::max(most, iters[s]);
  }
  if (small) hint = most;
}

struct SolveOut {
  std::vector<int> iters, flags, sweeps;
  std::vector<double> rel;
};

// Solve A_s x_s = B[bidx[s]] for s < nsys in FP64 (true-residual restarts) or
// mixed precision (FP32 inner Krylov solves inside FP64 iterative refinement).
// X receives the solutions [nsys][npw].
void solve(lgw_ctx* c, int kind, const z64* B, const std::vector<int>& bidx, const std::vector<z64>& shift,
           const std::vector<double>& w2, z64* X, SolveOut& out) {
  const int nsys = (int)bidx.size();
  const int npw = c->npw;
  const double tol = c->opts.tol;
  out.iters.assign(nsys, 0);
  out.flags.assign(nsys, 0);
  out.sweeps.assign(nsys, 0);
  out.rel.assign(nsys, 0.0);
  int* d_bidx = c->buf<int>("sv.bidx", nsys);
  h2d_param(c, d_bidx, bidx.data(), nsys * sizeof(int));
  z64* R = c->buf<z64>("sv.R", (size_t)nsys * npw);
  z64* AX = c->buf<z64>("sv.AX", (size_t)nsys * npw);
  z64* tmp = c->buf<z64>("sv.tmp", kind == K_CGSQ ? (size_t)nsys * npw : 1);
  z64* Tb = c->buf<z64>("sv.Tb", (size_t)nsys * c->N * c->ncols);
  // the slice norms of |b|^2 sit behind the true residuals' slice norms
  // (resp), so the first true-residual readback takes both with one copy
  const int rsn = std::max(1, std::min(64, npw / 1024));
  double* resp = c->buf<double>("sv.resp", (size_t)2 * nsys * rsn);
  double* bbp = resp + (size_t)nsys * rsn;
  z64* d_shift = c->buf<z64>("sv.shift", nsys);
  double* d_w2 = c->buf<double>("sv.w2", nsys);
  int* d_act = c->buf<int>("sv.act", nsys);
  h2d_param(c, d_shift, shift.data(), nsys * sizeof(z64));
  std::vector<double> w2v(w2);
  w2v.resize(nsys, 0.0);
  h2d_param(c, d_w2, w2v.data(), nsys * sizeof(double));
  std::vector<int> all(nsys);
  for (int s = 0; s < nsys; ++s) all[s] = s;
  h2d_param(c, d_act, all.data(), nsys * sizeof(int));
  // |b|^2 per system as slice norms (|B - 0|^2, no AX), read back with the
  // first true residuals: the host needs it only to form relative residuals.
  // The mixed path starts from R = B, which the same pass writes.
  std::vector<double> h_bb(nsys), h_res(nsys);
  bool have_bb = false;
  std::vector<double> h_resp((size_t)2 * nsys * rsn);
  const bool mixed = c->opts.precision != LGW_FP64;
  launch_resid_split<double>(B, npw, d_bidx, nullptr, npw, mixed ? R : nullptr, npw, bbp, rsn, npw, d_act, nsys,
                             c->stream);
  // true residual R = B - A X over the listed systems; returns rel. residuals
  auto true_resid = [&](const std::vector<int>& lst) {
    if (lst.empty()) return;
    h2d_param(c, d_act, lst.data(), lst.size() * sizeof(int));
    const int n = (int)lst.size();
    (void)c->buf<z64>("proj.part64", (size_t)proj_ksplit<double>(npw, n) * n * c->nv);
    replay(c, 1001, n,
           {(uintptr_t)kind, (uintptr_t)X, (uintptr_t)AX, (uintptr_t)tmp, (uintptr_t)Tb, (uintptr_t)d_shift,
            (uintptr_t)d_w2, (uintptr_t)d_act, (uintptr_t)B, (uintptr_t)d_bidx, (uintptr_t)R, (uintptr_t)resp,
            (uintptr_t)npw, (uintptr_t)rsn, (uintptr_t)c->buf<z64>("proj.part64", 1)},
           [&] {
             // the solution lives in the conduction space: remove what rounding
             // (or the single-precision corrections) left in the valence space,
             // which the projected residual below cannot see
             proj<double>(c, X, npw, d_act, n);
             apply_op<double>(c, kind, X, AX, tmp, Tb, npw, d_shift, d_w2, d_act, n);
             // slice norms over several workgroups per system, summed here in order
             launch_resid_split<double>(B, npw, d_bidx, AX, npw, R, npw, resp, rsn, npw, d_act, n, c->stream);
           });
    readback(c, {{h_resp.data(), resp, (size_t)(have_bb ? 1 : 2) * nsys * rsn * sizeof(double)}});
    if (!have_bb)
      for (int s = 0; s < nsys; ++s) {
        double t = 0.0;
        for (int k = 0; k < rsn; ++k) t += h_resp[(size_t)(nsys + s) * rsn + k];
        h_bb[s] = t;
      }
    have_bb = true;
    for (int s : lst) {
      double t = 0.0;
      for (int k = 0; k < rsn; ++k) t += h_resp[(size_t)s * rsn + k];
      h_res[s] = t;
    }
    for (int s : lst) out.rel[s] = h_bb[s] > 0 ? std::sqrt(h_res[s] / h_bb[s]) : 0.0;
  };

  if (c->opts.precision == LGW_FP64) {
    std::vector<z64> sh(shift);
    sh.resize(nsys);
    std::vector<double> w(w2v);
    Batch<double> b = make_batch<double>(c, "b64", kind, nsys, sh, w);
    // With the preconditioner the Krylov solve runs on S P A P S y = S b and
    // x = P S y (the projection happens in true_resid).  CG's tolerance is
    // tightened by min S / max S (a bound on how much the scaled relative
    // residual can understate the true one); SQMR keeps the requested one,
    // since asking it for more than its attainable accuracy costs the iterate
    // (below), and the true residual decides in both cases.
    const double* pre = b.pre;
    const double itol = kind == K_SQMR ? tol : tol * pre_ratio(c, kind);
    const z64* B0 = B;
    const int* bidx0 = d_bidx;
    if (pre) {
      z64* Bs = c->buf<z64>("sv.Bs", (size_t)nsys * npw);
      launch_scale_diag<double>(B, npw, d_bidx, Bs, npw, nullptr, pre, npw, nsys, c->stream);
      B0 = Bs;
      bidx0 = nullptr;
    }
    // X rows from the batch's iterates: all rows, or the rows listed in d_act
    auto x_out = [&](const int* rows, int n) {
      if (pre) launch_scale_diag<double>(b.v.x, npw, rows, X, npw, rows, pre, npw, n, c->stream);
      else if (!rows) HIPCHK(hipMemcpyAsync(X, b.v.x, (size_t)nsys * npw * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
      else launch_rows_out(b.v.x, npw, X, npw, rows, rows, nullptr, npw, n, c->stream);
    };
    // SQMR's recurrences lose accuracy when iterated past the attainable
    // residual (the quasi-residual stagnates and the iterate degrades within a
    // few tens of steps), so a system whose quasi-residual has not halved in
    // 32 iterations stops and is judged by its true residual (restarted from
    // it when above the tolerance).
    const int stall = kind == K_SQMR ? 32 : 0;
    // solve into the batch's x, then refine by restarts on the true residual
    run_batch<double>(c, b, B0, npw, bidx0, false, itol, all, stall);
    x_out(nullptr, nsys);
    std::vector<int> lst = all;
    for (int restart = 0; restart < 3; ++restart) {
      true_resid(lst);
      std::vector<int> bad;
      for (int s : lst)
        if (out.rel[s] > tol && b.h_flags[s] != FLAG_BREAK) bad.push_back(s);
      if (bad.empty()) break;
      // restart from x with the true residual: b.v.x already holds X (or y)
      h2d_param(c, d_act, bad.data(), bad.size() * sizeof(int));
      if (pre) launch_scale_diag<double>(R, npw, d_act, R, npw, d_act, pre, npw, (int)bad.size(), c->stream);
      run_batch<double>(c, b, R, npw, nullptr, true, itol, bad, stall, 1 + restart);
      h2d_param(c, d_act, bad.data(), bad.size() * sizeof(int));
      x_out(d_act, (int)bad.size());
      lst = bad;
    }
    // rows restarted last were not projected by a true-residual pass
    proj<double>(c, X, npw, nullptr, nsys);
    for (int s = 0; s < nsys; ++s) {
      out.iters[s] = b.h_iters[s];
      // the true residual decides; a Krylov breakdown is reported as such
      const int f = b.h_flags[s];
      out.flags[s] = out.rel[s] <= 10 * tol ? FLAG_CONV : (f == FLAG_BREAK ? FLAG_BREAK : FLAG_MAXIT);
      out.sweeps[s] = 1;
    }
  } else {
    // mixed precision: R = B (written with |b|^2 above); X is set by the
    // first sweep's correction, which every system enters
    // every system enters the first sweep (a zero right-hand side gets zero
    // scalings and converges at initialisation)
    for (int s = 0; s < nsys; ++s) out.rel[s] = 1.0;
    std::vector<cplx<float>> sh32(nsys);
    std::vector<float> w32(nsys);
    for (int s = 0; s < nsys; ++s) {
      sh32[s] = cplx<float>{(float)shift[s].x, (float)shift[s].y};
      w32[s] = (float)w2v[s];
    }
    Batch<float> b = make_batch<float>(c, "b32", kind, nsys, sh32, w32);
    double* rs = c->buf<double>("sv.rs", 2 * (size_t)nsys);   // |r| then 1/|r|, uploaded together
    double* irs = rs + nsys;
    z32* R32 = c->buf<z32>("sv.R32", (size_t)nsys * npw);
    std::vector<double> h_rsi(2 * (size_t)nsys);
    const double inner = std::max(c->opts.inner_tol, 1e-7);
    std::vector<int> lst = all;
    std::vector<double> prev(nsys, 1.0);
    bool x_set = false;   // the first sweep's correction assigns X (every system enters it)
    for (int sweep = 0; sweep < std::max(1, c->opts.max_sweeps); ++sweep) {
      std::vector<int> bad;
      for (int s : lst)
        if (out.rel[s] > tol && out.flags[s] == 0) bad.push_back(s);
      if (bad.empty()) break;
      if (sweep == 0 && (int)bad.size() != nsys) {
        HIPCHK(hipMemsetAsync(X, 0, (size_t)nsys * npw * sizeof(z64), c->stream));
        x_set = true;
      }
      for (int s : bad) {
        out.sweeps[s] += 1;
        prev[s] = out.rel[s];
      }
      if (sweep == 0) {
        launch_sqrt_inv(bbp, rsn, rs, irs, nsys, c->stream);   // |b| and 1/|b| from the device's slice norms
      } else {
        for (int s : bad) {
          h_rsi[s] = std::sqrt(h_res[s]);
          h_rsi[nsys + s] = h_rsi[s] > 0 ? 1.0 / h_rsi[s] : 0.0;
        }
        h2d_async(c, rs, h_rsi.data(), h_rsi.size() * sizeof(double));
      }
      h2d_param(c, d_act, bad.data(), bad.size() * sizeof(int));
      launch_scale_cvt(R, npw, R32, npw, irs, d_act, npw, (int)bad.size(), c->stream, b.pre);
      // FP32 SQMR stops on a 32-iteration stagnation window like the FP64 one
      // (an iterate pushed past its attainable accuracy spoils the correction);
      // CG keeps a longer window for slowly converging imaginary-axis systems
      // a sweep needs only the reduction that takes the worst listed system
      // from its FP64 residual to tol (with a factor 4 to spare): the
      // requested inner tolerance or that, whichever is looser, rounded down
      // to a half decade (the tolerance is baked into the replayed graphs,
      // so it takes few distinct values)
      double worst_rel = 0.0;
      for (int s : bad) worst_rel = std::max(worst_rel, out.rel[s]);
      double inner_s = inner;
      if (worst_rel > 0.0 && 0.25 * tol / worst_rel > inner)
        inner_s = std::max(inner, std::pow(10.0, std::floor(2.0 * std::log10(0.25 * tol / worst_rel)) / 2.0));
      run_batch<float>(c, b, R32, npw, nullptr, false, inner_s, bad, kind == K_SQMR ? 32 : 96, sweep);
      h2d_param(c, d_act, bad.data(), bad.size() * sizeof(int));
      launch_cvt_32_64_axpy(b.v.x, X, rs, d_act, npw, npw, (int)bad.size(), c->stream, b.pre, !x_set);
      x_set = true;
      true_resid(bad);
      for (int s : bad) {
        out.iters[s] += b.h_iters[s];
        // an inner FP32 breakdown only ends that sweep; stop refining when the
        // FP64 residual no longer drops by at least a factor of 2
        if (out.rel[s] > tol && out.rel[s] > 0.5 * prev[s]) out.flags[s] = FLAG_MAXIT;
      }
      lst = bad;
    }
    if (!x_set) HIPCHK(hipMemsetAsync(X, 0, (size_t)nsys * npw * sizeof(z64), c->stream));
    // Systems the FP32 sweeps could not bring to the tolerance (an inner
    // solve that stagnates or breaks down on a nearly singular system) get an
    // FP64 correction on their true residual: solve A e = R in FP64 to
    // tol |b| / |R| and x += e; judged by the combined residual.  The
    // correction runs unpreconditioned (the plain projected Krylov solve of
    // Sec. III.A): with the kinetic scaling, rounding in the scaled operator's
    // null space (the scaled valence directions) has broken down such a
    // correction for the highest valence band at 72^3.
    std::vector<int> fail;
    for (int s = 0; s < nsys; ++s)
      if (out.rel[s] > 10 * tol) fail.push_back(s);
    if (!fail.empty()) {
      true_resid(fail);   // R rows of the failing systems, h_res = |R|^2
      const int nf = (int)fail.size();
      z64* Rf = c->buf<z64>("sv.Rfb", (size_t)nf * npw);
      std::vector<int> rows(nf), ident(nf);
      for (int i = 0; i < nf; ++i) {
        rows[i] = fail[i];
        ident[i] = i;
      }
      int* d_rows = c->buf<int>("sv.fbrows", 2 * (size_t)nf);
      h2d_async(c, d_rows, rows.data(), nf * sizeof(int));
      h2d_async(c, d_rows + nf, ident.data(), nf * sizeof(int));
      launch_rows_out(R, npw, Rf, npw, d_rows + nf, d_rows, nullptr, npw, nf, c->stream);   // Rf[i] = R[fail[i]]
      std::vector<z64> fsh(nf);
      std::vector<double> fw2(nf, 0.0);
      double rtol = 0.5;
      for (int i = 0; i < nf; ++i) {
        const int sy = fail[i];
        fsh[i] = shift[sy];
        if (!w2v.empty()) fw2[i] = w2v[sy];
        if (h_res[sy] > 0) rtol = std::min(rtol, tol * std::sqrt(h_bb[sy] / h_res[sy]));
      }
      rtol = std::max(rtol, tol);
      z64* Ef = c->buf<z64>("sv.Efb", (size_t)nf * npw);
      SolveOut so;
      {
        struct OptScope {
          lgw_ctx* c;
          lgw_opts saved;
          ~OptScope() {
            c->drop_graphs();
            c->opts = saved;
          }
        } scope{c, c->opts};
        c->opts.precision = LGW_FP64;
        c->opts.precond = 0;
        c->opts.tol = rtol;
        c->drop_graphs();   // graphs captured with the preconditioner bake in its buffers
        solve(c, kind, Rf, ident, fsh, fw2, Ef, so);
      }
      // the inner call reused this call's workspace: X and the host copies stand
      for (int i = 0; i < nf; ++i) {
        z64* xr = X + (size_t)fail[i] * npw;
        launch_add(xr, xr, Ef + (size_t)i * npw, npw, c->stream);
        const int sy = fail[i];
        out.rel[sy] = h_bb[sy] > 0 ? so.rel[i] * std::sqrt(h_res[sy] / h_bb[sy]) : 0.0;
        out.iters[sy] += so.iters[i];
        out.sweeps[sy] += 1;
      }
      c->check_launch();
    }
    for (int s = 0; s < nsys; ++s) out.flags[s] = out.rel[s] <= 10 * tol ? FLAG_CONV : FLAG_MAXIT;
  }
  for (int s = 0; s < nsys; ++s) c->tot_iters += out.iters[s];
}

// ---------------------------------------------------------------- multi-shift
// Solution of (T - tau) y = r0 e_1 for the real symmetric tridiagonal T
// (diagonal al[0..k), off-diagonal be[0..k-1)), Gaussian elimination with
// partial pivoting (one extra super-diagonal appears).
void tri_shift_solve(const double* al, const double* be, int k, z64 tau, double r0, z64* y) {
  std::vector<z64> d(k), du(k > 1 ? k - 1 : 1), dl(k > 1 ? k - 1 : 1), du2(k > 2 ? k - 2 : 1), b(k, z64{0, 0});
  for (int i = 0; i < k; ++i) d[i] = z64{al[i] - tau.x, -tau.y};
  for (int i = 0; i + 1 < k; ++i) du[i] = dl[i] = z64{be[i], 0.0};
  b[0] = z64{r0, 0.0};
  auto div = [](z64 a, z64 c) {
    const double den = c.x * c.x + c.y * c.y;
    return z64{(a.x * c.x + a.y * c.y) / den, (a.y * c.x - a.x * c.y) / den};
  };
  auto mag = [](z64 a) { return std::abs(a.x) + std::abs(a.y); };
  for (int i = 0; i + 1 < k; ++i) {
    if (mag(d[i]) >= mag(dl[i])) {
      const z64 f = div(dl[i], d[i]);
      d[i + 1] = d[i + 1] - f * du[i];
      b[i + 1] = b[i + 1] - f * b[i];
      if (i + 2 < k) du2[i] = z64{0, 0};
    } else {
      const z64 f = div(d[i], dl[i]);
      d[i] = dl[i];
      const z64 t = d[i + 1];
      d[i + 1] = du[i] - f * t;
      if (i + 2 < k) {
        du2[i] = du[i + 1];
        du[i + 1] = z64{0, 0} - f * du2[i];
      }
      du[i] = t;
      const z64 bt = b[i];
      b[i] = b[i + 1];
      b[i + 1] = bt - f * b[i + 1];
    }
  }
  y[k - 1] = div(b[k - 1], d[k - 1]);
  if (k > 1) y[k - 2] = div(b[k - 2] - du[k - 2] * y[k - 1], d[k - 2]);
  for (int i = k - 3; i >= 0; --i) y[i] = div(b[i] - du[i] * y[i + 1] - du2[i] * y[i + 2], d[i]);
}

lgw_status worst(lgw_status a, lgw_status b);

// Every frequency of a chi0 call from one Lanczos recursion per system: with
// A_p = P (H - e_v) P and b_p = B0[p] (p = j * nv + v),
//   F[z][p] = (A_p - z)^-1 b_p + (A_p + z)^-1 b_p       (2 A_p^-1 b_p at z = 0),
// the sum the shifted pair and the squared form both produce.  The Krylov
// space of A_p - tau is that of A_p, so plain Lanczos (A Q = Q T + beta q e^T)
// gives every shift as x_tau = Q y_tau, (T - tau) y_tau = |b| e_1, with
// residual |b - (A - tau) x_tau| = beta_k |e_k^T y_tau|.  A system stops when
// that bound is below tol for all its shifts; every x_tau is then checked by
// its true residual, and any above tol is corrected by the shifted solver.
// base (or null): the shift of system p is base[p] instead of e_v.
lgw_status multishift(lgw_ctx* c, const z64* B0, int nb, int nz, const lgw_c128* zl, z64* F,
                      const double* base = nullptr) {
  const int npw = c->npw, nv = c->nv;
  const long ldt = (long)c->N * c->ncols;
  const double tol = c->opts.tol;
  std::vector<z64> tau;
  std::vector<int> tpos(nz), tneg(nz);
  for (int k = 0; k < nz; ++k) {
    const z64 z{zl[k].re, zl[k].im};
    if (z.x == 0.0 && z.y == 0.0) {
      tpos[k] = tneg[k] = (int)tau.size();
      tau.push_back(z64{0, 0});
    } else {
      tpos[k] = (int)tau.size();
      tau.push_back(z);
      tneg[k] = (int)tau.size();
      tau.push_back(z64{-z.x, -z.y});
    }
  }
  const int ntau = (int)tau.size();
  const int kcap = std::max(16, std::min(c->opts.max_iter, 384));
  // its launches are timed whatever their size (no graph capture here)
  struct TimeAll {
    lgw_ctx* c;
    bool old;
    ~TimeAll() { c->time_all = old; }
  } time_all_guard{c, c->time_all};
  c->time_all = true;
  const int check = std::max(1, c->opts.check_every);
  const double per = 16.0 * npw * (2.0 * (kcap + 1) + 3.0 * ntau) + 16.0 * ldt * (1.0 + ntau);
  const double budget = std::max(0.25, c->opts.mem_budget_gb) * 1e9;
  const int cap = std::max(1, (int)std::min((double)nb, budget / per));
  lgw_status st = LGW_OK;
  for (int s0 = 0; s0 < nb; s0 += cap) {
    const int n = std::min(cap, nb - s0);
    const long ldq = (long)(kcap + 1) * npw;
    z64* Q = c->buf<z64>("ms.Q", (size_t)n * ldq);
    z64* AQ = c->buf<z64>("ms.AQ", (size_t)n * ldq);   // A q_j as applied, for the true residuals
    double* mscratch = c->buf<double>("ms.scr", ms_step_scratch(n));
    // up to 8 bands: the projector folded into the steps (ProjPart)
    const bool fold = !c->no_proj && nv <= 8;
    const int nblk = zcol_blocks(c->geom);
    ProjPart<double> pp;
    if (fold) {
      pp.Phi = c->d_Phi.as<z64>();
      pp.ldphi = npw;
      pp.nv = nv;
      pp.part = c->buf<z64>("ms.ppart", (size_t)n * nblk * 8);
    }
    double* alpha = c->buf<double>("ms.al", (size_t)n * kcap);
    double* beta = c->buf<double>("ms.be", (size_t)n * kcap);
    double* nrm = c->buf<double>("ms.nrm", n);
    int* d_idx = c->buf<int>("ms.idx", n);
    int* d_act = c->buf<int>("ms.act", n);
    z64* d_sh = c->buf<z64>("ms.sh", n);
    z64* Tb = c->buf<z64>("ms.Tb", (size_t)n * ldt);
    std::vector<int> idx(n);
    std::vector<z64> sh(n);
    for (int s = 0; s < n; ++s) {
      idx[s] = s0 + s;
      sh[s] = z64{base ? base[s0 + s] : c->eps[(s0 + s) % nv], 0.0};
    }
    h2d_param(c, d_idx, idx.data(), n * sizeof(int));
    h2d_async(c, d_sh, sh.data(), n * sizeof(z64));
    launch_ms_init(B0, npw, d_idx, npw, Q, ldq, nrm, n, c->stream);
    c->check_launch();
    std::vector<double> hn(n), ha((size_t)n * kcap), hb((size_t)n * kcap);
    HIPCHK(hipMemcpyAsync(hn.data(), nrm, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    std::vector<int> act, kd(n, 0);
    for (int s = 0; s < n; ++s)
      if (hn[s] > 0.0) act.push_back(s);
    // Residual estimates |b - (A - tau) x_j| = |b| |e_j^T (T_j - tau)^-1 e_1| beta_j
    // = |b| prod_i beta_i / |det(T_j - tau)|, extended step by step through the
    // ratios u_i = det(T_i - tau) / det(T_{i-1} - tau) (continued fraction
    // u_{i+1} = alpha_i - tau - beta_{i-1}^2 / u_i); rho = prod beta / prod |u|.
    std::vector<z64> cu((size_t)n * ntau, z64{0, 0});
    std::vector<double> crho((size_t)n * ntau, 1.0);
    std::vector<int> cj(n, 0);
    int j = 0;
    while (!act.empty() && j < kcap) {
      h2d_param(c, d_act, act.data(), act.size() * sizeof(int));
      const int na = (int)act.size();
      const int steps = std::min(check, kcap - j);
      for (int t = 0; t < steps; ++t, ++j) {
        if (fold) {
          // the projection of A q_j folded into the transform (coefficients)
          // and the recursion step (the update): no projector launches
          happly<double>(c, Q + (size_t)j * npw, ldq, AQ + (size_t)j * npw, ldq, d_sh, nullptr, 0, nullptr, Tb, d_act,
                         na, nullptr, nullptr, nullptr, nullptr, nullptr, &pp);
          launch_ms_step(Q, AQ, ldq, npw, j, d_act, na, alpha, beta, kcap, mscratch, c->stream, &pp, nblk);
        } else {
          apply_op<double>(c, K_CGLIN, Q + (size_t)j * npw, AQ + (size_t)j * npw, nullptr, Tb, ldq, d_sh,
                           nullptr, d_act, na);
          launch_ms_step(Q, AQ, ldq, npw, j, d_act, na, alpha, beta, kcap, mscratch, c->stream);
        }
      }
      c->check_launch();
      readback(c, {{ha.data(), alpha, ha.size() * sizeof(double)}, {hb.data(), beta, hb.size() * sizeof(double)}});
      std::vector<int> next;
      for (int s : act) {
        const double* al = ha.data() + (size_t)s * kcap;
        const double* be = hb.data() + (size_t)s * kcap;
        double amax = 0.0;
        for (int i = 0; i < j; ++i) amax = std::max(amax, std::abs(al[i]));
        bool done = be[j - 1] <= 1e-14 * amax;   // invariant subspace: exact for every shift
        double worst_rho = 0.0;
        for (int t = 0; t < ntau; ++t) {
          z64& u = cu[(size_t)s * ntau + t];
          double& rho = crho[(size_t)s * ntau + t];
          for (int i = cj[s]; i < j; ++i) {
            const z64 d{al[i] - tau[t].x, -tau[t].y};
            if (i == 0) {
              u = d;
            } else {
              const double den = norm2(u);
              const double b2 = be[i - 1] * be[i - 1];
              u = z64{d.x - b2 * u.x / den, d.y + b2 * u.y / den};   // d - b2 / u
            }
            // a (nearly) singular leading block, possible for real shifts only,
            // gives a huge estimate at that step and recovers at the next
            double au = std::sqrt(norm2(u));
            if (!(au >= 1e-150)) {
              u = z64{1e-150, 0.0};
              au = 1e-150;
            }
            rho *= be[i] / au;
          }
          worst_rho = std::max(worst_rho, rho);
        }
        cj[s] = j;
        done = done || worst_rho <= tol;
        if (done) kd[s] = j;
        else next.push_back(s);
      }
      act.swap(next);
    }
    for (int s : act) kd[s] = j;   // not converged in kcap steps: the check below decides
    c->tot_iters += [&] { long long t = 0; for (int s = 0; s < n; ++s) t += kd[s]; return t; }();
    // x_tau = Q y_tau for every system and shift: the tridiagonal solves on
    // host threads into pinned Y[s][j][t] (shifts padded to ntp), then one
    // combine on the matrix cores
    const int kmax = std::max(1, *std::max_element(kd.begin(), kd.end()));
    const int ntp = (ntau + 15) / 16 * 16;
    const size_t ybytes = (size_t)n * kmax * ntp * sizeof(z64);
    z64* hy = static_cast<z64*>(c->pinned(ybytes));   // the stream is idle here (synchronised at the last poll)
    {
      auto fill = [&](int sb, int se) {
        std::vector<z64> yv(kmax);
        for (int s = sb; s < se; ++s) {
          const double* al = ha.data() + (size_t)s * kcap;
          const double* be = hb.data() + (size_t)s * kcap;
          z64* ys = hy + (size_t)s * kmax * ntp;
          for (int t = 0; t < ntp; ++t) {
            if (t < ntau && kd[s] > 0) tri_shift_solve(al, be, kd[s], tau[t], hn[s], yv.data());
            for (int jj = 0; jj < kmax; ++jj) ys[(size_t)jj * ntp + t] = (t < ntau && jj < kd[s]) ? yv[jj] : z64{0, 0};
          }
        }
      };
      const int nth = std::max(1, std::min({8, n, (int)std::thread::hardware_concurrency() / 2}));
      std::vector<std::thread> th;
      for (int q = 1; q < nth; ++q) th.emplace_back(fill, (int)((long)n * q / nth), (int)((long)n * (q + 1) / nth));
      fill(0, n / nth);
      for (auto& x : th) x.join();
    }
    z64* Yd = c->buf<z64>("ms.Y", ybytes / sizeof(z64));
    int* d_kd = c->buf<int>("ms.kd", n);
    HIPCHK(hipMemcpyAsync(Yd, hy, ybytes, hipMemcpyHostToDevice, c->stream));
    h2d_async(c, d_kd, kd.data(), n * sizeof(int));
    const int nr = n * ntau;
    z64* X = c->buf<z64>("ms.X", (size_t)nr * npw);
    // x_tau and its true residual b - (A - tau) x_tau = b - (A Q) y_tau + tau Q y_tau
    // from the products A q_j the recursion applied (linearity of A; rounding
    // of the same order as applying A to x_tau), for every (system, shift)
    std::vector<z64> taup(ntp, z64{0, 0});
    std::copy(tau.begin(), tau.end(), taup.begin());
    z64* d_tau = c->buf<z64>("ms.tau", ntp);
    h2d_async(c, d_tau, taup.data(), ntp * sizeof(z64));
    double* rpart = c->buf<double>("ms.rpart", (size_t)n * ntp * ms_res_tiles(npw));
    double* res = c->buf<double>("ms.res", (size_t)n * ntp);
    launch_ms_combine_res(Q, AQ, ldq, npw, d_kd, Yd, kmax, ntp, ntau, d_tau, B0, npw, d_idx, X, rpart, res, n,
                          c->stream);
    proj<double>(c, X, npw, nullptr, nr);
    std::vector<double> hres((size_t)n * ntp);
    HIPCHK(hipMemcpyAsync(hres.data(), res, hres.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    std::vector<double> hr(nr), rel(nr, 0.0);
    std::vector<int> fit(nr, 0), flg(nr, FLAG_CONV), bad;
    for (int r = 0; r < nr; ++r) {
      hr[r] = hres[(size_t)(r / ntau) * ntp + r % ntau];
      const double nb2 = hn[r / ntau];
      rel[r] = nb2 > 0.0 ? std::sqrt(hr[r]) / nb2 : 0.0;
      if (rel[r] > tol) bad.push_back(r);
    }
    // shifts of row r = s * ntau + t: e_v + tau_t (the systems (H - e_v - tau) x = b)
    std::vector<z64> rs(nr);
    for (int s = 0; s < n; ++s)
      for (int t = 0; t < ntau; ++t) rs[(size_t)s * ntau + t] = z64{sh[s].x + tau[t].x, tau[t].y};
    z64* R = nullptr;
    if (!bad.empty()) {
      // the residual vectors of the rows to correct, from an explicit H application
      std::vector<int> rb(nr);
      for (int r = 0; r < nr; ++r) rb[r] = s0 + r / ntau;
      int* d_rb = c->buf<int>("ms.rb", nr);
      z64* d_rs = c->buf<z64>("ms.rs", nr);
      int* d_bad = c->buf<int>("ms.bad", bad.size());
      h2d_async(c, d_rb, rb.data(), nr * sizeof(int));
      h2d_async(c, d_rs, rs.data(), nr * sizeof(z64));
      h2d_async(c, d_bad, bad.data(), bad.size() * sizeof(int));
      z64* AX = c->buf<z64>("ms.AX", (size_t)nr * npw);
      R = c->buf<z64>("ms.R", (size_t)nr * npw);
      z64* TbV = c->buf<z64>("ms.TbV", (size_t)nr * ldt);
      double* rres = c->buf<double>("ms.rres", nr);
      apply_op<double>(c, K_SQMR, X, AX, nullptr, TbV, npw, d_rs, nullptr, d_bad, (int)bad.size());
      launch_resid<double>(B0, npw, d_rb, AX, npw, R, npw, rres, npw, d_bad, (int)bad.size(), c->stream);
      std::vector<double> hrr(nr);
      HIPCHK(hipMemcpyAsync(hrr.data(), rres, nr * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      for (int r : bad) hr[r] = hrr[r];
    }
    if (!bad.empty()) {
      // correction on the true residual with the shifted solver (SQMR)
      std::vector<z64> bsh(bad.size());
      for (size_t i = 0; i < bad.size(); ++i) bsh[i] = rs[bad[i]];
      // The correction needs tol |b| / |R| relative to its own right-hand
      // side: solve at the tightest of those (all are at least tol) and judge
      // each system by its combined residual relative to |b|.
      double rtol = 0.5;
      for (int r : bad) rtol = std::min(rtol, tol * hn[r / ntau] / std::sqrt(hr[r]));
      rtol = std::max(rtol, tol);
      z64* E = c->buf<z64>("ms.E", bad.size() * (size_t)npw);
      SolveOut so;
      const double tol_saved = c->opts.tol;
      c->opts.tol = rtol;
      c->time_all = false;   // the shifted solver may capture graphs
      try {
        solve(c, K_SQMR, R, bad, bsh, {}, E, so);
      } catch (...) {
        c->opts.tol = tol_saved;
        throw;
      }
      c->opts.tol = tol_saved;
      c->time_all = true;
      for (size_t i = 0; i < bad.size(); ++i) {
        z64* xr = X + (size_t)bad[i] * npw;
        launch_add(xr, xr, E + i * (size_t)npw, npw, c->stream);
        const int r = bad[i];
        rel[r] = so.rel[i] * std::sqrt(hr[r]) / hn[r / ntau];
        fit[r] = so.iters[i];
        flg[r] = rel[r] <= 10 * tol ? FLAG_CONV : (so.flags[i] == FLAG_BREAK ? FLAG_BREAK : FLAG_MAXIT);
      }
      c->check_launch();
    }
    // F[z][p] = x(+z) + x(-z)
    std::vector<int> oi(3 * (size_t)n * nz);
    const int np = n * nz;
    for (int s = 0; s < n; ++s)
      for (int k = 0; k < nz; ++k) {
        const int q = s * nz + k;
        oi[q] = k * nb + s0 + s;
        oi[np + q] = s * ntau + tpos[k];
        oi[2 * np + q] = s * ntau + tneg[k];
      }
    int* d_oi = c->buf<int>("ms.oi", oi.size());
    h2d_async(c, d_oi, oi.data(), oi.size() * sizeof(int));
    launch_rows_out(X, npw, F, npw, d_oi, d_oi + np, d_oi + 2 * np, npw, np, c->stream);
    c->check_launch();
    c->sync();
    for (int s = 0; s < n; ++s)
      for (int t = 0; t < ntau; ++t) {
        const int r = s * ntau + t;
        c->st_iters.push_back(kd[s] + fit[r]);
        c->st_flags.push_back(flg[r]);
        c->st_sweeps.push_back(1);
        c->st_res.push_back(rel[r]);
        if (flg[r] == FLAG_BREAK) st = worst(st, LGW_EBREAKDOWN);
        else if (flg[r] != FLAG_CONV) st = worst(st, LGW_ENOCONV);
      }
  }
  return st;
}

// ---------------------------------------------------------------- v^1/2
// in-place on zxy grid vectors: G <- scale_sign * v^1/2 G
// G = v^1/2 src (src null: in place; otherwise src is left unchanged)
void vhalf_inplace(lgw_ctx* c, z64* G, int n, double sign, const z64* src = nullptr) {
  launch_plane_full<double>(c->N, c->d_tw64.as<z64>(), G, c->n3, n, -1, c->stream, src);
  launch_zfull_mul<double>(c->N, c->d_tw64.as<z64>(), G, c->n3, c->d_sqrtv.as<double>(), sign / (double)c->n3, n,
                           c->stream);
  launch_plane_full<double>(c->N, c->d_tw64.as<z64>(), G, c->n3, n, +1, c->stream);
}

// ---------------------------------------------------------------- chi0
// out[z][j] = chi0(z) X[j] on zxy grid vectors.
lgw_status chi0_internal(lgw_ctx* c, int nrhs, const z64* X, int nz, const lgw_c128* zl, z64* out, long ldz) {
  const int nv = c->nv, npw = c->npw;
  const long n3 = c->n3;
  const int nb = nrhs * nv;                 // (j, v) pairs, index j*nv + v
  const long ldt = (long)c->N * c->ncols;
  c->st_iters.clear();
  c->st_flags.clear();
  c->st_sweeps.clear();
  c->st_res.clear();
  // right-hand sides b_{j,v} = P_c Gather(conj(psi_v) x_j)
  z64* Tb = c->buf<z64>("c.Tb", (size_t)nb * ldt);
  z64* B0 = c->buf<z64>("c.B0", (size_t)nb * npw);     // b
  z64* B2 = c->buf<z64>("c.B2", (size_t)nb * npw);     // 2 b
  (void)c->buf<z64>("proj.part64", (size_t)proj_ksplit<double>(npw, nb) * nb * nv);
  replay(c, 1002, nb,
         {(uintptr_t)X, (uintptr_t)nrhs, (uintptr_t)Tb, (uintptr_t)B0, (uintptr_t)B2,
          (uintptr_t)c->buf<z64>("proj.part64", 1)},
         [&] {
           launch_plane_pair_fwd<double>(c->geom, c->d_tw64.as<z64>(), c->d_u.as<z64>(), nv, X, n3, nrhs, Tb, ldt,
                                         c->stream);
           launch_zfwd<double>(c->geom, c->d_tw64.as<z64>(), Tb, ldt, std::sqrt(c->omega) / (double)n3, nullptr, 0,
                               nullptr, nullptr, 0, nullptr, B0, npw, nullptr, nb, c->stream);
           proj<double>(c, B0, npw, nullptr, nb);
           launch_add(B2, B0, B0, (long)nb * npw, c->stream);
         });
  if (c->opts.model == 1) {
    // model operator (H -> T): f[z][p] = P ((T - e_v - z)^-1 + (T - e_v + z)^-1) b_p
    z64* F = c->buf<z64>("c.F", (size_t)nz * nb * npw);
    double* d_eps = c->buf<double>("c.eps", nv);
    z64* d_z = c->buf<z64>("c.z", nz);
    std::vector<z64> hz(nz);
    for (int k = 0; k < nz; ++k) hz[k] = z64{zl[k].re, zl[k].im};
    h2d_async(c, d_eps, c->eps.data(), nv * sizeof(double));
    h2d_async(c, d_z, hz.data(), nz * sizeof(z64));
    launch_model_div(B0, npw, c->d_kin.as<double>(), d_eps, nv, nb, d_z, nz, F, c->stream);
    proj<double>(c, F, npw, nullptr, nz * nb);
    c->st_iters.assign((size_t)nz * nb, 0);
    c->st_flags.assign((size_t)nz * nb, FLAG_CONV);
    c->st_sweeps.assign((size_t)nz * nb, 0);
    c->st_res.assign((size_t)nz * nb, 0.0);
    for (int k = 0; k < nz; ++k) {
      launch_zinv<double>(c->geom, c->d_tw64.as<z64>(), F + (size_t)k * nb * npw, npw, Tb, ldt, 1.0, nullptr, nb,
                          c->stream);
      launch_plane_acc<double>(c->geom, c->d_tw64.as<z64>(), Tb, ldt, c->d_psi.as<z64>(), nv,
                               out + (size_t)k * ldz, n3, -2.0 / std::sqrt(c->omega), nrhs, false, c->stream);
    }
    c->check_launch();
    return LGW_OK;
  }
  // all frequencies from one Lanczos recursion per system when there are at
  // least three shifts (one frequency is left to the preconditioned solvers)
  int nshift = 0;
  for (int k = 0; k < nz; ++k) nshift += (zl[k].re == 0.0 && zl[k].im == 0.0) ? 1 : 2;
  const bool ms = c->opts.multishift == 1 && nshift >= 3;
  // imaginary frequencies in the squared form need 2 P (H - e_v) b
  const bool squared = c->opts.imag_form == 0 && !ms;
  bool any_imag = false;
  for (int k = 0; k < nz; ++k)
    if (squared && zl[k].re == 0.0 && zl[k].im != 0.0) any_imag = true;
  z64* B1 = nullptr;   // 2 P (H - e_v) b
  std::vector<z64> eps_shift(nb);
  for (int p = 0; p < nb; ++p) eps_shift[p] = z64{c->eps[p % nv], 0.0};
  if (any_imag) {
    B1 = c->buf<z64>("c.B1", (size_t)nb * npw);
    z64* d_sh = c->buf<z64>("c.sh", nb);
    h2d_async(c, d_sh, eps_shift.data(), nb * sizeof(z64));
    happly<double>(c, B2, npw, B1, npw, d_sh, nullptr, 0, nullptr, Tb, nullptr, nb);
    proj<double>(c, B1, npw, nullptr, nb);
  }
  c->check_launch();
  // solutions f[z][j*nv+v]
  z64* F = c->buf<z64>("c.F", (size_t)nz * nb * npw);
  // systems by kind
  struct Sys { int z, p, sign; };
  std::vector<Sys> lin, sq, qm;
  for (int k = 0; k < nz; ++k) {
    for (int p = 0; p < nb; ++p) {
      if (zl[k].re == 0.0 && zl[k].im == 0.0) lin.push_back({k, p, 0});
      else if (zl[k].re == 0.0 && squared) sq.push_back({k, p, 0});
      else {
        qm.push_back({k, p, -1});
        qm.push_back({k, p, +1});
      }
    }
  }
  // per-system workspace in bytes (FP64 vectors, FP32 state in mixed mode)
  const double vec = 16.0 * npw, tb = 16.0 * ldt;
  const double per = 10 * vec + 2 * tb;
  const double budget = std::max(0.25, c->opts.mem_budget_gb) * 1e9;
  const int cap = std::max(2, (int)std::min(1e6, budget / per)) & ~1;
  lgw_status st = LGW_OK;
  auto run_kind = [&](int kind, const std::vector<Sys>& sy) {
    for (size_t s0 = 0; s0 < sy.size(); s0 += cap) {
      const int n = (int)std::min<size_t>(cap, sy.size() - s0);
      std::vector<int> bidx(n);
      std::vector<z64> sh(n);
      std::vector<double> w2(n, 0.0);
      for (int i = 0; i < n; ++i) {
        const Sys& q = sy[s0 + i];
        const double e = c->eps[q.p % nv];
        bidx[i] = q.p;
        if (kind == K_SQMR) sh[i] = z64{e + q.sign * zl[q.z].re, q.sign * zl[q.z].im};
        else sh[i] = z64{e, 0.0};
        if (kind == K_CGSQ) w2[i] = zl[q.z].im * zl[q.z].im;
      }
      const z64* B = kind == K_CGLIN ? B2 : (kind == K_CGSQ ? B1 : B0);
      z64* Xs = c->buf<z64>("c.Xs", (size_t)n * npw);
      SolveOut so;
      solve(c, kind, B, bidx, sh, w2, Xs, so);
      // write f into F
      std::vector<int> didx, a, b;
      if (kind == K_SQMR) {
        for (int i = 0; i < n; i += 2) {
          didx.push_back(sy[s0 + i].z * nb + sy[s0 + i].p);
          a.push_back(i);
          b.push_back(i + 1);
        }
      } else {
        for (int i = 0; i < n; ++i) {
          didx.push_back(sy[s0 + i].z * nb + sy[s0 + i].p);
          a.push_back(i);
        }
      }
      const int np = (int)didx.size();
      int* d_idx = c->buf<int>("c.idx", 3 * (size_t)np);
      std::vector<int> all(didx);
      all.insert(all.end(), a.begin(), a.end());
      all.insert(all.end(), b.begin(), b.end());
      h2d_param(c, d_idx, all.data(), all.size() * sizeof(int));
      launch_rows_out(Xs, npw, F, npw, d_idx, d_idx + np, kind == K_SQMR ? d_idx + 2 * np : nullptr, npw, np,
                      c->stream);
      for (int i = 0; i < n; ++i) {
        c->st_iters.push_back(so.iters[i]);
        c->st_flags.push_back(so.flags[i]);
        c->st_sweeps.push_back(so.sweeps[i]);
        c->st_res.push_back(so.rel[i]);
        if (so.flags[i] == FLAG_BREAK) st = LGW_EBREAKDOWN;
        else if (so.flags[i] != FLAG_CONV && st == LGW_OK) st = LGW_ENOCONV;
      }
    }
  };
  if (ms) {
    st = multishift(c, B0, nb, nz, zl, F);
  } else {
    run_kind(K_CGLIN, lin);
    run_kind(K_CGSQ, sq);
    run_kind(K_SQMR, qm);
  }
  if (c->keep_b && nz == 1 && zl[0].re == 0.0 && zl[0].im == 0.0 && c->keep_n + nrhs <= c->keep_cap) {
    const size_t off = (size_t)c->keep_n * nb * npw, bytes = (size_t)nb * npw * sizeof(z64);
    HIPCHK(hipMemcpyAsync(c->keep_b + off, B0, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->keep_f + off, F, bytes, hipMemcpyDeviceToDevice, c->stream));
    c->keep_n += nrhs;
  }
  // dn_j(z) = -2 sum_v psi_v Scatter(f_{j,v}(z))
  for (int k = 0; k < nz; ++k) {
    launch_zinv<double>(c->geom, c->d_tw64.as<z64>(), F + (size_t)k * nb * npw, npw, Tb, ldt, 1.0, nullptr, nb,
                        c->stream);
    launch_plane_acc<double>(c->geom, c->d_tw64.as<z64>(), Tb, ldt, c->d_psi.as<z64>(), nv, out + (size_t)k * ldz,
                             n3, -2.0 / std::sqrt(c->omega), nrhs, false, c->stream);
  }
  c->check_launch();
  return st;
}

// Sphere rows Y [n][npw] -> grid vectors out [n][N^3] (zxy), Scatter.
void scatter_rows(lgw_ctx* c, const z64* Y, int n, z64* out) {
  const long ldt = (long)c->N * c->ncols;
  z64* Tb = c->buf<z64>("sc.Tb", (size_t)n * ldt);
  z64* ones = c->buf<z64>("sc.ones", c->n3);
  if (!c->ones_ready) {
    std::vector<z64> h1(c->n3, z64{1.0, 0.0});
    h2d(c, ones, h1.data(), c->n3 * sizeof(z64));
    c->ones_ready = true;
  }
  launch_zinv<double>(c->geom, c->d_tw64.as<z64>(), Y, c->npw, Tb, ldt, 1.0, nullptr, n, c->stream);
  launch_plane_acc<double>(c->geom, c->d_tw64.as<z64>(), Tb, ldt, ones, 1, out, c->n3, 1.0 / std::sqrt(c->omega), n,
                           false, c->stream);
}

// out[x * nu + u] = scale * Gather(U[u] * X[x]) for grid vectors U [nu], X [nx]
void gather_products(lgw_ctx* c, const z64* U, int nu, const z64* X, int nx, z64* out, double scale) {
  const long ldt = (long)c->N * c->ncols;
  z64* Tb = c->buf<z64>("gp.Tb", (size_t)nu * nx * ldt);
  launch_plane_pair_fwd<double>(c->geom, c->d_tw64.as<z64>(), U, nu, X, c->n3, nx, Tb, ldt, c->stream);
  launch_zfwd<double>(c->geom, c->d_tw64.as<z64>(), Tb, ldt, scale * std::sqrt(c->omega) / (double)c->n3, nullptr, 0,
                      nullptr, nullptr, 0, nullptr, out, c->npw, nullptr, nu * nx, c->stream);
}

// Vector-Jacobian product of dn[z][j] = chi0(z) X[j] with respect to the local
// potential, the valence orbitals and energies relaxing with it (first-order
// perturbation theory), for L = Re sum_{z,j,r} conj(G[z][j](r)) dn[z][j](r).
// With f_{v,s} = P (H - e_v - s z)^-1 P b_v, a_{v,s} = P (H - e_v - s conj z)^-1 P G_v,
// G_v = Gather(g conj(psi_v)) and ~ denoting Scatter to the grid:
//   dL/dV = 2 Re sum conj(~a) ~f                        (H inside the resolvents)
//         - 2 Re(sum_s a^H f) |psi_v|^2                  (e_v in the shifts)
//         - dV Re conj(~eta_w) conj(psi_w)               (conduction part of d psi_w)
//         + dV Re sum_k t_wk psi_k conj(psi_w)           (valence rotations)
// where eta_w = P (H - e_w)^-1 P S_w solves one static Sternheimer system per
// band for the total sensitivity S_w of L to the sphere coefficients of
// conj(psi_w) (through b_v, G_v and the projector), and t_wk = S_w^H Phi_k / (e_w - e_k).
lgw_status vjp_internal(lgw_ctx* c, int nrhs, const z64* X, int nz, const lgw_c128* zl, const z64* G, double* gV,
                        bool accumulate = false) {
  const int nv = c->nv, npw = c->npw;
  const long n3 = c->n3;
  const int nb = nrhs * nv;
  const double dvol = c->dV;
  lgw_status st = LGW_OK;
  if (!accumulate) HIPCHK(hipMemsetAsync(gV, 0, n3 * sizeof(double), c->stream));
  z64* Xun = c->buf<z64>("vj.Xun", (size_t)nb * npw);   // Gather(conj psi_v x_j), rows j*nv+v
  z64* B0 = c->buf<z64>("vj.B0", (size_t)nb * npw);
  gather_products(c, c->d_u.as<z64>(), nv, X, nrhs, Xun, 1.0);
  HIPCHK(hipMemcpyAsync(B0, Xun, (size_t)nb * npw * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
  proj<double>(c, B0, npw, nullptr, nb);
  z64* S = c->buf<z64>("vj.S", (size_t)nv * npw);      // total orbital sensitivity
  HIPCHK(hipMemsetAsync(S, 0, (size_t)nv * npw * sizeof(z64), c->stream));
  z64* Gun = c->buf<z64>("vj.Gun", (size_t)nb * npw);
  z64* PG = c->buf<z64>("vj.PG", (size_t)nb * npw);
  z64* Fs = c->buf<z64>("vj.F", (size_t)2 * nb * npw);  // f_{s} rows s*nb + (j*nv+v)
  z64* As = c->buf<z64>("vj.A", (size_t)2 * nb * npw);
  z64* Fsum = c->buf<z64>("vj.Fsum", (size_t)nb * npw);
  z64* Asum = c->buf<z64>("vj.Asum", (size_t)nb * npw);
  z64* gf = c->buf<z64>("vj.gf", (size_t)2 * nb * n3);  // grids of f
  z64* ga = c->buf<z64>("vj.ga", (size_t)2 * nb * n3);  // grids of a
  z64* cg = c->buf<z64>("vj.cg", (size_t)nrhs * n3);    // conj(g_j)
  z64* cx = c->buf<z64>("vj.cx", (size_t)nrhs * n3);    // conj(x_j)
  z64* tmpS = c->buf<z64>("vj.tS", (size_t)nv * npw);
  z64* Cm = c->buf<z64>("vj.Cm", (size_t)nv * nb);
  z64* part = c->buf<z64>("vj.part", (size_t)64 * nv * nb + 64);
  launch_conj(X, cx, (long)nrhs * n3, c->stream);
  const z64 zero{0, 0};
  for (int k = 0; k < nz; ++k) {
    const z64 zz{zl[k].re, zl[k].im};
    const bool zero_z = zz.x == 0.0 && zz.y == 0.0;
    const z64* Gk = G + (size_t)k * nrhs * n3;
    gather_products(c, c->d_u.as<z64>(), nv, Gk, nrhs, Gun, 1.0);
    HIPCHK(hipMemcpyAsync(PG, Gun, (size_t)nb * npw * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    proj<double>(c, PG, npw, nullptr, nb);
    launch_conj(Gk, cg, (long)nrhs * n3, c->stream);
    // forward and adjoint solves
    const int ns = zero_z ? 1 : 2;
    for (int which = 0; which < 2; ++which) {   // 0: forward (z), 1: adjoint (conj z)
      std::vector<int> bidx;
      std::vector<z64> sh;
      std::vector<double> w2;
      for (int si = 0; si < ns; ++si) {
        const double sg = si == 0 ? 1.0 : -1.0;
        const z64 zs = which == 0 ? zz : conj(zz);
        for (int p = 0; p < nb; ++p) {
          bidx.push_back(p);
          sh.push_back(z64{c->eps[p % nv] + sg * zs.x, sg * zs.y});
          w2.push_back(0.0);
        }
      }
      SolveOut so;
      solve(c, zero_z ? K_CGLIN : K_SQMR, which == 0 ? B0 : PG, bidx, sh, w2, which == 0 ? Fs : As, so);
      for (size_t i = 0; i < so.flags.size(); ++i) {
        if (so.flags[i] == FLAG_BREAK) st = LGW_EBREAKDOWN;
        else if (so.flags[i] != FLAG_CONV && st == LGW_OK) st = LGW_ENOCONV;
      }
    }
    const double mult = zero_z ? 2.0 : 1.0;   // at z = 0 both shifts give the same system
    // F_v = sum_s f_s, A_v = sum_s a_s
    if (zero_z) {
      launch_add(Fsum, Fs, Fs, (long)nb * npw, c->stream);
      launch_add(Asum, As, As, (long)nb * npw, c->stream);
    } else {
      launch_add(Fsum, Fs, Fs + (size_t)nb * npw, (long)nb * npw, c->stream);
      launch_add(Asum, As, As + (size_t)nb * npw, (long)nb * npw, c->stream);
    }
    scatter_rows(c, Fs, ns * nb, gf);
    scatter_rows(c, As, ns * nb, ga);
    // T1: 2 Re sum_s conj(~a_s) ~f_s
    for (int q = 0; q < ns * nb; ++q)
      launch_acc_re(gV, ga + (size_t)q * n3, gf + (size_t)q * n3, z64{2.0 * mult, 0.0}, n3, c->stream);
    // T2: -2 Re(sum_s a_s^H f_s) |psi_v|^2
    {
      std::vector<z64> e(ns * nb);
      z64* d_e = c->buf<z64>("vj.e", ns * nb);
      for (int q = 0; q < ns * nb; ++q)
        launch_dots(As + (size_t)q * npw, 0, 1, Fs + (size_t)q * npw, npw, d_e + q, part, c->stream);
      HIPCHK(hipMemcpyAsync(e.data(), d_e, e.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      std::vector<double> ev(nv, 0.0);
      for (int q = 0; q < ns * nb; ++q) ev[q % nv] += mult * e[q].x;
      for (int v = 0; v < nv; ++v)
        launch_acc_re(gV, c->d_psi.as<z64>() + (size_t)v * n3, c->d_psi.as<z64>() + (size_t)v * n3,
                      z64{-2.0 * ev[v], 0.0}, n3, c->stream);
    }
    // sensitivities through b_v and G_v: S_v += -(2/dV) Gather(conj(g_j) ~F_v + ~A_v conj(x_j))
    scatter_rows(c, Fsum, nb, gf);
    scatter_rows(c, Asum, nb, ga);
    for (int j = 0; j < nrhs; ++j) {
      gather_products(c, cg + (size_t)j * n3, 1, gf + (size_t)j * nv * n3, nv, tmpS, -2.0 / dvol);
      launch_add(S, S, tmpS, (long)nv * npw, c->stream);
      gather_products(c, cx + (size_t)j * n3, 1, ga + (size_t)j * nv * n3, nv, tmpS, -2.0 / dvol);
      launch_add(S, S, tmpS, (long)nv * npw, c->stream);
    }
    // sensitivities through the projector
    {
      std::vector<z64> cvw((size_t)nv * nb), dvw((size_t)nb * nv), cm((size_t)nv * nb);
      launch_gemm_hn(Gun, npw, nb, c->d_Phi.as<z64>(), npw, nv, npw, Cm, part, c->stream);   // [w][i] = Gun_i^H Phi_w
      HIPCHK(hipMemcpyAsync(cvw.data(), Cm, cvw.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      launch_gemm_hn(c->d_Phi.as<z64>(), npw, nv, Xun, npw, nb, npw, Cm, part, c->stream);   // [i][w] = Phi_w^H Xun_i
      HIPCHK(hipMemcpyAsync(dvw.data(), Cm, dvw.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      for (int w = 0; w < nv; ++w)
        for (int i = 0; i < nb; ++i) cm[(size_t)w * nb + i] = (-2.0 / dvol) * cvw[(size_t)w * nb + i];
      h2d(c, Cm, cm.data(), cm.size() * sizeof(z64));
      launch_block_sub(S, npw, nv, Fsum, npw, nb, Cm, npw, c->stream);
      for (int w = 0; w < nv; ++w)
        for (int i = 0; i < nb; ++i) cm[(size_t)w * nb + i] = (-2.0 / dvol) * conj(dvw[(size_t)i * nv + w]);
      h2d(c, Cm, cm.data(), cm.size() * sizeof(z64));
      launch_block_sub(S, npw, nv, Asum, npw, nb, Cm, npw, c->stream);
    }
    c->check_launch();
  }
  // orbital response: eta_w = P (H - e_w)^-1 P S_w
  {
    z64* PS = c->buf<z64>("vj.PS", (size_t)nv * npw);
    z64* eta = c->buf<z64>("vj.eta", (size_t)nv * npw);
    HIPCHK(hipMemcpyAsync(PS, S, (size_t)nv * npw * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    proj<double>(c, PS, npw, nullptr, nv);
    std::vector<int> bidx(nv);
    std::vector<z64> sh(nv);
    std::vector<double> w2(nv, 0.0);
    for (int w = 0; w < nv; ++w) {
      bidx[w] = w;
      sh[w] = z64{c->eps[w], 0.0};
    }
    SolveOut so;
    solve(c, K_CGLIN, PS, bidx, sh, w2, eta, so);
    for (size_t i = 0; i < so.flags.size(); ++i) {
      if (so.flags[i] == FLAG_BREAK) st = LGW_EBREAKDOWN;
      else if (so.flags[i] != FLAG_CONV && st == LGW_OK) st = LGW_ENOCONV;
    }
    z64* geta = c->buf<z64>("vj.geta", (size_t)nv * n3);
    scatter_rows(c, eta, nv, geta);
    for (int w = 0; w < nv; ++w)
      launch_acc_re(gV, geta + (size_t)w * n3, c->d_u.as<z64>() + (size_t)w * n3, z64{-dvol, 0.0}, n3, c->stream);
    // valence rotations
    z64* tw = c->buf<z64>("vj.t", (size_t)nv * nv);
    launch_gemm_hn(S, npw, nv, c->d_Phi.as<z64>(), npw, nv, npw, tw, part, c->stream);   // [k][w] = S_w^H Phi_k
    std::vector<z64> t((size_t)nv * nv);
    HIPCHK(hipMemcpyAsync(t.data(), tw, t.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    for (int w = 0; w < nv; ++w)
      for (int kk = 0; kk < nv; ++kk) {
        if (kk == w) continue;
        const double de = c->eps[w] - c->eps[kk];
        if (std::abs(de) < 1e-10) continue;   // degenerate pair: the contribution cancels
        const z64 twk = (1.0 / de) * t[(size_t)kk * nv + w];
        launch_acc_re(gV, c->d_u.as<z64>() + (size_t)kk * n3, c->d_u.as<z64>() + (size_t)w * n3, dvol * twk, n3,
                      c->stream);
      }
  }
  (void)zero;
  c->check_launch();
  return st;
}

lgw_status worst(lgw_status a, lgw_status b) {
  if (a == LGW_EBREAKDOWN || b == LGW_EBREAKDOWN) return LGW_EBREAKDOWN;
  if (a == LGW_ENOCONV || b == LGW_ENOCONV) return LGW_ENOCONV;
  return LGW_OK;
}

// stage a user array on the device (copy when the context works on host memory)
const void* stage_in(lgw_ctx* c, const void* user, size_t bytes, const char* name) {
  if (c->opts.mem == LGW_MEM_DEVICE) return user;
  void* d = c->buf<char>(name, bytes);
  h2d(c, d, user, bytes);
  return d;
}
void* stage_out(lgw_ctx* c, void* user, size_t bytes, const char* name) {
  if (c->opts.mem == LGW_MEM_DEVICE) return user;
  return c->buf<char>(name, bytes);
}
void finish_out(lgw_ctx* c, void* user, const void* dev, size_t bytes) {
  if (c->opts.mem == LGW_MEM_DEVICE) return;
  HIPCHK(hipMemcpyAsync(user, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  c->sync();
}

lgw_status set_err(lgw_ctx* c, lgw_status st, const std::string& m) {
  if (c) c->err = m;
  return st;
}

thread_local std::string g_setup_err;

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device -> address of its copy of scratch

// Called by lgw_setup with the context's device current; once per device.
hipError_t scratch_init(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(dev)) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) g_scratch_ptr[dev] = static_cast<char*>(p);
  return e;
}

char* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// bytes of scratch lgw_hpsi_noalloc needs for n vectors (256-byte aligned parts)
size_t hpsi_noalloc_bytes(int precision, long n, long npw, long ldt) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  if (precision == LGW_FP64) return al(n * sizeof(z64)) + al(n * ldt * sizeof(z64));
  return al(n * sizeof(z32)) + al(n * ldt * sizeof(z32)) + 2 * al(n * npw * sizeof(z32));
}

// Solve statistics gathered over several internal chi0 calls.
struct SolveTally {
  std::vector<int> it, fl, sw;
  std::vector<double> res;
  long long tot_it = 0, tot_h = 0;
  void add(const lgw_ctx* c) {
    it.insert(it.end(), c->st_iters.begin(), c->st_iters.end());
    fl.insert(fl.end(), c->st_flags.begin(), c->st_flags.end());
    sw.insert(sw.end(), c->st_sweeps.begin(), c->st_sweeps.end());
    res.insert(res.end(), c->st_res.begin(), c->st_res.end());
    tot_it += c->tot_iters;
    tot_h += c->tot_h;
  }
  void store(lgw_ctx* c) const {
    c->st_iters = it;
    c->st_flags = fl;
    c->st_sweeps = sw;
    c->st_res = res;
    c->tot_iters = tot_it;
    c->tot_h = tot_h;
  }
};

// w = (eps(z) - 1) q = -v^1/2 chi0(z) v^1/2 q on plane-major grids, z = c->lz_z
// (the static operator unless a real-frequency recursion set it)
lgw_status apply_M0(lgw_ctx* c, const z64* q, z64* w, SolveTally& tally) {
  const long n3 = c->n3;
  z64* x1 = c->buf<z64>("lz.x1", n3);
  vhalf_inplace(c, x1, 1, 1.0, q);
  const lgw_c128 z0{c->lz_z.x, c->lz_z.y};
  c->tot_iters = c->tot_h = 0;
  const lgw_status st = chi0_internal(c, 1, x1, 1, &z0, w, n3);
  tally.add(c);
  vhalf_inplace(c, w, 1, -1.0);
  return st;
}

// Checks the starting vector (user layout, opts.mem) and writes q_0 = q0/|q0|
// plane-major into Q.
lgw_status lanczos_start(lgw_ctx* c, const lgw_c128* q0, z64* Q) {
  const long n3 = c->n3;
  const z64* d_q0 = static_cast<const z64*>(stage_in(c, q0, n3 * sizeof(z64), "io.q0"));
  int* d_flag = c->buf<int>("flag", 1);
  HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), c->stream));
  launch_finite_check(reinterpret_cast<const double*>(d_q0), 2 * n3, d_flag, c->stream);
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  if (hflag) return set_err(c, LGW_ENAN, "non-finite value in q0");
  z64* w = c->buf<z64>("lz.w", n3);
  z64* part = c->buf<z64>("lz.part0", 64);
  double* d_nrm = c->buf<double>("lz.nrm", 1);
  launch_xyz_to_zxy(c->N, d_q0, n3, w, n3, 1, false, c->stream);
  launch_norm(w, n3, d_nrm, part, c->stream);
  double h_nrm = 0;
  HIPCHK(hipMemcpyAsync(&h_nrm, d_nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  if (!(h_nrm > 0)) return set_err(c, LGW_EINVAL, "q0 is zero");
  launch_scale_into(w, d_nrm, Q, n3, c->stream);
  return LGW_OK;
}

// Lanczos with full reorthogonalisation on eps(0) - 1 (Sec. IV): from q_0 in
// Q[0], for j < k: w = M q_j, classical Gram-Schmidt of w against q_0..q_j
// twice (the first pass's coefficients are alpha_j = Re <q_j, w> on q_j and
// beta_{j-1} up to rounding on q_{j-1}, so it also performs the three-term
// recurrence's subtraction), beta_j = |w|, q_{j+1} = w / beta_j.  Stops early
// when beta_j < 1e-14 max|alpha|.  W0 (or null) keeps every product M q_j.
// j0 > 0 resumes a recursion whose vectors q_0..q_{j0} are in Qd and whose
// coefficients alpha, beta up to j0 - 1 are in d_alpha, d_beta (amax0 = the
// largest |alpha| among them): steps j0..k-1 run as they would have.
lgw_status lanczos_core(lgw_ctx* c, int k, z64* Qd, z64* W0, double* d_alpha, double* d_beta, int* done_out,
                        const std::function<void(int)>& ready = nullptr, int j0 = 0, double amax0 = 0.0) {
  const long n3 = c->n3;
  z64* wbuf = c->buf<z64>("lz.w", n3);
  z64* h = c->buf<z64>("lz.h", k);
  z64* part = c->buf<z64>("lz.part", (size_t)64 * (k + 1));
  double* pair = c->buf<double>("lz.pair", 2);
  lgw_status st = LGW_OK;
  SolveTally tally;
  double amax = amax0;
  int done = j0;
  for (int j = j0; j < k; ++j) {
    z64* qj = Qd + (size_t)j * n3;
    // the product lands in W0[j] when the caller keeps the products, and the
    // three-term update reads it from there into wbuf
    z64* mq = W0 ? W0 + (size_t)j * n3 : wbuf;
    st = worst(st, apply_M0(c, qj, mq, tally));
    // two classical Gram-Schmidt passes against q_0..q_j; the first one's
    // coefficient on q_j is alpha_j = Re <q_j, M q_j>, and its coefficients on
    // q_j and q_{j-1} take out the three-term recurrence's part
    launch_cgs_pass(Qd, n3, j + 1, wbuf, W0 ? mq : nullptr, n3, h, part, d_alpha + j, c->stream);
    launch_cgs_pass(Qd, n3, j + 1, wbuf, nullptr, n3, h, part, nullptr, c->stream);
    launch_norm(wbuf, n3, d_beta + j, part, c->stream, d_alpha + j, pair);
    double hb[2];
    readback(c, {{hb, pair, 2 * sizeof(double)}});
    amax = std::max(amax, std::abs(hb[0]));
    done = j + 1;
    if (hb[1] < 1e-14 * amax) break;
    if (j + 1 < k) {
      launch_scale_into(wbuf, d_beta + j, Qd + (size_t)(j + 1) * n3, n3, c->stream);
      if (ready) ready(j + 2);   // q_0 .. q_{j+1} are (being) written on the stream
    }
  }
  tally.store(c);
  *done_out = done;
  return st;
}

// Cholesky of the Hermitian m x m matrix C (row-major): log det C and C^{-1}.
// False when C is not numerically positive definite.
bool hpd_logdet_inverse(const std::vector<z64>& C, int m, double& logdet, std::vector<z64>& inv) {
  std::vector<z64> Lf((size_t)m * m, z64{0, 0});
  auto at = [&](int i, int j) -> z64& { return Lf[(size_t)i * m + j]; };
  logdet = 0.0;
  for (int j = 0; j < m; ++j) {
    double d = C[(size_t)j * m + j].x;
    for (int p = 0; p < j; ++p) d -= at(j, p).x * at(j, p).x + at(j, p).y * at(j, p).y;
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    at(j, j) = z64{ljj, 0.0};
    logdet += 2.0 * std::log(ljj);
    for (int i = j + 1; i < m; ++i) {
      z64 s = C[(size_t)i * m + j];
      for (int p = 0; p < j; ++p) s = s - cmulc(at(j, p), at(i, p));   // L[i][p] conj(L[j][p])
      at(i, j) = z64{s.x / ljj, s.y / ljj};
    }
  }
  // inverse column by column: L y = e_c, L^H x = y
  inv.assign((size_t)m * m, z64{0, 0});
  std::vector<z64> y(m), x(m);
  for (int cc = 0; cc < m; ++cc) {
    for (int i = 0; i < m; ++i) {
      z64 s = z64{i == cc ? 1.0 : 0.0, 0.0};
      for (int p = 0; p < i; ++p) s = s - at(i, p) * y[p];
      y[i] = z64{s.x / at(i, i).x, s.y / at(i, i).x};
    }
    for (int i = m - 1; i >= 0; --i) {
      z64 s = y[i];
      for (int p = i + 1; p < m; ++p) s = s - cmulc(at(p, i), x[p]);   // conj(L[p][i]) x[p]
      x[i] = z64{s.x / at(i, i).x, s.y / at(i, i).x};
    }
    for (int i = 0; i < m; ++i) inv[(size_t)i * m + cc] = x[i];
  }
  return true;
}

void dup_buf(lgw_ctx* c, DevBuf& dst, const DevBuf& src) {
  if (!src.p) return;
  dst.ensure(src.n);
  HIPCHK(hipMemcpyAsync(dst.p, src.p, src.n, hipMemcpyDeviceToDevice, c->stream));
}

// The context's i-th twin (see lgw_ctx::twins): same system and options, own
// stream, device copies of the read-only data.
lgw_ctx* twin_of(lgw_ctx* c, size_t i) {
  while (c->twins.size() <= i) c->twins.emplace_back();
  if (c->twins[i]) return c->twins[i].get();
  std::unique_ptr<lgw_ctx> t(new lgw_ctx);
  t->device = c->device;
  HIPCHK(hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking));
  t->own_stream = true;
  t->opts = c->opts;
  t->opts.stream = t->stream;
  for (int i = 0; i < 3; ++i) t->L[i] = c->L[i];
  t->N = c->N;
  t->n3 = c->n3;
  t->ecut = c->ecut;
  t->omega = c->omega;
  t->dV = c->dV;
  t->nv = c->nv;
  t->npw = c->npw;
  t->ncols = c->ncols;
  t->hx = c->hx;
  t->hy = c->hy;
  t->m = c->m;
  t->col_start = c->col_start;
  t->col_h = c->col_h;
  t->col_pos = c->col_pos;
  t->kin = c->kin;
  t->eps = c->eps;
  t->pre_ratio[0] = c->pre_ratio[0];
  t->pre_ratio[1] = c->pre_ratio[1];
  dup_buf(c, t->d_col_start, c->d_col_start);
  dup_buf(c, t->d_col_h, c->d_col_h);
  dup_buf(c, t->d_col_pos, c->d_col_pos);
  dup_buf(c, t->d_col_of, c->d_col_of);
  dup_buf(c, t->d_kin, c->d_kin);
  dup_buf(c, t->d_Vt, c->d_Vt);
  dup_buf(c, t->d_Vt32, c->d_Vt32);
  dup_buf(c, t->d_sqrtv, c->d_sqrtv);
  dup_buf(c, t->d_tw64, c->d_tw64);
  dup_buf(c, t->d_tw32, c->d_tw32);
  dup_buf(c, t->d_psi, c->d_psi);
  dup_buf(c, t->d_u, c->d_u);
  dup_buf(c, t->d_Phi, c->d_Phi);
  dup_buf(c, t->d_Phi32, c->d_Phi32);
  for (int f = 0; f < 2; ++f) {
    dup_buf(c, t->d_pre64[f], c->d_pre64[f]);
    dup_buf(c, t->d_pre32[f], c->d_pre32[f]);
  }
  c->sync();
  t->geom = Geom{t->N, t->npw, t->ncols, t->hx, t->hy, t->d_col_start.as<int>(), t->d_col_h.as<int>(),
                 t->d_col_pos.as<int>(), t->d_kin.as<double>(), t->d_col_of.as<int>()};
  c->twins[i] = std::move(t);
  return c->twins[i].get();
}

// Lower Cholesky factor L of the Hermitian positive definite m x m matrix G
// (row-major, G = L L^H) and its inverse; false if G is not positive definite.
bool chol_lower_inverse(const std::vector<z64>& G, int m, std::vector<z64>& Linv) {
  std::vector<z64> Lf((size_t)m * m, z64{0, 0});
  auto at = [&](int i, int j) -> z64& { return Lf[(size_t)i * m + j]; };
  for (int j = 0; j < m; ++j) {
    double d = G[(size_t)j * m + j].x;
    for (int p = 0; p < j; ++p) d -= norm2(at(j, p));
    if (!(d > 0.0)) return false;
    at(j, j) = z64{std::sqrt(d), 0.0};
    for (int i = j + 1; i < m; ++i) {
      z64 s = G[(size_t)i * m + j];
      for (int p = 0; p < j; ++p) s = s - cmulc(at(j, p), at(i, p));
      at(i, j) = (1.0 / at(j, j).x) * s;
    }
  }
  Linv.assign((size_t)m * m, z64{0, 0});
  for (int c = 0; c < m; ++c)           // column c of L^{-1}: L y = e_c
    for (int i = c; i < m; ++i) {
      z64 s = z64{i == c ? 1.0 : 0.0, 0.0};
      for (int p = c; p < i; ++p) s = s - at(i, p) * Linv[(size_t)p * m + c];
      Linv[(size_t)i * m + c] = (1.0 / at(i, i).x) * s;
    }
  return true;
}

double re_dot(lgw_ctx* c, const z64* a, const z64* b) {
  double* d = c->buf<double>("ll.red", 1);
  z64* part = c->buf<z64>("ll.redp", 64);
  launch_lanczos_alpha(a, b, c->n3, d, part, c->stream);
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  return v;
}

// Reverse pass through the Lanczos recursion of lanczos_core (steps j = m-2
// .. 0 that produced q_1 .. q_{m-1}).  Qb holds dL/dQ (convention dL = Re
// sum_j <Qb_j, dq_j>) and is consumed; the products M q_j are read from W0.
// Every step's sensitivity to M is a pair (q_j, wb_j) with dL += Re <wb_j,
// dM q_j>; these are handed to the chi0 VJP at z = 0 at the end, and
// M wb_j feeds back into Qb_j (M(0) is Hermitian).
lgw_status lanczos_reverse(lgw_ctx* c, int m, const z64* Qd, const z64* W0, const double* d_alpha,
                           const double* d_beta, z64* Qb, double* gV, SolveTally& tally) {
  const long n3 = c->n3;
  std::vector<double> al(m), be(m);
  readback(c, {{al.data(), d_alpha, m * sizeof(double)}, {be.data(), d_beta, m * sizeof(double)}});
  std::vector<double> bb(m, 0.0);                     // dL/d beta_j
  z64* w1 = c->buf<z64>("lr.w1", n3);
  z64* w2 = c->buf<z64>("lr.w2", n3);
  z64* pr = c->buf<z64>("lr.pair", 2 * (size_t)n3);   // rows: adjoint vector, forward vector
  z64* mw = c->buf<z64>("lr.mw", n3);
  z64* Xp = c->buf<z64>("lr.X", (size_t)(m - 1) * n3);
  z64* Gp = c->buf<z64>("lr.G", (size_t)(m - 1) * n3);
  z64* cd = c->buf<z64>("lr.c", 4 * (size_t)m);       // c1, c2, d (device)
  z64* part = c->buf<z64>("lr.part", (size_t)64 * (m + 1));
  z64* Cm = c->buf<z64>("lr.Cm", 2 * (size_t)m);
  std::vector<z64> hc(3 * (size_t)m), cm(2 * (size_t)m);
  lgw_status st = LGW_OK;
  const z64 one{1.0, 0.0};
  auto fetch = [&](const z64* d, int n, z64* hdst) {
    HIPCHK(hipMemcpyAsync(hdst, d, n * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
    c->sync();
  };
  // Qb[i] -= conj(a[i]) pr[0] + conj(b[i]) pr[1] for i <= j
  auto rank2 = [&](int j, const z64* a, const z64* b) {
    for (int i = 0; i <= j; ++i) {
      cm[2 * i] = z64{a[i].x, -a[i].y};
      cm[2 * i + 1] = z64{b[i].x, -b[i].y};
    }
    h2d(c, Cm, cm.data(), 2 * (j + 1) * sizeof(z64));
    launch_block_sub(Qb, n3, j + 1, pr, n3, 2, Cm, n3, c->stream);
  };
  for (int j = m - 2; j >= 0; --j) {
    const z64* qj = Qd + (size_t)j * n3;
    const z64* qn = Qd + (size_t)(j + 1) * n3;
    z64* qbn = Qb + (size_t)(j + 1) * n3;
    const int nj = j + 1;
    z64* c1 = cd;
    z64* c2 = cd + m;
    z64* dv = cd + 2 * m;
    // forward intermediates of step j: w1 = M q_j - alpha_j q_j - beta_{j-1} q_{j-1},
    // c1 = Q^H w1, w2 = w1 - Q c1, c2 = Q^H w2
    HIPCHK(hipMemcpyAsync(w1, W0 + (size_t)j * n3, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    launch_axpby(w1, qj, z64{-al[j], 0.0}, one, n3, c->stream);
    if (j > 0) launch_axpby(w1, qj - n3, z64{-be[j - 1], 0.0}, one, n3, c->stream);
    launch_dots(Qd, n3, nj, w1, n3, c1, part, c->stream);
    HIPCHK(hipMemcpyAsync(w2, w1, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    launch_gemv_sub(Qd, n3, nj, c1, w2, n3, c->stream);
    launch_dots(Qd, n3, nj, w2, n3, c2, part, c->stream);
    // q_{j+1} = w3 / beta_j:  wb3 = (Qb_{j+1} - q_{j+1} Re<q_{j+1}, Qb_{j+1}>) / beta_j + bb_j q_{j+1}
    const double r = re_dot(c, qn, qbn);
    z64* wb = pr;
    HIPCHK(hipMemcpyAsync(wb, qbn, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    launch_axpby(wb, qn, z64{-r / be[j] + bb[j], 0.0}, z64{1.0 / be[j], 0.0}, n3, c->stream);
    // second CGS pass w3 = w2 - Q (Q^H w2)
    HIPCHK(hipMemcpyAsync(pr + n3, w2, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    launch_dots(Qd, n3, nj, wb, n3, dv, part, c->stream);
    fetch(c2, nj, hc.data() + m);
    fetch(dv, nj, hc.data() + 2 * m);
    rank2(j, hc.data() + m, hc.data() + 2 * m);
    launch_gemv_sub(Qd, n3, nj, dv, wb, n3, c->stream);
    // first CGS pass w2 = w1 - Q (Q^H w1)
    HIPCHK(hipMemcpyAsync(pr + n3, w1, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    launch_dots(Qd, n3, nj, wb, n3, dv, part, c->stream);
    fetch(c1, nj, hc.data());
    fetch(dv, nj, hc.data() + 2 * m);
    rank2(j, hc.data(), hc.data() + 2 * m);
    launch_gemv_sub(Qd, n3, nj, dv, wb, n3, c->stream);
    // three-term step: wb is now dL/d w1
    z64* qbj = Qb + (size_t)j * n3;
    const double abar = -re_dot(c, qj, wb);
    launch_axpby(qbj, wb, z64{-al[j], 0.0}, one, n3, c->stream);
    if (j > 0) {
      bb[j - 1] += -re_dot(c, qj - n3, wb);
      launch_axpby(qbj - n3, wb, z64{-be[j - 1], 0.0}, one, n3, c->stream);
    }
    // alpha_j = Re <q_j, M q_j>: wb += abar q_j (now dL/d(M q_j)), Qb_j += abar M q_j
    launch_axpby(wb, qj, z64{abar, 0.0}, one, n3, c->stream);
    launch_axpby(qbj, W0 + (size_t)j * n3, z64{abar, 0.0}, one, n3, c->stream);
    // w = M q_j: Qb_j += M wb
    st = worst(st, apply_M0(c, wb, mw, tally));
    launch_add(qbj, qbj, mw, n3, c->stream);
    HIPCHK(hipMemcpyAsync(Xp + (size_t)j * n3, qj, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(Gp + (size_t)j * n3, wb, n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
  }
  // sum_j Re <wb_j, dM q_j>, M = -v^1/2 chi0(0) v^1/2: chi0 VJP with x = v^1/2 q_j, g = -v^1/2 wb_j
  vhalf_inplace(c, Xp, m - 1, 1.0);
  vhalf_inplace(c, Gp, m - 1, -1.0);
  const lgw_c128 z0{0.0, 0.0};
  c->tot_iters = c->tot_h = 0;
  st = worst(st, vjp_internal(c, m - 1, Xp, 1, &z0, Gp, gV, true));
  tally.add(c);
  c->check_launch();
  return st;
}


// ---------------------------------------------------------------- recycling
// Frequency recycling of the static basis (Sec. VI).  Bk, Fk: [m][nv][npw]
// right-hand sides b_{l,v} and static solutions f_{l,v}(0) of the recursion.
// For every band: the basis gamma of span{f_{l,v}(0), P (H - e_v) P b_{l,v}}
// (Gram matrix on the matrix cores, its eigen-decomposition on the host with
// directions below 1e-7 of the largest singular value dropped, then a Cholesky
// pass so that gamma is orthonormal to rounding), h = gamma^H (H - e_v) gamma,
// and gamma^H b.  The imaginary-axis solution f = 2 A (A^2 + w^2)^-1 b
// (A = P (H - e_v) P) is taken as gamma 2 h (h^2 + w^2)^-1 gamma^H b, so with
// h = W diag(e) W^H and B' = W^H gamma^H b,
//   E(i w)[a][b] = <q_a, (eps(i w) - 1) q_b> = (2 / dV) sum_v <b_{a,v}, f_{b,v}>
//                = (4 / dV) sum_v sum_i conj(B'_v[i][a]) e_i / (e_i^2 + w^2) B'_v[i][b].
// E: host [n_w][m][m].
void recycle_E(lgw_ctx* c, int m, const z64* Bk, const z64* Fk, int n_w, const double* w, std::vector<z64>& E) {
  const int nv = c->nv, npw = c->npw, n2 = 2 * m;
  const long ldt = (long)c->N * c->ncols;
  const int nb = m * nv;
  E.assign((size_t)n_w * m * m, z64{0, 0});
  // large-frequency directions D = P (H - e_v) P b (b is projected)
  z64* D = c->buf<z64>("rc.D", (size_t)nb * npw);
  z64* Tb = c->buf<z64>("rc.Tb", (size_t)std::max(nb, nv * n2) * ldt);
  z64* d_sh = c->buf<z64>("rc.sh", (size_t)std::max(nb, nv * n2));
  std::vector<z64> sh(nb);
  for (int p = 0; p < nb; ++p) sh[p] = z64{c->eps[p % nv], 0.0};
  h2d_async(c, d_sh, sh.data(), nb * sizeof(z64));
  happly<double>(c, Bk, npw, D, npw, d_sh, nullptr, 0, nullptr, Tb, nullptr, nb);
  proj<double>(c, D, npw, nullptr, nb);
  // V_v = [f_{0..m-1,v}(0); D_{0..m-1,v}] contiguous, and their Gram matrices
  z64* Vb = c->buf<z64>("rc.V", (size_t)nv * n2 * npw);
  const size_t row = (size_t)npw * sizeof(z64);
  for (int v = 0; v < nv; ++v) {
    z64* Vv = Vb + (size_t)v * n2 * npw;
    HIPCHK(hipMemcpy2DAsync(Vv, row, Fk + (size_t)v * npw, nv * row, row, m, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpy2DAsync(Vv + (size_t)m * npw, row, D + (size_t)v * npw, nv * row, row, m,
                            hipMemcpyDeviceToDevice, c->stream));
  }
  z64* Gd = c->buf<z64>("rc.G", (size_t)nv * n2 * n2);
  // the K split is largest for the fewest B rows: size for one, times the most rows
  z64* part = c->buf<z64>("rc.part", (size_t)gemm_hn_slices(npw, 1) * std::min(n2, 64) * n2);
  for (int v = 0; v < nv; ++v)
    launch_gemm_hn_mfma(Vb + (size_t)v * n2 * npw, npw, n2, Vb + (size_t)v * n2 * npw, npw, n2, npw,
                        Gd + (size_t)v * n2 * n2, part, c->stream);
  std::vector<z64> hG((size_t)nv * n2 * n2);
  HIPCHK(hipMemcpyAsync(hG.data(), Gd, hG.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  // bands in parallel host threads
  auto par = [&](auto&& fn) {
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> ex(nv);
    for (int v = 0; v < nv; ++v)
      th.emplace_back([&, v] {
        try {
          fn(v);
        } catch (...) {
          ex[v] = std::current_exception();
        }
      });
    for (auto& t : th) t.join();
    for (auto& e : ex)
      if (e) std::rethrow_exception(e);
  };
  // first pass: M = U diag(lam) U^H (M[a][b] = <V_a, V_b>), T1[k][l] = lam_k^-1/2 U[l][k]
  std::vector<int> r(nv, 0);
  std::vector<std::vector<z64>> T1(nv);
  par([&](int v) {
    std::vector<std::complex<double>> M((size_t)n2 * n2);
    for (int a = 0; a < n2; ++a)
      for (int b = 0; b < n2; ++b) {
        const z64 g = hG[((size_t)v * n2 + b) * n2 + a];
        const z64 gt = hG[((size_t)v * n2 + a) * n2 + b];
        M[(size_t)a * n2 + b] = {0.5 * (g.x + gt.x), 0.5 * (g.y - gt.y)};   // exactly Hermitian
      }
    std::vector<double> lam;
    std::vector<std::complex<double>> U;
    herm_eig(n2, M.data(), lam, U);
    const double top = lam.empty() ? 0.0 : lam.back();
    std::vector<int> keep;
    for (int k = n2 - 1; k >= 0; --k)
      if (top > 0.0 && lam[k] > 1e-14 * top) keep.push_back(k);
    r[v] = (int)keep.size();
    T1[v].assign((size_t)r[v] * n2, z64{0, 0});
    for (int i = 0; i < r[v]; ++i) {
      const int k = keep[i];
      const double sc = 1.0 / std::sqrt(lam[k]);
      for (int l = 0; l < n2; ++l) {
        const auto u = U[(size_t)l * n2 + k];
        T1[v][(size_t)i * n2 + l] = z64{sc * u.real(), sc * u.imag()};
      }
    }
  });
  int rsum = 0;
  for (int v = 0; v < nv; ++v) rsum += r[v];
  if (rsum == 0) return;
  // gamma = T V (block_sub subtracts: coefficients negated into a zeroed buffer)
  z64* Gam = c->buf<z64>("rc.Gam", (size_t)nv * n2 * npw);
  z64* Cm = c->buf<z64>("rc.Cm", (size_t)nv * n2 * n2);
  auto combine = [&](const std::vector<std::vector<z64>>& T) {
    std::vector<z64> hc((size_t)nv * n2 * n2, z64{0, 0});
    for (int v = 0; v < nv; ++v)
      for (size_t q = 0; q < T[v].size(); ++q) hc[(size_t)v * n2 * n2 + q] = z64{-T[v][q].x, -T[v][q].y};
    h2d(c, Cm, hc.data(), hc.size() * sizeof(z64));
    HIPCHK(hipMemsetAsync(Gam, 0, (size_t)nv * n2 * npw * sizeof(z64), c->stream));
    for (int v = 0; v < nv; ++v)
      launch_block_sub(Gam + (size_t)v * n2 * npw, npw, r[v], Vb + (size_t)v * n2 * npw, npw, n2,
                       Cm + (size_t)v * n2 * n2, npw, c->stream);
  };
  combine(T1);
  // second pass: M2[a][b] = <g1_a, g1_b> = L L^H, T = conj(L^-1) T1
  for (int v = 0; v < nv; ++v)
    if (r[v] > 0)
      launch_gemm_hn_mfma(Gam + (size_t)v * n2 * npw, npw, r[v], Gam + (size_t)v * n2 * npw, npw, r[v], npw,
                          Gd + (size_t)v * n2 * n2, part, c->stream);
  HIPCHK(hipMemcpyAsync(hG.data(), Gd, hG.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  std::vector<std::vector<z64>> T(nv);
  for (int v = 0; v < nv; ++v) {
    const int rv = r[v];
    if (rv == 0) continue;
    std::vector<z64> M2((size_t)rv * rv), Linv;
    for (int a = 0; a < rv; ++a)
      for (int b = 0; b < rv; ++b) {
        const z64 g = hG[(size_t)v * n2 * n2 + (size_t)b * rv + a];
        const z64 gt = hG[(size_t)v * n2 * n2 + (size_t)a * rv + b];
        M2[(size_t)a * rv + b] = z64{0.5 * (g.x + gt.x), 0.5 * (g.y - gt.y)};
      }
    if (!chol_lower_inverse(M2, rv, Linv)) throw Fail{LGW_EBREAKDOWN, "recycling basis lost orthogonality"};
    T[v].assign((size_t)rv * n2, z64{0, 0});
    for (int i = 0; i < rv; ++i)
      for (int j = 0; j <= i; ++j) {
        const z64 li{Linv[(size_t)i * rv + j].x, -Linv[(size_t)i * rv + j].y};
        for (int l = 0; l < n2; ++l)
          T[v][(size_t)i * n2 + l] = T[v][(size_t)i * n2 + l] + li * T1[v][(size_t)j * n2 + l];
      }
  }
  combine(T);
  // h and gamma^H b: (H - e_v) gamma for every band in one application (rows v * n2 + i)
  z64* HG = c->buf<z64>("rc.HG", (size_t)nv * n2 * npw);
  std::vector<int> rows;
  std::vector<z64> shg((size_t)nv * n2, z64{0, 0});
  for (int v = 0; v < nv; ++v)
    for (int i = 0; i < r[v]; ++i) {
      rows.push_back(v * n2 + i);
      shg[(size_t)v * n2 + i] = z64{c->eps[v], 0.0};
    }
  int* d_rows = c->buf<int>("rc.rows", rows.size());
  h2d_async(c, d_rows, rows.data(), rows.size() * sizeof(int));
  h2d_async(c, d_sh, shg.data(), shg.size() * sizeof(z64));
  happly<double>(c, Gam, npw, HG, npw, d_sh, nullptr, 0, nullptr, Tb, d_rows, (int)rows.size());
  proj<double>(c, HG, npw, d_rows, (int)rows.size());
  z64* Hh = c->buf<z64>("rc.h", (size_t)nv * n2 * n2);
  z64* Bg = c->buf<z64>("rc.bg", (size_t)nv * n2 * m);
  for (int v = 0; v < nv; ++v) {
    if (r[v] == 0) continue;
    const z64* Gv = Gam + (size_t)v * n2 * npw;
    launch_gemm_hn_mfma(Gv, npw, r[v], HG + (size_t)v * n2 * npw, npw, r[v], npw, Hh + (size_t)v * n2 * n2, part,
                        c->stream);   // [b][a] = <g_a, H g_b>
    launch_gemm_hn_mfma(Gv, npw, r[v], Bk + (size_t)v * npw, (long)nv * npw, m, npw, Bg + (size_t)v * n2 * m, part,
                        c->stream);   // [l][a] = <g_a, b_l>
  }
  std::vector<z64> hh((size_t)nv * n2 * n2), hb((size_t)nv * n2 * m);
  readback(c, {{hh.data(), Hh, hh.size() * sizeof(z64)}, {hb.data(), Bg, hb.size() * sizeof(z64)}});
  // per band: h = W diag(e) W^H, B' = W^H (gamma^H b), and its part of E
  std::vector<std::vector<z64>> Ev(nv);
  const double pref = 4.0 / c->dV;
  par([&](int v) {
    const int rv = r[v];
    Ev[v].assign((size_t)n_w * m * m, z64{0, 0});
    if (rv == 0) return;
    std::vector<std::complex<double>> h((size_t)rv * rv);
    for (int a = 0; a < rv; ++a)
      for (int b = 0; b < rv; ++b) {
        const z64 x = hh[(size_t)v * n2 * n2 + (size_t)b * rv + a];    // <g_a, H g_b>
        const z64 xt = hh[(size_t)v * n2 * n2 + (size_t)a * rv + b];   // <g_b, H g_a>
        h[(size_t)a * rv + b] = {0.5 * (x.x + xt.x), 0.5 * (x.y - xt.y)};
      }
    std::vector<double> e;
    std::vector<std::complex<double>> W;
    herm_eig(rv, h.data(), e, W);
    std::vector<std::complex<double>> Bp((size_t)rv * m);   // B'[i][l]
    for (int i = 0; i < rv; ++i)
      for (int l = 0; l < m; ++l) {
        std::complex<double> acc(0, 0);
        for (int a = 0; a < rv; ++a) {
          const z64 g = hb[(size_t)v * n2 * m + (size_t)l * rv + a];
          acc += std::conj(W[(size_t)a * rv + i]) * std::complex<double>(g.x, g.y);
        }
        Bp[(size_t)i * m + l] = acc;
      }
    for (int q = 0; q < n_w; ++q) {
      const double w2 = w[q] * w[q];
      for (int i = 0; i < rv; ++i) {
        const double f = pref * e[i] / (e[i] * e[i] + w2);
        for (int a = 0; a < m; ++a) {
          const std::complex<double> ca = f * std::conj(Bp[(size_t)i * m + a]);
          z64* Er = Ev[v].data() + ((size_t)q * m + a) * m;
          for (int b = 0; b < m; ++b) {
            const std::complex<double> t = ca * Bp[(size_t)i * m + b];
            Er[b] = z64{Er[b].x + t.real(), Er[b].y + t.imag()};
          }
        }
      }
    }
  });
  for (int v = 0; v < nv; ++v)
    for (size_t q = 0; q < E.size(); ++q) E[q] = E[q] + Ev[v][q];
}

}  // namespace

// ======================================================================= ABI
namespace {

void tune_file_read_locked() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("LGW_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    int N, f32, bucket, best, rep;
    double u[4];
    if (std::sscanf(line, "plane %d %d %d %d %d %lf %lf %lf %lf", &N, &f32, &bucket, &best, &rep, &u[0], &u[1], &u[2],
                    &u[3]) == 9 &&
        best >= 0 && best < 4 && bucket >= 0 && bucket < kTuneBuckets) {
      PlaneTune t;
      t.best = best;
      t.rep = rep;
      for (int v = 0; v < 4; ++v) t.us[v] = u[v];
      g_tune[std::make_tuple(N, f32, bucket)] = t;
    }
  }
  std::fclose(f);
}

// Measure the plane-pass variants for this context's grid in each batch
// bucket not yet in the table (FP64, and FP32 when the context uses it).
void autotune_plane(lgw_ctx* c) {
  if (c->opts.autotune == 0) return;
  std::vector<std::pair<int, int>> todo;   // (single precision, bucket)
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_file_read_locked();
    for (int f32 = 0; f32 <= (c->opts.precision == LGW_MIXED ? 1 : 0); ++f32)
      for (int b = 0; b < kTuneBuckets; ++b)
        if (!g_tune.count(std::make_tuple(c->N, f32, b))) todo.push_back({f32, b});
  }
  if (todo.empty()) return;
  const long ldt = (long)c->N * c->ncols;
  const size_t cap_bytes = size_t(256) << 20;
  std::vector<std::string> lines;
  DevBuf buf;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (const auto& fb : todo) {
    const int f32 = fb.first, b = fb.second;
    const size_t e = f32 ? sizeof(z32) : sizeof(z64);
    const int rep = (int)std::max<long>(1, std::min<long>(kTuneRep[b], (long)(cap_bytes / (ldt * e))));
    buf.ensure((size_t)rep * ldt * e);
    HIPCHK(hipMemsetAsync(buf.p, 0, (size_t)rep * ldt * e, c->stream));
    PlaneTune t;
    t.rep = rep;
    for (int v = 0; v < plane_variants(); ++v) {
      auto launch = [&] {
        if (f32)
          launch_plane_hv<float>(c->geom, c->d_tw32.as<z32>(), buf.as<z32>(), ldt, c->d_Vt32.as<float>(), nullptr,
                                 rep, c->stream, v);
        else
          launch_plane_hv<double>(c->geom, c->d_tw64.as<z64>(), buf.as<z64>(), ldt, c->d_Vt.as<double>(), nullptr,
                                  rep, c->stream, v);
      };
      launch();   // warm-up
      const int reps = b == 0 ? 8 : 3;
      HIPCHK(hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps; ++r) launch();
      HIPCHK(hipEventRecord(e1, c->stream));
      HIPCHK(hipEventSynchronize(e1));
      c->check_launch();
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      t.us[v] = 1e3 * ms / reps;
      if (t.best < 0 || t.us[v] < t.us[t.best]) t.best = v;
    }
    char line[256];
    std::snprintf(line, sizeof line, "plane %d %d %d %d %d %.3f %.3f %.3f %.3f\n", c->N, f32, b, t.best, rep, t.us[0],
                  t.us[1], t.us[2], t.us[3]);
    lines.push_back(line);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(c->N, f32, b)] = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->sync();
  const char* path = std::getenv("LGW_TUNE_CACHE");
  if (path && *path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (FILE* f = std::fopen(path, "a")) {
      for (const auto& l : lines) std::fputs(l.c_str(), f);
      std::fclose(f);
    }
  }
}

}  // namespace

namespace {

// E[z][a][b] = <q_a, (eps(z) - 1) q_b> (host, row-major) for the plane-major
// basis Qz [k][N^3] on the device.
lgw_status project_internal(lgw_ctx* c, int k, const z64* Qz, int n_z, const lgw_c128* z, std::vector<z64>& e) {
  const long n3 = c->n3;
  z64* X = c->buf<z64>("pj.X", (size_t)k * n3);
  HIPCHK(hipMemcpyAsync(X, Qz, (size_t)k * n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
  vhalf_inplace(c, X, k, 1.0);
  z64* D = c->buf<z64>("pj.D", (size_t)n_z * k * n3);
  c->tot_iters = c->tot_h = 0;
  lgw_status st = chi0_internal(c, k, X, n_z, z, D, (long)k * n3);
  vhalf_inplace(c, D, n_z * k, -1.0);
  z64* Et = c->buf<z64>("pj.E", (size_t)n_z * k * k);
  z64* part = c->buf<z64>("pj.part", (size_t)gemm_hn_slices(n3, n_z * k) * std::min(k, 64) * n_z * k);
  launch_gemm_hn_mfma(Qz, n3, k, D, n3, n_z * k, n3, Et, part, c->stream);   // Et[z * k + b][a]
  c->check_launch();
  std::vector<z64> h((size_t)n_z * k * k);
  HIPCHK(hipMemcpyAsync(h.data(), Et, h.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  // Et[z][b][a] = <q_a, M q_b>  ->  E[z][a][b]
  e.assign(h.size(), z64{0, 0});
  for (int i = 0; i < n_z; ++i)
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) e[((size_t)i * k + a) * k + b] = h[((size_t)i * k + b) * k + a];
  return st;
}

// Scope of the self-energy's resolvents of H: FP64, no preconditioner and
// no conduction projector; graphs captured with the other settings are
// dropped on entry and those captured inside on exit.
struct ResolventScope {
  lgw_ctx* c;
  lgw_opts saved;
  explicit ResolventScope(lgw_ctx* cc) : c(cc), saved(cc->opts) {
    c->drop_graphs();
    c->opts.precision = LGW_FP64;
    c->opts.precond = 0;
    c->no_proj = true;
  }
  ~ResolventScope() {
    c->drop_graphs();
    c->no_proj = false;
    c->opts = saved;
  }
};

// Re tr(A B) for k x k row-major matrices
double re_trace_prod(const std::vector<z64>& A, const std::vector<z64>& B, int k) {
  double t = 0.0;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      const z64 x = A[(size_t)a * k + b], y = B[(size_t)b * k + a];
      t += x.x * y.x - x.y * y.y;
    }
  return t;
}

// F_ne of the Lorentzian model: (1/2) a / (w + a sgn w), 0 at w = 0
double lorentz_F(double w, double a) {
  if (std::abs(w) <= 1e-12) return 0.0;
  return 0.5 * a / (w + (w > 0 ? a : -a));
}

}  // namespace

extern "C" {

void lgw_default_opts(lgw_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = LGW_FP64;
  o->tol = 1e-13;
  o->max_iter = 5000;
  o->check_every = 8;
  o->precond = 0;
  o->deterministic = 1;
  o->mem = LGW_MEM_DEVICE;
  o->stream = nullptr;
  o->mem_budget_gb = 16.0;
  o->inner_tol = 1e-5;
  o->max_sweeps = 8;
  o->use_graph = 1;
  o->precond_shift = 3.0;
  o->imag_form = 0;
  o->multishift = 0;
  o->model = 0;
  o->autotune = 1;
}

lgw_status lgw_setup(lgw_ctx** out, const double cell[9], const int grid[3], double ecut, const double* V_loc,
                     int n_v, const lgw_c128* psi_v, const double* eps_v, const lgw_opts* opts) {
  if (!out) return LGW_EINVAL;
  *out = nullptr;
  lgw_opts o;
  lgw_default_opts(&o);
  if (opts) o = *opts;
  auto bad = [&](const std::string& m) {
    g_setup_err = m;
    return LGW_EINVAL;
  };
  if (!cell || !grid || !V_loc || !psi_v || !eps_v) return bad("null argument");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (i != j && cell[3 * i + j] != 0.0) return bad("cell must be orthorhombic (diagonal)");
  for (int i = 0; i < 3; ++i)
    if (!(cell[4 * i] > 0.0) || !std::isfinite(cell[4 * i])) return bad("cell lengths must be positive");
  if (grid[0] != grid[1] || grid[1] != grid[2]) return bad("grid must be cubic (N, N, N)");
  if (!grid_supported(grid[0])) return bad("grid N must be one of 16, 24, 32, 40, 48, 64, 72");
  if (!(ecut > 0.0) || !std::isfinite(ecut)) return bad("ecut must be positive");
  if (n_v < 1 || n_v > kMaxBands) return bad("n_v must be in 1..32");
  for (int v = 0; v < n_v; ++v) {
    if (!std::isfinite(eps_v[v])) { g_setup_err = "non-finite eps_v"; return LGW_ENAN; }
    if (v > 0 && eps_v[v] < eps_v[v - 1]) return bad("eps_v must be ascending");
  }
  if (!(o.tol > 0.0) || o.max_iter < 1 || o.check_every < 1) return bad("invalid solver options");
  if (o.precision != LGW_FP64 && o.precision != LGW_MIXED) return bad("invalid precision");
  if (o.precond != 0 && o.precond != 1) return bad("precond must be 0 or 1");
  if (o.precond == 1 && !(o.precond_shift > 0.0 && std::isfinite(o.precond_shift)))
    return bad("precond_shift must be positive");
  if (o.imag_form != 0 && o.imag_form != 1) return bad("imag_form must be 0 or 1");
  if (o.multishift != 0 && o.multishift != 1) return bad("multishift must be 0 or 1");
  if (o.model != 0 && o.model != 1) return bad("model must be 0 or 1");
  if (o.autotune != 0 && o.autotune != 1) return bad("autotune must be 0 or 1");
  if (o.mem != LGW_MEM_DEVICE && o.mem != LGW_MEM_HOST) return bad("invalid mem mode");
  const int N = grid[0];
  const long n3 = (long)N * N * N;
  if (o.mem == LGW_MEM_HOST) {
    for (long i = 0; i < n3; ++i)
      if (!std::isfinite(V_loc[i])) { g_setup_err = "non-finite V_loc"; return LGW_ENAN; }
    for (long i = 0; i < n3 * n_v; ++i)
      if (!std::isfinite(psi_v[i].re) || !std::isfinite(psi_v[i].im)) { g_setup_err = "non-finite psi_v"; return LGW_ENAN; }
  }
  // plane-wave sphere in lexicographic (mx, my, mz) order
  const double L[3] = {cell[0], cell[4], cell[8]};
  const double g0[3] = {2 * M_PI / L[0], 2 * M_PI / L[1], 2 * M_PI / L[2]};
  const int hmax = N / 2 - 1;
  std::vector<int> m, col_start, col_h, col_pos;
  std::vector<double> kin;
  int hx = 0, hy = 0;
  const int lim = N;  // search range beyond the grid to detect overflow
  for (int mx = -lim; mx <= lim; ++mx)
    for (int my = -lim; my <= lim; ++my) {
      const double exy = 0.5 * (std::pow(g0[0] * mx, 2) + std::pow(g0[1] * my, 2));
      if (exy > ecut) continue;
      int h = 0;
      while (0.5 * std::pow(g0[2] * (h + 1), 2) + exy <= ecut) ++h;
      if (std::abs(mx) > hmax || std::abs(my) > hmax || h > hmax)
        return bad("plane-wave sphere does not fit the grid (max|m_i| must be <= N/2-1)");
      col_start.push_back((int)kin.size());
      col_h.push_back(h);
      col_pos.push_back(((mx + N) % N) * N + ((my + N) % N));
      hx = std::max(hx, std::abs(mx));
      hy = std::max(hy, std::abs(my));
      for (int mz = -h; mz <= h; ++mz) {
        m.push_back(mx);
        m.push_back(my);
        m.push_back(mz);
        kin.push_back(exy + 0.5 * std::pow(g0[2] * mz, 2));
      }
    }
  if (kin.size() <= (size_t)n_v) return bad("plane-wave sphere smaller than the valence set");

  std::unique_ptr<lgw_ctx> c(new lgw_ctx);
  try {
    c->opts = o;
    HIPCHK(hipGetDevice(&c->device));
    {
      // the no-allocation entry point's scratch on this device (once per device)
      const hipError_t se = scratch_init(c->device);
      if (se != hipSuccess)
        c->scratch_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(se);
    }
    if (o.stream) c->stream = (hipStream_t)o.stream;
    else {
      HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    c->L[0] = L[0]; c->L[1] = L[1]; c->L[2] = L[2];
    c->N = N;
    c->n3 = n3;
    c->ecut = ecut;
    c->omega = L[0] * L[1] * L[2];
    c->dV = c->omega / (double)n3;
    c->nv = n_v;
    c->npw = (int)kin.size();
    c->ncols = (int)col_start.size();
    c->hx = hx;
    c->hy = hy;
    c->m = m;
    c->col_start = col_start;
    c->col_h = col_h;
    c->col_pos = col_pos;
    c->kin = kin;
    c->eps.assign(eps_v, eps_v + n_v);
    upload(c.get(), c->d_col_start, col_start);
    upload(c.get(), c->d_col_h, col_h);
    upload(c.get(), c->d_col_pos, col_pos);
    {
      // plane position -> column (the transforms' direct loads and stores)
      std::vector<int> col_of((size_t)N * N, -1);
      for (size_t ci = 0; ci < col_pos.size(); ++ci) col_of[col_pos[ci]] = (int)ci;
      upload(c.get(), c->d_col_of, col_of);
    }
    upload(c.get(), c->d_kin, kin);
    if (o.precond == 1) {
      double kmax = 0.0;
      for (double k : kin) kmax = std::max(kmax, k);
      for (int f = 0; f < 2; ++f) {
        std::vector<double> d(kin.size());
        std::vector<float> d32(kin.size());
        for (size_t i = 0; i < kin.size(); ++i) {
          const double g = kin[i] + o.precond_shift;
          d[i] = f == 0 ? 1.0 / std::sqrt(g) : 1.0 / g;
          d32[i] = (float)d[i];
        }
        upload(c.get(), c->d_pre64[f], d);
        upload(c.get(), c->d_pre32[f], d32);
        const double q = o.precond_shift / (kmax + o.precond_shift);
        c->pre_ratio[f] = f == 0 ? std::sqrt(q) : q;
      }
    }
    c->geom = Geom{N, c->npw, c->ncols, hx, hy, c->d_col_start.as<int>(), c->d_col_h.as<int>(),
                   c->d_col_pos.as<int>(), c->d_kin.as<double>(), c->d_col_of.as<int>()};
    // twiddles exp(-2 pi i j / N)
    std::vector<z64> tw(N);
    std::vector<z32> tw32(N);
    for (int j = 0; j < N; ++j) {
      const double a = 2.0 * M_PI * (double)j / (double)N;
      tw[j] = z64{std::cos(a), -std::sin(a)};
      tw32[j] = z32{(float)tw[j].x, (float)tw[j].y};
    }
    upload(c.get(), c->d_tw64, tw);
    upload(c.get(), c->d_tw32, tw32);
    // truncated Coulomb square root on the zxy grid
    {
      const double R = 0.5 * std::min(L[0], std::min(L[1], L[2]));
      std::vector<double> s(n3);
      for (int z = 0; z < N; ++z)
        for (int x = 0; x < N; ++x)
          for (int y = 0; y < N; ++y) {
            const int fx = x <= N / 2 - (N % 2 == 0 ? 1 : 0) ? x : x - N;
            const int fy = y <= N / 2 - (N % 2 == 0 ? 1 : 0) ? y : y - N;
            const int fz = z <= N / 2 - (N % 2 == 0 ? 1 : 0) ? z : z - N;
            // signed FFT frequencies: 0..N/2-1, -N/2..-1
            const double kx = g0[0] * fx, ky = g0[1] * fy, kz = g0[2] * fz;
            const double k2 = kx * kx + ky * ky + kz * kz;
            double v;
            if (k2 == 0.0) v = 2.0 * M_PI * R * R;
            else v = 4.0 * M_PI * (1.0 - std::cos(std::sqrt(k2) * R)) / k2;
            s[(long)z * N * N + (long)x * N + y] = std::sqrt(v);
          }
      upload(c.get(), c->d_sqrtv, s);
    }
    lgw_ctx* cp = c.get();
    // potential
    const double* dVloc = static_cast<const double*>(stage_in(cp, V_loc, n3 * sizeof(double), "in.V"));
    int* d_flag = cp->buf<int>("flag", 1);
    HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), cp->stream));
    launch_finite_check(dVloc, n3, d_flag, cp->stream);
    c->d_Vt.ensure(n3 * sizeof(double));
    launch_real_xyz_to_zxy(N, dVloc, c->d_Vt.as<double>(), cp->stream);
    {
      std::vector<double> hv(n3);
      HIPCHK(hipMemcpyAsync(hv.data(), c->d_Vt.p, n3 * sizeof(double), hipMemcpyDeviceToHost, cp->stream));
      cp->sync();
      std::vector<float> hf(n3);
      for (long i = 0; i < n3; ++i) hf[i] = (float)hv[i];
      upload(cp, c->d_Vt32, hf);
    }
    // orbitals
    const z64* dpsi = static_cast<const z64*>(stage_in(cp, psi_v, (size_t)n_v * n3 * sizeof(z64), "in.psi"));
    launch_finite_check(reinterpret_cast<const double*>(dpsi), 2 * n3 * n_v, d_flag, cp->stream);
    c->d_psi.ensure((size_t)n_v * n3 * sizeof(z64));
    c->d_u.ensure((size_t)n_v * n3 * sizeof(z64));
    launch_xyz_to_zxy(N, dpsi, n3, c->d_psi.as<z64>(), n3, n_v, false, cp->stream);
    launch_xyz_to_zxy(N, dpsi, n3, c->d_u.as<z64>(), n3, n_v, true, cp->stream);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, d_flag, sizeof(int), hipMemcpyDeviceToHost, cp->stream));
    cp->sync();
    if (hflag) {
      g_setup_err = "non-finite V_loc or psi_v";
      return LGW_ENAN;
    }
    // Phi = Gather(conj(psi_v)) via the pair transform with a unit potential
    const int npw = c->npw;
    const long ldt = (long)N * c->ncols;
    {
      z64* ones = cp->buf<z64>("tmp.ones", n3);
      std::vector<z64> h1(n3, z64{1.0, 0.0});
      h2d(cp, ones, h1.data(), n3 * sizeof(z64));
      z64* Tb = cp->buf<z64>("tmp.Tb", (size_t)n_v * ldt);
      c->d_Phi.ensure((size_t)n_v * npw * sizeof(z64));
      launch_plane_pair_fwd<double>(c->geom, c->d_tw64.as<z64>(), c->d_u.as<z64>(), n_v, ones, n3, 1, Tb, ldt,
                                    cp->stream);
      launch_zfwd<double>(c->geom, c->d_tw64.as<z64>(), Tb, ldt, std::sqrt(c->omega) / (double)n3, nullptr, 0,
                          nullptr, nullptr, 0, nullptr, c->d_Phi.as<z64>(), npw, nullptr, n_v, cp->stream);
      // overlaps <Phi_a, Phi_b> and grid norms
      z64* ov = cp->buf<z64>("tmp.ov", (size_t)n_v * n_v);
      z64* part = cp->buf<z64>("tmp.part", (size_t)n_v * n_v * 64 + 64 * n_v);
      launch_gemm_hn(c->d_Phi.as<z64>(), npw, n_v, c->d_Phi.as<z64>(), npw, n_v, npw, ov, part, cp->stream);
      z64* gn = cp->buf<z64>("tmp.gn", n_v);
      for (int v = 0; v < n_v; ++v)
        launch_dots(c->d_psi.as<z64>() + (size_t)v * n3, 0, 1, c->d_psi.as<z64>() + (size_t)v * n3, n3, gn + v,
                    part + (size_t)n_v * n_v * 64, cp->stream);
      // eigen-residual |H phi - e phi|
      z64* R = cp->buf<z64>("tmp.R", (size_t)n_v * npw);
      z64* Tb2 = cp->buf<z64>("tmp.Tb2", (size_t)n_v * ldt);
      z64* sh = cp->buf<z64>("tmp.sh", n_v);
      std::vector<z64> hs(n_v);
      for (int v = 0; v < n_v; ++v) hs[v] = z64{eps_v[v], 0.0};
      h2d(cp, sh, hs.data(), n_v * sizeof(z64));
      happly<double>(cp, c->d_Phi.as<z64>(), npw, R, npw, sh, nullptr, 0, nullptr, Tb2, nullptr, n_v);
      double* rn = cp->buf<double>("tmp.rn", n_v);
      z64* zero = cp->buf<z64>("tmp.zero", (size_t)n_v * npw);
      HIPCHK(hipMemsetAsync(zero, 0, (size_t)n_v * npw * sizeof(z64), cp->stream));
      launch_resid<double>(R, npw, nullptr, zero, npw, nullptr, 0, rn, npw, nullptr, n_v, cp->stream);
      cp->check_launch();
      std::vector<z64> h_ov(n_v * n_v), h_gn(n_v);
      std::vector<double> h_rn(n_v);
      readback(cp, {{h_ov.data(), ov, h_ov.size() * sizeof(z64)}, {h_gn.data(), gn, n_v * sizeof(z64)}, {h_rn.data(), rn, n_v * sizeof(double)}});
      for (int a = 0; a < n_v; ++a) {
        for (int b = 0; b < n_v; ++b) {
          const z64 x = h_ov[(size_t)b * n_v + a];
          const double target = a == b ? 1.0 : 0.0;
          if (std::abs(x.x - target) > 1e-8 || std::abs(x.y) > 1e-8) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "valence orbitals not orthonormal on the sphere (<%d|%d> = %.3e%+.3ei)",
                          a, b, x.x, x.y);
            return bad(msg);
          }
        }
        if (std::abs(h_gn[a].x * c->dV - 1.0) > 1e-8) return bad("psi_v not normalised or not band-limited");
        if (std::sqrt(h_rn[a]) > 1e-8) {
          char msg[160];
          std::snprintf(msg, sizeof msg, "eigen-residual of band %d is %.3e Ha", a, std::sqrt(h_rn[a]));
          return bad(msg);
        }
      }
      // Orthonormalise the valence block within its span (G = L L^H, Phi <-
      // conj(L^-1) Phi): the projector 1 - Phi^H Phi is then exact to rounding.
      // It matters once the Krylov vectors leave range(P), as with the
      // preconditioner: a defect d of the supplied orbitals (1e-14 from an
      // iterative eigensolver) leaves valence directions with eigenvalues of
      // either sign of order d in the projected operator.
      {
        std::vector<z64> G((size_t)n_v * n_v), Linv;
        for (int a = 0; a < n_v; ++a)
          for (int b = 0; b < n_v; ++b) G[(size_t)a * n_v + b] = h_ov[(size_t)b * n_v + a];
        for (int a = 0; a < n_v; ++a)          // exactly Hermitian
          for (int b = 0; b < a; ++b) {
            const z64 u = G[(size_t)a * n_v + b], l = G[(size_t)b * n_v + a];
            const z64 avg{0.5 * (u.x + l.x), 0.5 * (u.y - l.y)};
            G[(size_t)a * n_v + b] = avg;
            G[(size_t)b * n_v + a] = z64{avg.x, -avg.y};
          }
        if (!chol_lower_inverse(G, n_v, Linv)) return bad("valence overlap matrix not positive definite");
        // block_sub: W[c] -= sum_i X[i] Cm[c][i]; W = 0, Cm = -conj(Linv)
        std::vector<z64> cm((size_t)n_v * n_v);
        for (size_t e = 0; e < cm.size(); ++e) cm[e] = z64{-Linv[e].x, Linv[e].y};
        z64* dcm = cp->buf<z64>("tmp.cm", cm.size());
        h2d(cp, dcm, cm.data(), cm.size() * sizeof(z64));
        z64* W = cp->buf<z64>("tmp.W", (size_t)n_v * npw);
        HIPCHK(hipMemsetAsync(W, 0, (size_t)n_v * npw * sizeof(z64), cp->stream));
        launch_block_sub(W, npw, n_v, c->d_Phi.as<z64>(), npw, n_v, dcm, npw, cp->stream);
        HIPCHK(hipMemcpyAsync(c->d_Phi.p, W, (size_t)n_v * npw * sizeof(z64), hipMemcpyDeviceToDevice,
                              cp->stream));
        cp->check_launch();
      }
      c->d_Phi32.ensure((size_t)n_v * npw * sizeof(z32));
      launch_cvt_64_32(c->d_Phi.as<z64>(), c->d_Phi32.as<z32>(), (long)n_v * npw, cp->stream);
      cp->sync();
    }
    autotune_plane(cp);
    c->drop_graphs();
    c->ws.clear();
    c->up_cache.clear();
    *out = c.release();
    return LGW_OK;
  } catch (const Fail& f) {
    g_setup_err = f.msg;
    return f.st;
  } catch (const std::bad_alloc&) {
    g_setup_err = "host allocation failed";
    return LGW_ENOMEM;
  }
}

lgw_status lgw_chi0_apply(lgw_ctx* c, int n_rhs, const lgw_c128* dV, int n_z, const lgw_c128* z, lgw_c128* dn) {
  if (!c) return LGW_EINVAL;
  if (n_rhs < 0 || n_z < 0 || (n_rhs > 0 && (!dV || !dn)) || (n_z > 0 && !z))
    return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int k = 0; k < n_z; ++k) {
    if (!std::isfinite(z[k].re) || !std::isfinite(z[k].im)) return set_err(c, LGW_ENAN, "non-finite frequency");
    if (z[k].re != 0.0 && z[k].im < 0.0) return set_err(c, LGW_EINVAL, "real-axis broadening must be >= 0");
  }
  if (n_rhs == 0 || n_z == 0) return LGW_OK;
  try {
    const long n3 = c->n3;
    const size_t in_bytes = (size_t)n_rhs * n3 * sizeof(z64);
    const z64* d_in = static_cast<const z64*>(stage_in(c, dV, in_bytes, "io.in"));
    int* d_flag = c->buf<int>("flag", 1);
    HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), c->stream));
    launch_finite_check(reinterpret_cast<const double*>(d_in), 2 * (long)n_rhs * n3, d_flag, c->stream);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    if (hflag) return set_err(c, LGW_ENAN, "non-finite value in dV");
    c->tot_iters = c->tot_h = 0;
    z64* X = c->buf<z64>("io.X", (size_t)n_rhs * n3);
    launch_xyz_to_zxy(c->N, d_in, n3, X, n3, n_rhs, false, c->stream);
    z64* O = c->buf<z64>("io.O", (size_t)n_z * n_rhs * n3);
    lgw_status st = chi0_internal(c, n_rhs, X, n_z, z, O, (long)n_rhs * n3);
    const size_t out_bytes = (size_t)n_z * n_rhs * n3 * sizeof(z64);
    z64* d_out = static_cast<z64*>(stage_out(c, dn, out_bytes, "io.out"));
    launch_zxy_to_xyz(c->N, O, n3, d_out, n3, n_z * n_rhs, c->stream);
    c->check_launch();
    c->sync();
    finish_out(c, dn, d_out, out_bytes);
    if (st != LGW_OK) c->err = st == LGW_ENOCONV ? "some Sternheimer solves did not converge" : "Krylov breakdown";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_chi0_apply_many(int n_sys, lgw_ctx* const* ctx, const int* n_rhs, const lgw_c128* const* dV,
                               int n_z, const lgw_c128* z, lgw_c128* const* dn) {
  if (n_sys < 0 || (n_sys > 0 && (!ctx || !n_rhs || !dV || !dn))) return LGW_EINVAL;
  for (int i = 0; i < n_sys; ++i) {
    if (!ctx[i]) return LGW_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctx[j] == ctx[i]) return set_err(ctx[i], LGW_EINVAL, "a context appears twice");
  }
  // every system on its own stream, driven by its own host thread, so that
  // small systems fill the GPU together
  std::vector<lgw_status> st(n_sys, LGW_OK);
  std::vector<std::thread> th;
  th.reserve(n_sys);
  for (int i = 0; i < n_sys; ++i)
    th.emplace_back([&, i] {
      if (hipSetDevice(ctx[i]->device) != hipSuccess) {
        st[i] = LGW_EDEVICE;
        return;
      }
      st[i] = lgw_chi0_apply(ctx[i], n_rhs[i], dV[i], n_z, z, dn[i]);
    });
  for (auto& t : th) t.join();
  lgw_status out = LGW_OK;
  for (int i = 0; i < n_sys; ++i) {
    if (st[i] == LGW_OK) continue;
    if (st[i] != LGW_ENOCONV && st[i] != LGW_EBREAKDOWN) return st[i];
    out = worst(out, st[i]);
  }
  return out;
}

lgw_status lgw_lanczos(lgw_ctx* c, const lgw_c128* q0, int k, double* alpha, double* beta, lgw_c128* Q,
                       int* k_done) {
  if (!c) return LGW_EINVAL;
  if (k < 1 || !q0 || !alpha || !beta || !k_done) return set_err(c, LGW_EINVAL, "invalid arguments");
  try {
    const long n3 = c->n3;
    z64* Qd = c->buf<z64>("lz.Q", (size_t)k * n3);
    double* ab = c->buf<double>("lz.ab", 2 * (size_t)k);   // alpha[0..k), beta[0..k)
    double* d_alpha = ab;
    double* d_beta = ab + k;
    const lgw_status pre = lanczos_start(c, q0, Qd);
    if (pre != LGW_OK) return pre;
    int done = 0;
    const lgw_status st = lanczos_core(c, k, Qd, nullptr, d_alpha, d_beta, &done);
    // outputs
    if (c->opts.mem == LGW_MEM_DEVICE) {
      HIPCHK(hipMemcpyAsync(alpha, d_alpha, done * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(beta, d_beta, done * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIPCHK(hipMemcpyAsync(alpha, d_alpha, done * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(beta, d_beta, done * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    if (Q) {
      const size_t qb = (size_t)done * n3 * sizeof(z64);
      z64* dq = static_cast<z64*>(stage_out(c, Q, qb, "io.Qout"));
      launch_zxy_to_xyz(c->N, Qd, n3, dq, n3, done, c->stream);
      c->check_launch();
      c->sync();
      finish_out(c, Q, dq, qb);
    }
    c->sync();
    *k_done = done;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_lanczos_resume(lgw_ctx* c, int k0, int k, double* alpha, double* beta, lgw_c128* Q, int* k_done) {
  if (!c) return LGW_EINVAL;
  if (k0 < 1 || k < k0 || !alpha || !beta || !Q || !k_done) return set_err(c, LGW_EINVAL, "invalid arguments");
  try {
    const long n3 = c->n3;
    z64* Qd = c->buf<z64>("lz.Q", (size_t)k * n3);
    double* ab = c->buf<double>("lz.ab", 2 * (size_t)k);
    double* d_alpha = ab;
    double* d_beta = ab + k;
    // the prior state: q_0..q_{k0-1} and their coefficients
    std::vector<double> ha(k0), hb(k0);
    if (c->opts.mem == LGW_MEM_DEVICE) {
      HIPCHK(hipMemcpyAsync(ha.data(), alpha, k0 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(hb.data(), beta, k0 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      c->sync();
    } else {
      std::memcpy(ha.data(), alpha, k0 * sizeof(double));
      std::memcpy(hb.data(), beta, k0 * sizeof(double));
    }
    double amax0 = 0.0;
    for (int j = 0; j < k0; ++j) {
      if (!std::isfinite(ha[j]) || !std::isfinite(hb[j])) return set_err(c, LGW_ENAN, "non-finite Lanczos coefficient");
      if (j + 1 < k0) {
        if (!(hb[j] > 0.0)) return set_err(c, LGW_EINVAL, "the prior recursion broke down before k0");
        amax0 = std::max(amax0, std::abs(ha[j]));
      }
    }
    const z64* dq = static_cast<const z64*>(stage_in(c, Q, (size_t)k0 * n3 * sizeof(z64), "io.Qres"));
    int* d_flag = c->buf<int>("flag", 1);
    HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), c->stream));
    launch_finite_check(reinterpret_cast<const double*>(dq), 2 * (long)k0 * n3, d_flag, c->stream);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    if (hflag) return set_err(c, LGW_ENAN, "non-finite value in Q");
    launch_xyz_to_zxy(c->N, dq, n3, Qd, n3, k0, false, c->stream);
    if (k0 > 1) {
      h2d(c, d_alpha, ha.data(), (k0 - 1) * sizeof(double));
      h2d(c, d_beta, hb.data(), (k0 - 1) * sizeof(double));
    }
    // step k0 - 1 runs again (one chi0 application) to produce q_{k0}
    int done = 0;
    const lgw_status st = lanczos_core(c, k, Qd, nullptr, d_alpha, d_beta, &done, nullptr, k0 - 1, amax0);
    if (c->opts.mem == LGW_MEM_DEVICE) {
      HIPCHK(hipMemcpyAsync(alpha, d_alpha, done * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(beta, d_beta, done * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIPCHK(hipMemcpyAsync(alpha, d_alpha, done * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(beta, d_beta, done * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    const size_t qb = (size_t)done * n3 * sizeof(z64);
    z64* qo = static_cast<z64*>(stage_out(c, Q, qb, "io.Qout"));
    launch_zxy_to_xyz(c->N, Qd, n3, qo, n3, done, c->stream);
    c->check_launch();
    c->sync();
    finish_out(c, Q, qo, qb);
    c->sync();
    *k_done = done;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_lanczos_recycle(lgw_ctx* c, const lgw_c128* q0, int k, int n_w, const double* w, double* alpha,
                               double* beta, lgw_c128* Q, lgw_c128* E, int* k_done) {
  if (!c) return LGW_EINVAL;
  if (c->opts.model == 1) return set_err(c, LGW_EINVAL, "recycling works on the exact operator (model = 0)");
  if (k < 1 || n_w < 1 || !q0 || !w || !alpha || !beta || !E || !k_done)
    return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int i = 0; i < n_w; ++i)
    if (!std::isfinite(w[i]) || w[i] < 0.0)
      return set_err(c, LGW_EINVAL, "recycling frequencies are i*w with finite w >= 0");
  struct KeepOff {
    lgw_ctx* c;
    ~KeepOff() {
      c->keep_b = c->keep_f = nullptr;
      c->keep_n = c->keep_cap = 0;
    }
  } keep_off{c};
  try {
    const long n3 = c->n3;
    const int nv = c->nv, npw = c->npw;
    z64* Qd = c->buf<z64>("lz.Q", (size_t)k * n3);
    double* ab = c->buf<double>("lz.ab", 2 * (size_t)k);
    z64* Bk = c->buf<z64>("rc.Bk", (size_t)k * nv * npw);
    z64* Fk = c->buf<z64>("rc.Fk", (size_t)k * nv * npw);
    const lgw_status pre = lanczos_start(c, q0, Qd);
    if (pre != LGW_OK) return pre;
    c->keep_b = Bk;
    c->keep_f = Fk;
    c->keep_n = 0;
    c->keep_cap = k;
    int done = 0;
    const lgw_status st = lanczos_core(c, k, Qd, nullptr, ab, ab + k, &done);
    const int m = std::min(done, c->keep_n);
    c->keep_b = c->keep_f = nullptr;
    std::vector<z64> Eh;
    if (m > 0) recycle_E(c, m, Bk, Fk, n_w, w, Eh);
    std::vector<z64> e((size_t)n_w * k * k, z64{0, 0});
    for (int i = 0; i < n_w; ++i)
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) e[((size_t)i * k + a) * k + b] = Eh[((size_t)i * m + a) * m + b];
    if (c->opts.mem == LGW_MEM_DEVICE) {
      h2d(c, E, e.data(), e.size() * sizeof(z64));
      HIPCHK(hipMemcpyAsync(alpha, ab, done * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(beta, ab + k, done * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else {
      std::memcpy(E, e.data(), e.size() * sizeof(z64));
      HIPCHK(hipMemcpyAsync(alpha, ab, done * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(beta, ab + k, done * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    if (Q) {
      const size_t qb = (size_t)done * n3 * sizeof(z64);
      z64* dq = static_cast<z64*>(stage_out(c, Q, qb, "io.Qout"));
      launch_zxy_to_xyz(c->N, Qd, n3, dq, n3, done, c->stream);
      c->check_launch();
      c->sync();
      finish_out(c, Q, dq, qb);
    }
    c->sync();
    *k_done = done;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_lanczos_loss_vjp(lgw_ctx* c, const lgw_c128* q0, int k, int n_z, const lgw_c128* z, double* loss,
                                double* g_Vloc, int* k_done) {
  if (!c) return LGW_EINVAL;
  if (c->opts.model == 1) return set_err(c, LGW_EINVAL, "the adjoint is of the exact operator (model = 0)");
  if (k < 1 || n_z < 1 || !q0 || !z || !loss) return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int i = 0; i < n_z; ++i) {
    if (!std::isfinite(z[i].re) || !std::isfinite(z[i].im)) return set_err(c, LGW_ENAN, "non-finite frequency");
    if (z[i].re != 0.0 || z[i].im < 0.0)
      return set_err(c, LGW_EINVAL, "loss frequencies must be i*w with w >= 0 (imaginary axis)");
  }
  try {
    const long n3 = c->n3;
    z64* Qd = c->buf<z64>("lz.Q", (size_t)k * n3);
    z64* W0 = c->buf<z64>("ll.W0", (size_t)k * n3);
    double* ab = c->buf<double>("lz.ab", 2 * (size_t)k);
    const lgw_status pre = lanczos_start(c, q0, Qd);
    if (pre != LGW_OK) return pre;
    SolveTally tally;
    int m = 0;
    lgw_status st = lanczos_core(c, k, Qd, W0, ab, ab + k, &m);
    tally.add(c);
    const bool grad = g_Vloc != nullptr;
    z64* X = c->buf<z64>("ll.X", (size_t)m * n3);
    z64* Wz = c->buf<z64>("ll.Wz", (size_t)m * n3);
    z64* Gb = grad ? c->buf<z64>("ll.Gb", (size_t)m * n3) : nullptr;   // adjoint of Q
    double* gV = grad ? c->buf<double>("ll.gV", n3) : nullptr;
    z64* Et = c->buf<z64>("ll.E", (size_t)m * m);
    z64* part = c->buf<z64>("ll.part", (size_t)std::max<long>((long)m * m * 64,
                                                               (long)gemm_hn_slices(n3, m) * std::min(m, 64) * m));
    z64* Cm = c->buf<z64>("ll.Cm", (size_t)m * m);
    if (grad) {
      HIPCHK(hipMemsetAsync(Gb, 0, (size_t)m * n3 * sizeof(z64), c->stream));
      HIPCHK(hipMemsetAsync(gV, 0, n3 * sizeof(double), c->stream));
    }
    double L = 0.0;
    std::vector<z64> h((size_t)m * m), A((size_t)m * m), cm((size_t)m * m), cm2((size_t)m * m);
    for (int iz = 0; iz < n_z; ++iz) {
      // W = (eps(z) - 1) Q; the z = 0 products are the Lanczos recursion's own
      const z64* W = W0;
      if (z[iz].im != 0.0) {
        HIPCHK(hipMemcpyAsync(X, Qd, (size_t)m * n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
        vhalf_inplace(c, X, m, 1.0);
        c->tot_iters = c->tot_h = 0;
        st = worst(st, chi0_internal(c, m, X, 1, &z[iz], Wz, (long)m * n3));
        tally.add(c);
        vhalf_inplace(c, Wz, m, -1.0);
        W = Wz;
      }
      launch_gemm_hn_mfma(Qd, n3, m, W, n3, m, n3, Et, part, c->stream);   // Et[b][a] = <q_a, W_b>
      HIPCHK(hipMemcpyAsync(h.data(), Et, h.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      // I + E, made exactly Hermitian; log det and inverse through Cholesky
      std::vector<z64> C((size_t)m * m);
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
          const z64 eab = h[(size_t)b * m + a], eba = h[(size_t)a * m + b];
          C[(size_t)a * m + b] = z64{0.5 * (eab.x + eba.x) + (a == b ? 1.0 : 0.0), 0.5 * (eab.y - eba.y)};
        }
      double ld = 0.0;
      if (!hpd_logdet_inverse(C, m, ld, A))
        throw Fail{LGW_EBREAKDOWN, "I + E(z) is not positive definite"};
      L += ld;
      if (!grad) continue;
      // Cm[c][i] = -A[i][c]: block_sub then adds sum_i X_i A[i][c] to column c
      for (int cc = 0; cc < m; ++cc)
        for (int i = 0; i < m; ++i) {
          const z64 v = A[(size_t)i * m + cc];
          cm[(size_t)cc * m + i] = z64{-v.x, -v.y};
        }
      // adjoint of Q: dL/dQ = 2 sum_z (eps(z)-1) Q A_z  (A_z and eps(z)-1 Hermitian)
      for (size_t e = 0; e < cm.size(); ++e) cm2[e] = 2.0 * cm[e];
      h2d(c, Cm, cm2.data(), cm2.size() * sizeof(z64));
      launch_block_sub(Gb, n3, m, W, n3, m, Cm, n3, c->stream);
      h2d(c, Cm, cm.data(), cm.size() * sizeof(z64));   // stream-ordered after the launch above
      // explicit term tr[A_z Q^H d(eps(z)-1) Q]: chi0 VJP with x = v^1/2 Q A_z, g = -v^1/2 Q
      HIPCHK(hipMemsetAsync(X, 0, (size_t)m * n3 * sizeof(z64), c->stream));
      launch_block_sub(X, n3, m, Qd, n3, m, Cm, n3, c->stream);
      vhalf_inplace(c, X, m, 1.0);
      HIPCHK(hipMemcpyAsync(Wz, Qd, (size_t)m * n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
      vhalf_inplace(c, Wz, m, -1.0);
      c->tot_iters = c->tot_h = 0;
      st = worst(st, vjp_internal(c, m, X, 1, &z[iz], Wz, gV, true));
      tally.add(c);
    }
    if (grad && m > 1) {
      st = worst(st, lanczos_reverse(c, m, Qd, W0, ab, ab + k, Gb, gV, tally));
    }
    tally.store(c);
    if (c->opts.mem == LGW_MEM_DEVICE) h2d(c, loss, &L, sizeof(double));
    else *loss = L;
    if (grad) {
      double* d_out = static_cast<double*>(stage_out(c, g_Vloc, n3 * sizeof(double), "io.llg"));
      launch_real_zxy_to_xyz(c->N, gV, d_out, c->stream);
      c->check_launch();
      finish_out(c, g_Vloc, d_out, n3 * sizeof(double));
    }
    c->sync();
    if (k_done) *k_done = m;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_lanczos_project(lgw_ctx* c, const lgw_c128* q0, int k, int n_z, const lgw_c128* z, double* alpha,
                               double* beta, lgw_c128* Q, lgw_c128* E, int* k_done) {
  if (!c) return LGW_EINVAL;
  if (k < 1 || n_z < 1 || !q0 || !z || !alpha || !beta || !E || !k_done)
    return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int i = 0; i < n_z; ++i) {
    if (!std::isfinite(z[i].re) || !std::isfinite(z[i].im)) return set_err(c, LGW_ENAN, "non-finite frequency");
    if (z[i].re != 0.0 && z[i].im < 0.0) return set_err(c, LGW_EINVAL, "real-axis broadening must be >= 0");
  }
  try {
    const long n3 = c->n3;
    z64* Qd = c->buf<z64>("lz.Q", (size_t)k * n3);
    double* ab = c->buf<double>("lz.ab", 2 * (size_t)k);
    // W[iz][b] = (eps(z_iz) - 1) q_b, plane-major; z = 0 comes from the recursion
    z64* W = c->buf<z64>("lp.W", (size_t)n_z * k * n3);
    const lgw_status pre = lanczos_start(c, q0, Qd);
    if (pre != LGW_OK) return pre;
    int iz0 = -1;
    std::vector<lgw_c128> zw;
    std::vector<int> zw_idx;
    for (int i = 0; i < n_z; ++i) {
      if (z[i].re == 0.0 && z[i].im == 0.0 && iz0 < 0) iz0 = i;
      else {
        zw.push_back(z[i]);
        zw_idx.push_back(i);
      }
    }
    // workers: each projects chunks of finished Lanczos vectors on a twin's
    // stream; two run at once, so that one chunk's transforms (LDS-bound)
    // overlap another's vector and projector kernels (HBM-bound)
    const int kChunk = c->opts.multishift == 1 ? LGW_PROJECT_CHUNK_MS : LGW_PROJECT_CHUNK;
    constexpr int kWorkers = LGW_PROJECT_WORKERS;
    std::vector<lgw_ctx*> tws(kWorkers);
    for (int i = 0; i < kWorkers; ++i) {
      tws[i] = twin_of(c, i);
      tws[i]->prof = c->prof;
    }
    struct Job {
      int from, to;
    };
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job> queue;
    bool finished = false;
    std::vector<lgw_status> wst(kWorkers, LGW_OK);
    std::vector<std::string> werr(kWorkers);
    std::vector<SolveTally> wt(kWorkers);
    auto work = [&](int wi) {
      lgw_ctx* tw = tws[wi];
      try {
        HIPCHK(hipSetDevice(c->device));
        for (;;) {
          Job job;
          {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return !queue.empty() || finished; });
            if (queue.empty()) break;
            job = queue.front();
            queue.pop_front();
          }
          const int nb = job.to - job.from;
          if (nb <= 0 || zw.empty()) continue;
          z64* X = tw->buf<z64>("lp.X", (size_t)nb * n3);
          z64* D = tw->buf<z64>("lp.D", (size_t)zw.size() * nb * n3);
          HIPCHK(hipMemcpyAsync(X, Qd + (size_t)job.from * n3, (size_t)nb * n3 * sizeof(z64),
                                hipMemcpyDeviceToDevice, tw->stream));
          vhalf_inplace(tw, X, nb, 1.0);
          tw->tot_iters = tw->tot_h = 0;
          wst[wi] = worst(wst[wi], chi0_internal(tw, nb, X, (int)zw.size(), zw.data(), D, (long)nb * n3));
          wt[wi].add(tw);
          vhalf_inplace(tw, D, (int)zw.size() * nb, -1.0);
          for (size_t i = 0; i < zw.size(); ++i)
            HIPCHK(hipMemcpyAsync(W + ((size_t)zw_idx[i] * k + job.from) * n3, D + i * (size_t)nb * n3,
                                  (size_t)nb * n3 * sizeof(z64), hipMemcpyDeviceToDevice, tw->stream));
          tw->check_launch();
        }
        tw->sync();
      } catch (const Fail& f) {
        wst[wi] = f.st;
        werr[wi] = f.msg;
      }
    };
    std::vector<std::thread> workers;
    for (int i = 0; i < kWorkers; ++i) workers.emplace_back(work, i);
    auto join_all = [&] {
      {
        std::lock_guard<std::mutex> lk(mu);
        finished = true;
      }
      cv.notify_all();
      for (auto& t : workers) t.join();
    };
    int pushed = 0;
    // A chunk is handed over once the recursion's stream has written its
    // vectors (a host synchronisation between two steps).  No event of that
    // stream is shared with the workers: waiting on one, from another stream
    // or the host, breaks the HIP graph the recursion may be capturing then.
    auto push = [&](int upto) {
      c->sync();
      {
        std::lock_guard<std::mutex> lk(mu);
        queue.push_back(Job{pushed, upto});
      }
      cv.notify_one();
      pushed = upto;
    };
    // Chunks taper towards the end of the recursion (full ones while two remain,
    // then half of what remains, at least a quarter chunk), so that the work
    // left once the last vector exists is a small chunk.
    auto next_size = [&] {
      const int rem = k - pushed;
      return rem >= 2 * kChunk ? kChunk : std::max(std::max(1, kChunk / 4), rem / 2);
    };
    int m = 0;
    lgw_status st = LGW_OK;
    try {
      st = lanczos_core(c, k, Qd, iz0 >= 0 ? W + (size_t)iz0 * k * n3 : nullptr, ab, ab + k, &m,
                        [&](int avail) {
                          if (avail - pushed >= next_size()) push(avail);
                        });
      if (m > pushed) push(m);
    } catch (...) {
      join_all();
      throw;
    }
    SolveTally tally;
    tally.add(c);
    join_all();
    for (int i = 0; i < kWorkers; ++i)
      if (!werr[i].empty()) throw Fail{wst[i], werr[i]};
    for (int i = 0; i < kWorkers; ++i) {
      st = worst(st, wst[i]);
      const SolveTally& w = wt[i];
      tally.it.insert(tally.it.end(), w.it.begin(), w.it.end());
      tally.fl.insert(tally.fl.end(), w.fl.begin(), w.fl.end());
      tally.sw.insert(tally.sw.end(), w.sw.begin(), w.sw.end());
      tally.res.insert(tally.res.end(), w.res.begin(), w.res.end());
      tally.tot_it += w.tot_it;
      tally.tot_h += w.tot_h;
    }
    tally.store(c);
    if (c->prof) {   // the projection's launches ran on the twins
      for (lgw_ctx* tw : tws)
        for (int i = 0; i < 2 * LGW_K_FP32; ++i) {
          c->kt_ms[i] += tw->kt_ms[i];
          c->kt_bytes[i] += tw->kt_bytes[i];
          c->kt_launches[i] += tw->kt_launches[i];
          tw->kt_ms[i] = tw->kt_bytes[i] = 0;
          tw->kt_launches[i] = 0;
        }
    }
    // E[z][a][b] = <q_a, W[z][b]> for a, b < m (zero beyond): every frequency
    // in one product, Et[z * k + b][a] (rows b >= m of each W[z] are unused)
    const int pz = n_z * k;
    z64* Et = c->buf<z64>("lp.E", (size_t)pz * m);
    z64* part = c->buf<z64>("lp.part", (size_t)gemm_hn_slices(n3, pz) * std::min(m, 64) * pz);
    launch_gemm_hn_mfma(Qd, n3, m, W, n3, pz, n3, Et, part, c->stream);
    c->check_launch();
    std::vector<z64> h((size_t)pz * m);
    HIPCHK(hipMemcpyAsync(h.data(), Et, h.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    std::vector<z64> e((size_t)n_z * k * k, z64{0, 0});
    for (int i = 0; i < n_z; ++i)
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) e[((size_t)i * k + a) * k + b] = h[((size_t)i * k + b) * m + a];
    if (c->opts.mem == LGW_MEM_DEVICE) h2d(c, E, e.data(), e.size() * sizeof(z64));
    else std::memcpy(E, e.data(), e.size() * sizeof(z64));
    if (c->opts.mem == LGW_MEM_DEVICE) {
      HIPCHK(hipMemcpyAsync(alpha, ab, m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(beta, ab + k, m * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else {
      HIPCHK(hipMemcpyAsync(alpha, ab, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(beta, ab + k, m * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    if (Q) {
      const size_t qb = (size_t)m * n3 * sizeof(z64);
      z64* dq = static_cast<z64*>(stage_out(c, Q, qb, "io.Qout"));
      launch_zxy_to_xyz(c->N, Qd, n3, dq, n3, m, c->stream);
      c->check_launch();
      c->sync();
      finish_out(c, Q, dq, qb);
    }
    c->sync();
    *k_done = m;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_block_lanczos(lgw_ctx* c, int b, const lgw_c128* Q0, int nblk, lgw_c128* A, lgw_c128* B,
                             lgw_c128* Q, int* nblk_done) {
  if (!c) return LGW_EINVAL;
  if (b < 1 || b > 16 || nblk < 1 || !Q0 || !A || !B || !nblk_done)
    return set_err(c, LGW_EINVAL, "invalid arguments (block size 1..16)");
  try {
    const long n3 = c->n3;
    const int kmax = b * nblk;
    const z64* d_q0 = static_cast<const z64*>(stage_in(c, Q0, (size_t)b * n3 * sizeof(z64), "io.bq0"));
    int* d_flag = c->buf<int>("flag", 1);
    HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), c->stream));
    launch_finite_check(reinterpret_cast<const double*>(d_q0), 2 * (long)b * n3, d_flag, c->stream);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    if (hflag) return set_err(c, LGW_ENAN, "non-finite value in Q0");
    z64* Qd = c->buf<z64>("bl.Q", (size_t)(kmax + b) * n3);
    z64* W = c->buf<z64>("bl.W", (size_t)b * n3);
    z64* X1 = c->buf<z64>("bl.X1", (size_t)b * n3);
    z64* Cm = c->buf<z64>("bl.Cm", (size_t)b * (kmax + b));
    z64* part = c->buf<z64>("bl.part", (size_t)64 * (kmax + b) * b + 64 * (kmax + b));
    double* nrm = c->buf<double>("bl.nrm", 1);
    z64* Rcol = c->buf<z64>("bl.R", kmax + b);
    std::vector<z64> hA((size_t)nblk * b * b), hB((size_t)nblk * b * b);
    double wnorm_max = 0.0;
    unsigned long long rng = 0x9E3779B97F4A7C15ull;
    // orthonormalise the columns of blk (b grid vectors at rows `row0` of Qd)
    // against Qd[0, row0) and each other, twice-classical Gram-Schmidt per
    // column; returns R (upper triangular, row-major b x b)
    auto qr_block = [&](z64* blk, int row0, std::vector<z64>& R, double wfro) {
      R.assign((size_t)b * b, z64{0, 0});
      for (int k = 0; k < b; ++k) {
        z64* wk = blk + (size_t)k * n3;
        std::vector<z64> rk(k, z64{0, 0});
        for (int pass = 0; pass < 2; ++pass) {
          if (k > 0) {
            launch_dots(blk, n3, k, wk, n3, Rcol, part, c->stream);
            launch_gemv_sub(blk, n3, k, Rcol, wk, n3, c->stream);
            std::vector<z64> h(k);
            HIPCHK(hipMemcpyAsync(h.data(), Rcol, k * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
            c->sync();
            for (int i = 0; i < k; ++i) rk[i] = rk[i] + h[i];
          }
        }
        launch_norm(wk, n3, nrm, part, c->stream);
        double rkk = 0;
        HIPCHK(hipMemcpyAsync(&rkk, nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        c->sync();
        if (!(rkk > 1e-10 * wfro)) {
          // deflation: a fixed-seed random direction orthogonal to everything so far
          std::vector<z64> r(n3);
          for (long e = 0; e < n3; ++e) {
            rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
            r[e] = z64{(double)(rng >> 11) * 0x1.0p-53 - 0.5, 0.0};
          }
          h2d(c, wk, r.data(), n3 * sizeof(z64));
          const int m = row0 + k;
          for (int pass = 0; pass < 2; ++pass) {
            launch_dots(Qd, n3, row0, wk, n3, Rcol, part, c->stream);
            launch_gemv_sub(Qd, n3, row0, Rcol, wk, n3, c->stream);
            if (k > 0) {
              launch_dots(blk, n3, k, wk, n3, Rcol, part, c->stream);
              launch_gemv_sub(blk, n3, k, Rcol, wk, n3, c->stream);
            }
          }
          (void)m;
          launch_norm(wk, n3, nrm, part, c->stream);
          launch_scale_into(wk, nrm, wk, n3, c->stream);
          for (int i = 0; i <= k; ++i) R[(size_t)i * b + k] = z64{0, 0};
          for (int cc = k; cc < b; ++cc) R[(size_t)k * b + cc] = z64{0, 0};
          continue;
        }
        launch_scale_into(wk, nrm, wk, n3, c->stream);
        for (int i = 0; i < k; ++i) R[(size_t)i * b + k] = rk[i];
        R[(size_t)k * b + k] = z64{rkk, 0.0};
      }
    };
    // first block
    launch_xyz_to_zxy(c->N, d_q0, n3, Qd, n3, b, false, c->stream);
    {
      std::vector<z64> R0;
      qr_block(Qd, 0, R0, 1.0);
    }
    const lgw_c128 z0{0.0, 0.0};
    lgw_status st = LGW_OK;
    std::vector<int> all_it, all_fl, all_sw;
    std::vector<double> all_res;
    long long tot_it = 0, tot_h = 0;
    int done = 0;
    for (int j = 0; j < nblk; ++j) {
      z64* Qj = Qd + (size_t)j * b * n3;
      // W = -v^1/2 chi0(0) v^1/2 Q_j : the b columns in one batched solve
      HIPCHK(hipMemcpyAsync(X1, Qj, (size_t)b * n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
      vhalf_inplace(c, X1, b, 1.0);
      c->tot_iters = c->tot_h = 0;
      st = worst(st, chi0_internal(c, b, X1, 1, &z0, W, n3));
      all_it.insert(all_it.end(), c->st_iters.begin(), c->st_iters.end());
      all_fl.insert(all_fl.end(), c->st_flags.begin(), c->st_flags.end());
      all_sw.insert(all_sw.end(), c->st_sweeps.begin(), c->st_sweeps.end());
      all_res.insert(all_res.end(), c->st_res.begin(), c->st_res.end());
      tot_it += c->tot_iters;
      tot_h += c->tot_h;
      vhalf_inplace(c, W, b, -1.0);
      // A_j = Q_j^H W (Hermitian part)
      launch_gemm_hn(Qj, n3, b, W, n3, b, n3, Cm, part, c->stream);
      std::vector<z64> G((size_t)b * b);
      HIPCHK(hipMemcpyAsync(G.data(), Cm, G.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      z64* Aj = hA.data() + (size_t)j * b * b;
      for (int r = 0; r < b; ++r)
        for (int q = 0; q < b; ++q) {
          // G[q][r] = <Q_j[r], W[q]> = A[r][q]
          const z64 x = G[(size_t)q * b + r], y = G[(size_t)r * b + q];
          Aj[(size_t)r * b + q] = z64{0.5 * (x.x + y.x), 0.5 * (x.y - y.y)};
        }
      // W -= Q_j A_j + Q_{j-1} B_{j-1}^H
      {
        const int m = j > 0 ? 2 * b : b;
        std::vector<z64> cm((size_t)b * m);
        for (int q = 0; q < b; ++q) {
          if (j > 0) {
            const z64* Bp = hB.data() + (size_t)(j - 1) * b * b;
            for (int i = 0; i < b; ++i) cm[(size_t)q * m + i] = conj(Bp[(size_t)q * b + i]);
          }
          for (int i = 0; i < b; ++i) cm[(size_t)q * m + (m - b) + i] = Aj[(size_t)i * b + q];
        }
        h2d(c, Cm, cm.data(), cm.size() * sizeof(z64));
        launch_block_sub(W, n3, b, Qd + (size_t)(j > 0 ? j - 1 : 0) * b * n3, n3, m, Cm, n3, c->stream);
      }
      // full reorthogonalisation against every previous block, twice
      const int m = (j + 1) * b;
      for (int pass = 0; pass < 2; ++pass) {
        launch_gemm_hn(Qd, n3, m, W, n3, b, n3, Cm, part, c->stream);
        launch_block_sub(W, n3, b, Qd, n3, m, Cm, n3, c->stream);
      }
      // B_j from the QR of W; the new block goes to rows (j+1) b of Qd
      launch_gemm_hn(W, n3, b, W, n3, b, n3, Cm, part, c->stream);
      std::vector<z64> gw((size_t)b * b);
      HIPCHK(hipMemcpyAsync(gw.data(), Cm, gw.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      double wf = 0;
      for (int q = 0; q < b; ++q) wf += gw[(size_t)q * b + q].x;
      wf = std::sqrt(std::max(wf, 0.0));
      wnorm_max = std::max(wnorm_max, wf);
      z64* Qn = Qd + (size_t)(j + 1) * b * n3;
      HIPCHK(hipMemcpyAsync(Qn, W, (size_t)b * n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
      std::vector<z64> R;
      qr_block(Qn, (j + 1) * b, R, wf);
      std::memcpy(hB.data() + (size_t)j * b * b, R.data(), R.size() * sizeof(z64));
      done = j + 1;
      if (!(wf > 1e-14 * std::max(1.0, wnorm_max)) && wf == 0.0) break;
    }
    c->st_iters = all_it;
    c->st_flags = all_fl;
    c->st_sweeps = all_sw;
    c->st_res = all_res;
    c->tot_iters = tot_it;
    c->tot_h = tot_h;
    const size_t ab = (size_t)done * b * b * sizeof(z64);
    if (c->opts.mem == LGW_MEM_DEVICE) {
      h2d(c, A, hA.data(), ab);
      h2d(c, B, hB.data(), ab);
    } else {
      std::memcpy(A, hA.data(), ab);
      std::memcpy(B, hB.data(), ab);
    }
    if (Q) {
      const size_t qb = (size_t)done * b * n3 * sizeof(z64);
      z64* dq = static_cast<z64*>(stage_out(c, Q, qb, "io.bQout"));
      launch_zxy_to_xyz(c->N, Qd, n3, dq, n3, done * b, c->stream);
      c->check_launch();
      c->sync();
      finish_out(c, Q, dq, qb);
    }
    c->sync();
    *nblk_done = done;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

// (I + E)^-1 of one k x k complex matrix (row-major) by Gaussian elimination
// with partial pivoting on [I + E | I]; false when a pivot vanishes.
static bool inverse_i_plus(const z64* E, int k, z64* out) {
  const int w = 2 * k;
  std::vector<z64> a((size_t)k * w, z64{0, 0});
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < k; ++j) a[(size_t)i * w + j] = E[(size_t)i * k + j];
    a[(size_t)i * w + i].x += 1.0;
    a[(size_t)i * w + k + i] = z64{1.0, 0.0};
  }
  auto mag = [](z64 v) { return std::hypot(v.x, v.y); };
  for (int col = 0; col < k; ++col) {
    int piv = col;
    for (int i = col + 1; i < k; ++i)
      if (mag(a[(size_t)i * w + col]) > mag(a[(size_t)piv * w + col])) piv = i;
    const z64 pv = a[(size_t)piv * w + col];
    const double den = pv.x * pv.x + pv.y * pv.y;
    if (!(den > 0.0) || !std::isfinite(den)) return false;
    if (piv != col)
      for (int j = 0; j < w; ++j) std::swap(a[(size_t)piv * w + j], a[(size_t)col * w + j]);
    const z64 inv{pv.x / den, -pv.y / den};
    for (int j = 0; j < w; ++j) a[(size_t)col * w + j] = inv * a[(size_t)col * w + j];
    for (int i = 0; i < k; ++i) {
      if (i == col) continue;
      const z64 f = a[(size_t)i * w + col];
      if (f.x == 0.0 && f.y == 0.0) continue;
      for (int j = 0; j < w; ++j) a[(size_t)i * w + j] = a[(size_t)i * w + j] - f * a[(size_t)col * w + j];
    }
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) out[(size_t)i * k + j] = a[(size_t)i * w + k + j];
  return true;
}

lgw_status lgw_eps_inverse(lgw_ctx* c, int k, int n_z, const lgw_c128* E, lgw_c128* Einv) {
  if (!c) return LGW_EINVAL;
  if (k < 1 || n_z < 1 || !E || !Einv) return set_err(c, LGW_EINVAL, "invalid arguments");
  try {
    const size_t nb = (size_t)n_z * k * k * sizeof(z64);
    std::vector<z64> h((size_t)n_z * k * k), o((size_t)n_z * k * k);
    if (c->opts.mem == LGW_MEM_DEVICE) {
      HIPCHK(hipMemcpyAsync(h.data(), E, nb, hipMemcpyDeviceToHost, c->stream));
      c->sync();
    } else {
      std::memcpy(h.data(), E, nb);
    }
    for (size_t v = 0; v < h.size(); ++v)
      if (!std::isfinite(h[v].x) || !std::isfinite(h[v].y)) return set_err(c, LGW_ENAN, "non-finite value in E");
    for (int iz = 0; iz < n_z; ++iz)
      if (!inverse_i_plus(h.data() + (size_t)iz * k * k, k, o.data() + (size_t)iz * k * k))
        return set_err(c, LGW_EBREAKDOWN, "I + E(z) is singular");
    if (c->opts.mem == LGW_MEM_DEVICE) h2d(c, Einv, o.data(), nb);
    else std::memcpy(Einv, o.data(), nb);
    return LGW_OK;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_ritz_values(lgw_ctx* c, int k, const double* alpha, const double* beta, double* theta) {
  if (!c) return LGW_EINVAL;
  if (k < 1 || !alpha || !theta || (k > 1 && !beta)) return set_err(c, LGW_EINVAL, "invalid arguments");
  try {
    std::vector<double> a(k), b(k > 1 ? k - 1 : 1, 0.0);
    if (c->opts.mem == LGW_MEM_DEVICE) {
      HIPCHK(hipMemcpyAsync(a.data(), alpha, k * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      if (k > 1) HIPCHK(hipMemcpyAsync(b.data(), beta, (k - 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      c->sync();
    } else {
      std::memcpy(a.data(), alpha, k * sizeof(double));
      if (k > 1) std::memcpy(b.data(), beta, (k - 1) * sizeof(double));
    }
    std::vector<std::complex<double>> T((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
      if (!std::isfinite(a[i]) || (i + 1 < k && !std::isfinite(b[i])))
        return set_err(c, LGW_ENAN, "non-finite Lanczos coefficient");
      T[(size_t)i * k + i] = a[i];
      if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = b[i];
    }
    std::vector<double> w;
    std::vector<std::complex<double>> V;
    herm_eig(k, T.data(), w, V);
    std::memcpy(theta, w.data(), k * sizeof(double));
    return LGW_OK;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_project(lgw_ctx* c, int k, const lgw_c128* Q, int n_z, const lgw_c128* z, lgw_c128* E) {
  if (!c) return LGW_EINVAL;
  if (k < 1 || n_z < 1 || !Q || !z || !E) return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int i = 0; i < n_z; ++i) {
    if (!std::isfinite(z[i].re) || !std::isfinite(z[i].im)) return set_err(c, LGW_ENAN, "non-finite frequency");
    if (z[i].re != 0.0 && z[i].im < 0.0) return set_err(c, LGW_EINVAL, "real-axis broadening must be >= 0");
  }
  try {
    const long n3 = c->n3;
    const z64* dQ = static_cast<const z64*>(stage_in(c, Q, (size_t)k * n3 * sizeof(z64), "io.Qin"));
    z64* Qz = c->buf<z64>("pj.Q", (size_t)k * n3);
    launch_xyz_to_zxy(c->N, dQ, n3, Qz, n3, k, false, c->stream);
    std::vector<z64> e;
    const lgw_status st = project_internal(c, k, Qz, n_z, z, e);
    if (c->opts.mem == LGW_MEM_DEVICE)
      h2d(c, E, e.data(), e.size() * sizeof(z64));
    else
      std::memcpy(E, e.data(), e.size() * sizeof(z64));
    c->sync();
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_sigma_traces(lgw_ctx* c, int e, double delta, double alpha, int k, const lgw_c128* Q, int n_w,
                            const double* w, double* sigma_N, double* sigma_N0, double* sigma_A) {
  if (!c) return LGW_EINVAL;
  if (e < 0 || e >= c->nv) return set_err(c, LGW_EINVAL, "e must index a valence state (0 .. n_v - 1)");
  if (!std::isfinite(delta)) return set_err(c, LGW_ENAN, "non-finite delta");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return set_err(c, LGW_EINVAL, "alpha must be positive");
  if (k < 1 || !Q || n_w < 0 || !sigma_A || (n_w > 0 && (!w || !sigma_N || !sigma_N0)))
    return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int i = 0; i < n_w; ++i)
    if (!(w[i] > 0.0) || !std::isfinite(w[i])) return set_err(c, LGW_EINVAL, "frequencies must be positive");
  if (c->opts.model == 1) return set_err(c, LGW_EINVAL, "the self-energy traces need the exact operator (model = 0)");
  try {
    const long n3 = c->n3;
    const int npw = c->npw, nv = c->nv;
    const double s = c->eps[e] + delta;
    const z64* dQ = static_cast<const z64*>(stage_in(c, Q, (size_t)k * n3 * sizeof(z64), "io.Qin"));
    z64* Qz = c->buf<z64>("sg.Q", (size_t)k * n3);
    launch_xyz_to_zxy(c->N, dQ, n3, Qz, n3, k, false, c->stream);
    // W(z) = (I + E(z))^-1 - I at z = 0 and every i w (Sec. IV: eps inverted in the basis)
    std::vector<lgw_c128> zl(1 + n_w, lgw_c128{0.0, 0.0});
    for (int i = 0; i < n_w; ++i) zl[1 + i] = lgw_c128{0.0, w[i]};
    std::vector<z64> E;
    lgw_status st = project_internal(c, k, Qz, 1 + n_w, zl.data(), E);
    std::vector<std::vector<z64>> W(1 + n_w);
    for (int i = 0; i <= n_w; ++i) {
      std::vector<z64> C((size_t)k * k);
      for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
          const z64 x = E[((size_t)i * k + a) * k + b], y = E[((size_t)i * k + b) * k + a];
          C[(size_t)a * k + b] = z64{0.5 * (x.x + y.x) + (a == b ? 1.0 : 0.0), 0.5 * (x.y - y.y)};
        }
      double ld = 0.0;
      if (!hpd_logdet_inverse(C, k, ld, W[i])) throw Fail{LGW_EBREAKDOWN, "I + E(i w) is not positive definite"};
      for (int a = 0; a < k; ++a) W[i][(size_t)a * k + a].x -= 1.0;
    }
    // right-hand sides g_l = Gather(conj(psi_e) v^1/2 q_l) (Eq. (kge))
    z64* X = c->buf<z64>("sg.X", (size_t)k * n3);
    HIPCHK(hipMemcpyAsync(X, Qz, (size_t)k * n3 * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
    vhalf_inplace(c, X, k, 1.0);
    z64* G = c->buf<z64>("sg.G", (size_t)k * npw);
    gather_products(c, c->d_u.as<z64>() + (size_t)e * n3, 1, X, k, G, 1.0);
    const double idv = 1.0 / c->dV;
    // K(i w)[l'][l] = (1/dV) g_l'^H (H - s)((H - s)^2 + w^2)^-1 g_l: all w from one
    // shift-Lanczos recursion per column (Sec. VI), shifts s -+ i w, no projector
    std::vector<std::vector<z64>> K(n_w);
    if (n_w > 0) {
      z64* F = c->buf<z64>("sg.F", (size_t)n_w * k * npw);   // F[i][l] = 2 (H - s)((H - s)^2 + w_i^2)^-1 g_l
      {
        ResolventScope scope(c);
        std::vector<double> base(k, s);
        std::vector<lgw_c128> zw(n_w);
        for (int i = 0; i < n_w; ++i) zw[i] = lgw_c128{0.0, w[i]};
        st = worst(st, multishift(c, G, k, n_w, zw.data(), F, base.data()));
      }
      z64* Ct = c->buf<z64>("sg.Ct", (size_t)n_w * k * k);
      z64* part = c->buf<z64>("sg.part", (size_t)gemm_hn_slices(npw, n_w * k) * std::min(k, 64) * n_w * k);
      launch_gemm_hn_mfma(G, npw, k, F, npw, n_w * k, npw, Ct, part, c->stream);   // Ct[i k + l][l'] = g_l'^H F[i][l]
      c->check_launch();
      std::vector<z64> h((size_t)n_w * k * k);
      HIPCHK(hipMemcpyAsync(h.data(), Ct, h.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      for (int i = 0; i < n_w; ++i) {
        K[i].assign((size_t)k * k, z64{0, 0});
        for (int l = 0; l < k; ++l)
          for (int lp = 0; lp < k; ++lp) K[i][(size_t)lp * k + l] = (0.5 * idv) * h[((size_t)i * k + l) * k + lp];
      }
    }
    // Sigma_A (Eqs. (he), (khe)): the conduction states, all above s, through
    // (H - s + a) y = P_c g on the conduction space; each valence state v
    // through its weight F(e_v - s) on the valence block
    std::vector<z64> KA((size_t)k * k, z64{0, 0});
    {
      z64* PG = c->buf<z64>("sg.PG", (size_t)k * npw);
      HIPCHK(hipMemcpyAsync(PG, G, (size_t)k * npw * sizeof(z64), hipMemcpyDeviceToDevice, c->stream));
      proj<double>(c, PG, npw, nullptr, k);
      std::vector<int> bidx(k);
      for (int l = 0; l < k; ++l) bidx[l] = l;
      std::vector<z64> sh(k, z64{s - alpha, 0.0});
      z64* YA = c->buf<z64>("sg.YA", (size_t)k * npw);
      SolveOut so;
      c->tot_iters = c->tot_h = 0;
      solve(c, K_CGLIN, PG, bidx, sh, {}, YA, so);
      for (int l = 0; l < k; ++l) {
        if (so.flags[l] == FLAG_BREAK) st = worst(st, LGW_EBREAKDOWN);
        else if (so.flags[l] != FLAG_CONV) st = worst(st, LGW_ENOCONV);
      }
      z64* Ct = c->buf<z64>("sg.CA", (size_t)k * k + (size_t)k * nv);
      z64* part = c->buf<z64>("sg.partA", (size_t)64 * k * std::max(k, nv) + 64);
      launch_gemm_hn(G, npw, k, YA, npw, k, npw, Ct, part, c->stream);                          // [l][l'] = g_l'^H y_l
      launch_gemm_hn(c->d_Phi.as<z64>(), npw, nv, G, npw, k, npw, Ct + (size_t)k * k, part, c->stream);   // [l][v] = u_v^H g_l
      c->check_launch();
      std::vector<z64> h((size_t)k * k + (size_t)k * nv);
      HIPCHK(hipMemcpyAsync(h.data(), Ct, h.size() * sizeof(z64), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      const z64* cm = h.data() + (size_t)k * k;
      std::vector<double> Fv(nv);
      for (int v = 0; v < nv; ++v) Fv[v] = lorentz_F(c->eps[v] - s, alpha);
      for (int lp = 0; lp < k; ++lp)
        for (int l = 0; l < k; ++l) {
          z64 acc = (0.5 * alpha) * h[(size_t)l * k + lp];
          for (int v = 0; v < nv; ++v) acc = acc + Fv[v] * cmulc(cm[(size_t)lp * nv + v], cm[(size_t)l * nv + v]);
          KA[(size_t)lp * k + l] = idv * acc;
        }
    }
    for (int i = 0; i < n_w; ++i) {
      sigma_N[i] = re_trace_prod(W[1 + i], K[i], k);
      sigma_N0[i] = alpha * alpha / (w[i] * w[i] + alpha * alpha) * re_trace_prod(W[0], K[i], k);
    }
    *sigma_A = re_trace_prod(W[0], KA, k);
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_sigma_residues(lgw_ctx* c, int e, double delta, int k_p, double* sigma_P, int* n_poles) {
  if (!c) return LGW_EINVAL;
  if (e < 0 || e >= c->nv) return set_err(c, LGW_EINVAL, "e must index a valence state (0 .. n_v - 1)");
  if (!std::isfinite(delta)) return set_err(c, LGW_ENAN, "non-finite delta");
  if (k_p < 1 || !sigma_P) return set_err(c, LGW_EINVAL, "invalid arguments");
  if (c->opts.model == 1) return set_err(c, LGW_EINVAL, "the residues need the exact operator (model = 0)");
  try {
    const long n3 = c->n3;
    const double s = c->eps[e] + delta;
    struct FreqScope {
      lgw_ctx* c;
      ~FreqScope() { c->lz_z = z64{0.0, 0.0}; }
    } fscope{c};
    double total = 0.0;
    int np = 0;
    lgw_status st = LGW_OK;
    z64* Qd = c->buf<z64>("sp.Q", (size_t)k_p * n3);
    double* ab = c->buf<double>("sp.ab", 2 * (size_t)k_p);
    z64* pv = c->buf<z64>("sp.p", n3);
    z64* part = c->buf<z64>("sp.part", 64);
    double* d_nrm = c->buf<double>("sp.nrm", 1);
    for (int v = 0; v < c->nv; ++v) {
      // poles of Eq. (pe): valence states above s, half weight on s (Theta(0) = 1/2)
      const double om = c->eps[v] - s;
      const double th = om > 1e-12 ? 1.0 : (om >= -1e-12 ? 0.5 : 0.0);
      if (th == 0.0) continue;
      ++np;
      // seed v^1/2 |v* e>: conj(psi_v) psi_e on the grid, then v^1/2
      launch_mul(pv, c->d_u.as<z64>() + (size_t)v * n3, c->d_psi.as<z64>() + (size_t)e * n3, n3, c->stream);
      vhalf_inplace(c, pv, 1, 1.0);
      launch_norm(pv, n3, d_nrm, part, c->stream);
      double nrm = 0.0;
      HIPCHK(hipMemcpyAsync(&nrm, d_nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      if (!(nrm > 0.0)) continue;   // a vanishing pair function has no residue
      launch_scale_into(pv, d_nrm, Qd, n3, c->stream);
      // Lanczos on eps(om) - 1 at the real frequency om (no broadening)
      c->lz_z = z64{th == 1.0 ? om : 0.0, 0.0};
      int done = 0;
      st = worst(st, lanczos_core(c, k_p, Qd, nullptr, ab, ab + k_p, &done));
      std::vector<double> h(2 * (size_t)k_p);
      HIPCHK(hipMemcpyAsync(h.data(), ab, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      c->sync();
      // |p|^2 dV [(I + T)^-1]_00 - |p|^2 dV: (T + 1) y = e_1
      std::vector<z64> y(done);
      tri_shift_solve(h.data(), h.data() + k_p, done, z64{-1.0, 0.0}, 1.0, y.data());
      const double elem = c->dV * nrm * nrm * (y[0].x - 1.0);
      total -= th * elem;
    }
    *sigma_P = total;
    if (n_poles) *n_poles = np;
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    c->lz_z = z64{0.0, 0.0};
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_chi0_apply_vjp(lgw_ctx* c, int n_rhs, const lgw_c128* dV, int n_z, const lgw_c128* z,
                              const lgw_c128* g_dn, lgw_c128* g_dV, double* g_Vloc) {
  if (!c) return LGW_EINVAL;
  if (c->opts.model == 1) return set_err(c, LGW_EINVAL, "the adjoint is of the exact operator (model = 0)");
  if (n_rhs < 1 || n_z < 1 || !dV || !z || !g_dn || (!g_dV && !g_Vloc))
    return set_err(c, LGW_EINVAL, "invalid arguments");
  for (int k = 0; k < n_z; ++k)
    if (!std::isfinite(z[k].re) || !std::isfinite(z[k].im)) return set_err(c, LGW_ENAN, "non-finite frequency");
  try {
    const long n3 = c->n3;
    const z64* d_in = static_cast<const z64*>(stage_in(c, dV, (size_t)n_rhs * n3 * sizeof(z64), "io.vin"));
    const z64* d_g = static_cast<const z64*>(stage_in(c, g_dn, (size_t)n_z * n_rhs * n3 * sizeof(z64), "io.vg"));
    int* d_flag = c->buf<int>("flag", 1);
    HIPCHK(hipMemsetAsync(d_flag, 0, sizeof(int), c->stream));
    launch_finite_check(reinterpret_cast<const double*>(d_in), 2 * (long)n_rhs * n3, d_flag, c->stream);
    launch_finite_check(reinterpret_cast<const double*>(d_g), 2 * (long)n_z * n_rhs * n3, d_flag, c->stream);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    if (hflag) return set_err(c, LGW_ENAN, "non-finite value in dV or g_dn");
    z64* X = c->buf<z64>("vi.X", (size_t)n_rhs * n3);
    z64* G = c->buf<z64>("vi.G", (size_t)n_z * n_rhs * n3);
    launch_xyz_to_zxy(c->N, d_in, n3, X, n3, n_rhs, false, c->stream);
    launch_xyz_to_zxy(c->N, d_g, n3, G, n3, n_z * n_rhs, false, c->stream);
    lgw_status st = LGW_OK;
    c->tot_iters = c->tot_h = 0;
    if (g_dV) {
      // dL/d dV = sum_z chi0(z)^H g = sum_z chi0(conj z) g
      z64* acc = c->buf<z64>("vi.acc", (size_t)n_rhs * n3);
      z64* one = c->buf<z64>("vi.one", (size_t)n_rhs * n3);
      HIPCHK(hipMemsetAsync(acc, 0, (size_t)n_rhs * n3 * sizeof(z64), c->stream));
      for (int k = 0; k < n_z; ++k) {
        const lgw_c128 zb{z[k].re, -z[k].im};
        st = worst(st, chi0_internal(c, n_rhs, G + (size_t)k * n_rhs * n3, 1, &zb, one, (long)n_rhs * n3));
        launch_add(acc, acc, one, (long)n_rhs * n3, c->stream);
      }
      const size_t ob = (size_t)n_rhs * n3 * sizeof(z64);
      z64* d_out = static_cast<z64*>(stage_out(c, g_dV, ob, "io.vgx"));
      launch_zxy_to_xyz(c->N, acc, n3, d_out, n3, n_rhs, c->stream);
      c->sync();
      finish_out(c, g_dV, d_out, ob);
    }
    if (g_Vloc) {
      double* gV = c->buf<double>("vi.gV", n3);
      st = worst(st, vjp_internal(c, n_rhs, X, n_z, z, G, gV));
      // plane-major -> [x][y][z]
      double* d_out = static_cast<double*>(stage_out(c, g_Vloc, n3 * sizeof(double), "io.vgv"));
      launch_real_zxy_to_xyz(c->N, gV, d_out, c->stream);
      c->check_launch();
      finish_out(c, g_Vloc, d_out, n3 * sizeof(double));
    }
    c->check_launch();
    c->sync();
    if (st != LGW_OK) c->err = "some Sternheimer solves did not converge";
    return st;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_hpsi(lgw_ctx* c, int n, lgw_c128 shift, const lgw_c128* x, lgw_c128* y) {
  if (!c) return LGW_EINVAL;
  if (n < 0 || (n > 0 && (!x || !y))) return set_err(c, LGW_EINVAL, "invalid arguments");
  if (n == 0) return LGW_OK;
  try {
    const int npw = c->npw;
    const size_t bytes = (size_t)n * npw * sizeof(z64);
    const z64* dx = static_cast<const z64*>(stage_in(c, x, bytes, "io.hx"));
    z64* dy = static_cast<z64*>(stage_out(c, y, bytes, "io.hy"));
    const long ldt = (long)c->N * c->ncols;
    std::vector<z64> sh(n, z64{shift.re, shift.im});
    if (c->opts.precision == LGW_FP64) {
      z64* d_sh = c->buf<z64>("h.sh", n);
      z64* Tb = c->buf<z64>("h.Tb", (size_t)n * ldt);
      h2d(c, d_sh, sh.data(), n * sizeof(z64));
      happly<double>(c, dx, npw, dy, npw, d_sh, nullptr, 0, nullptr, Tb, nullptr, n);
    } else {
      z32* x32 = c->buf<z32>("h.x32", (size_t)n * npw);
      z32* y32 = c->buf<z32>("h.y32", (size_t)n * npw);
      z32* Tb = c->buf<z32>("h.Tb32", (size_t)n * ldt);
      z32* d_sh = c->buf<z32>("h.sh32", n);
      std::vector<z32> s32(n, z32{(float)shift.re, (float)shift.im});
      h2d(c, d_sh, s32.data(), n * sizeof(z32));
      launch_cvt_64_32(dx, x32, (long)n * npw, c->stream);
      happly<float>(c, x32, npw, y32, npw, d_sh, nullptr, 0, nullptr, Tb, nullptr, n);
      double* one = c->buf<double>("h.one", n);
      std::vector<double> h1(n, 1.0);
      h2d(c, one, h1.data(), n * sizeof(double));
      HIPCHK(hipMemsetAsync(dy, 0, bytes, c->stream));
      launch_cvt_32_64_axpy(y32, dy, one, nullptr, npw, npw, n, c->stream);
    }
    c->check_launch();
    c->sync();
    finish_out(c, y, dy, bytes);
    return LGW_OK;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_hpsi_noalloc(lgw_ctx* c, int n, lgw_c128 shift, const lgw_c128* x, lgw_c128* y) {
  if (!c) return LGW_EINVAL;
  if (n < 0 || (n > 0 && (!x || !y))) return set_err(c, LGW_EINVAL, "invalid arguments");
  if (c->opts.mem != LGW_MEM_DEVICE)
    return set_err(c, LGW_EINVAL, "lgw_hpsi_noalloc needs a device-memory context (opts.mem = LGW_MEM_DEVICE)");
  if (n == 0) return LGW_OK;
  const long npw = c->npw, ldt = (long)c->N * c->ncols;
  const size_t need = hpsi_noalloc_bytes(c->opts.precision, n, npw, ldt);
  if (need > kScratchBytes) {
    long nmax = 0;
    while (hpsi_noalloc_bytes(c->opts.precision, nmax + 1, npw, ldt) <= kScratchBytes) ++nmax;
    return set_err(c, LGW_EINVAL, "lgw_hpsi_noalloc: " + std::to_string(n) + " vectors need " +
                                      std::to_string(need) + " bytes of scratch; the fixed scratch holds " +
                                      std::to_string(kScratchBytes) + " bytes (at most " + std::to_string(nmax) +
                                      " vectors on this grid and precision)");
  }
  char* base = scratch_of(c->device);
  if (!base)
    return set_err(c, LGW_EDEVICE, c->scratch_err.empty() ? "no scratch address for this device" : c->scratch_err);
  try {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const z64* dx = reinterpret_cast<const z64*>(x);
    z64* dy = reinterpret_cast<z64*>(y);
    if (c->opts.precision == LGW_FP64) {
      z64* sh = reinterpret_cast<z64*>(base);
      z64* Tb = reinterpret_cast<z64*>(base + al(n * sizeof(z64)));
      launch_fill<double>(sh, z64{shift.re, shift.im}, n, c->stream);
      launch_zinv<double>(c->geom, tw_of<double>(c), dx, npw, Tb, ldt, 1.0, nullptr, n, c->stream);
      launch_plane_hv<double>(c->geom, tw_of<double>(c), Tb, ldt, vt_of<double>(c), nullptr, n, c->stream,
                              plane_variant_for(c->N, false, n, c->opts.autotune != 0));
      launch_zfwd<double>(c->geom, tw_of<double>(c), Tb, ldt, 1.0 / (double)c->n3, dx, npw, sh, nullptr, 0,
                          nullptr, dy, npw, nullptr, n, c->stream, nullptr, CgDot<double>{});
    } else {
      char* p = base;
      z32* sh = reinterpret_cast<z32*>(p);
      p += al(n * sizeof(z32));
      z32* Tb = reinterpret_cast<z32*>(p);
      p += al(n * ldt * sizeof(z32));
      z32* x32 = reinterpret_cast<z32*>(p);
      p += al(n * npw * sizeof(z32));
      z32* y32 = reinterpret_cast<z32*>(p);
      launch_fill<float>(sh, z32{(float)shift.re, (float)shift.im}, n, c->stream);
      launch_cvt_64_32(dx, x32, (long)n * npw, c->stream);
      launch_zinv<float>(c->geom, tw_of<float>(c), x32, npw, Tb, ldt, 1.0f, nullptr, n, c->stream);
      launch_plane_hv<float>(c->geom, tw_of<float>(c), Tb, ldt, vt_of<float>(c), nullptr, n, c->stream,
                             plane_variant_for(c->N, true, n, c->opts.autotune != 0));
      launch_zfwd<float>(c->geom, tw_of<float>(c), Tb, ldt, (float)(1.0 / (double)c->n3), x32, npw, sh, nullptr,
                         0, nullptr, y32, npw, nullptr, n, c->stream, nullptr, CgDot<float>{});
      launch_cvt_32_64(y32, dy, (long)n * npw, c->stream);
    }
    c->check_launch();
    c->tot_h += n;
    return LGW_OK;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_vhalf(lgw_ctx* c, int n, const lgw_c128* x, lgw_c128* y) {
  if (!c) return LGW_EINVAL;
  if (n < 0 || (n > 0 && (!x || !y))) return set_err(c, LGW_EINVAL, "invalid arguments");
  if (n == 0) return LGW_OK;
  try {
    const long n3 = c->n3;
    const size_t bytes = (size_t)n * n3 * sizeof(z64);
    const z64* dx = static_cast<const z64*>(stage_in(c, x, bytes, "io.vx"));
    z64* dy = static_cast<z64*>(stage_out(c, y, bytes, "io.vy"));
    z64* G = c->buf<z64>("v.G", (size_t)n * n3);
    launch_xyz_to_zxy(c->N, dx, n3, G, n3, n, false, c->stream);
    vhalf_inplace(c, G, n, 1.0);
    launch_zxy_to_xyz(c->N, G, n3, dy, n3, n, c->stream);
    c->check_launch();
    c->sync();
    finish_out(c, y, dy, bytes);
    return LGW_OK;
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
}

lgw_status lgw_get_info(const lgw_ctx* c, lgw_info* out) {
  if (!c || !out) return LGW_EINVAL;
  out->N = c->N;
  out->npw = c->npw;
  out->ncols = c->ncols;
  out->n_v = c->nv;
  out->omega = c->omega;
  return LGW_OK;
}

lgw_status lgw_sphere(const lgw_ctx* c, int* m) {
  if (!c || !m) return LGW_EINVAL;
  std::memcpy(m, c->m.data(), c->m.size() * sizeof(int));
  return LGW_OK;
}

lgw_status lgw_get_stats(const lgw_ctx* c, lgw_stats* out) {
  if (!c || !out) return LGW_EINVAL;
  out->n_solves = (int)c->st_iters.size();
  out->iters = c->st_iters.data();
  out->rel_resid = c->st_res.data();
  out->refine_sweeps = c->st_sweeps.data();
  out->flags = c->st_flags.data();
  out->total_iters = c->tot_iters;
  out->total_happly = c->tot_h;
  return LGW_OK;
}

lgw_status lgw_profile(lgw_ctx* c, int enable) {
  if (!c) return LGW_EINVAL;
  try {
    c->sync();
  } catch (const Fail& f) {
    return set_err(c, f.st, f.msg);
  }
  c->prof = enable != 0;
  for (int k = 0; k < 2 * LGW_K_FP32; ++k) {
    c->kt_ms[k] = 0;
    c->kt_bytes[k] = 0;
    c->kt_launches[k] = 0;
  }
  return LGW_OK;
}

lgw_status lgw_kernel_timing(const lgw_ctx* c, int kernel, lgw_timing* out) {
  if (!c || !out || kernel < 0 || kernel >= 2 * LGW_K_FP32 || kernel % LGW_K_FP32 >= LGW_NKERNELS)
    return LGW_EINVAL;
  out->launches = c->kt_launches[kernel];
  out->total_ms = c->kt_ms[kernel];
  out->model_bytes = c->kt_bytes[kernel];
  return LGW_OK;
}

const char* lgw_last_error(const lgw_ctx* c) { return c ? c->err.c_str() : g_setup_err.c_str(); }

lgw_status lgw_tune_info(const lgw_ctx* c, int precision, int nsys, int* variant, int* threads, int* pad,
                         double* us) {
  if (!c || !variant || (precision != LGW_FP64 && precision != LGW_MIXED) || nsys < 1) return LGW_EINVAL;
  const bool f32 = precision == LGW_MIXED;
  const int v = plane_variant_for(c->N, f32, nsys, c->opts.autotune != 0);
  *variant = v;
  int nt = 0, pd = 0;
  plane_variant_shape(c->N, v, &nt, &pd);
  if (threads) *threads = nt;
  if (pad) *pad = pd;
  if (us) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(c->N, f32 ? 1 : 0, tune_bucket(nsys)));
    for (int i = 0; i < 4; ++i) us[i] = it == g_tune.end() ? 0.0 : it->second.us[i];
  }
  return LGW_OK;
}

void lgw_free(lgw_ctx* c) {
  if (!c) return;
  hipStream_t s = c->stream;
  const bool own = c->own_stream;
  if (s) (void)hipStreamSynchronize(s);
  try {
    c->harvest();
  } catch (const Fail&) {
  }
  c->drop_graphs();
  c->ws.clear();
  c->stream = nullptr;
  delete c;
  if (own && s) (void)hipStreamDestroy(s);
}

}  // extern "C"
