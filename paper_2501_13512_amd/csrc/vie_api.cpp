// C ABI of libvie: context, problem set-up (block plan, spectra cache),
// products, preconditioner and the block-preconditioned BiCGSTAB driver.
// See include/vie.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <shared_mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "api_lock.h"
#include "kernels.h"
#include "vie.h"

using vie::KBatch;
using vie::KState;
using vie::MvmBatch;

namespace vie {
// Graph capture takes this exclusively; allocation, frees, stream and event
// creation or destruction and device-wide synchronisation take it shared.
// HIP refuses such calls while any thread captures, so with concurrent
// solves (the request server's slots) they must not overlap a capture.
std::shared_mutex& api_mutex() {
  static std::shared_mutex m;
  return m;
}
}  // namespace vie

namespace {

using ApiShared = vie::ApiShared;

thread_local std::string g_last_error;
// Device bytes whose hipFree failed (kept counted against every budget), and
// whether a free failed on this thread since the flag was last cleared.
std::atomic<size_t> g_unfreed_bytes{0};
thread_local bool t_free_failed = false;
std::string vie_last_error_str() { return g_last_error; }

struct VieError : std::runtime_error {
  vie_status code;
  VieError(vie_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(vie_status c, const std::string& m) { throw VieError(c, m); }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    fail(VIE_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
  fail(VIE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  void alloc(size_t n) {
    reset();
    if (n == 0) return;
    hipError_t e;
    {
      ApiShared api;
      e = hipMalloc(&p, n);
    }
    hip_check(e, "hipMalloc");
    bytes = n;
  }
  // Stream-ordered: work on `s` sees the zeros (the null stream is not
  // ordered with the library's non-blocking streams).
  void zero(hipStream_t s) {
    if (p) hip_check(hipMemsetAsync(p, 0, bytes, s), "hipMemsetAsync");
  }
  void reset() {
    if (p) {
      hipError_t e;
      {
        ApiShared api;
        e = hipFree(p);
      }
      if (e != hipSuccess) {
        // the memory stays held: keep it counted against every budget, flag
        // the failure for the caller, and clear the error so that it is not
        // reported by the next unrelated launch check
        (void)hipGetLastError();
        g_unfreed_bytes += bytes;
        t_free_failed = true;
      }
    }
    p = nullptr;
    bytes = 0;
  }
  ~DevBuf() { reset(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <class T>
void upload(DevBuf& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(h.size() * sizeof(T));
  if (h.empty()) return;
  // ordered on s and complete before h can go away
  hip_check(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
  hip_check(hipStreamSynchronize(s), "upload");
}

template <class F>
vie_status guarded(F&& f) {
  try {
    vie_status s = f();
    if (s == VIE_OK) g_last_error.clear();
    return s;
  } catch (const VieError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return VIE_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return VIE_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown internal error";
    return VIE_EINTERNAL;
  }
}

// exp(-2 pi i t / L) with exact values on the quadrant points.
void cis_neg(long t, long L, double* c, double* s) {
  t %= L;
  const long q = (4 * t) / L;
  const long r4 = 4 * t - q * L;  // angle = (q + r4 / L) pi / 2
  double cs, sn;
  if (2 * r4 <= L) {
    const double th = (M_PI / 2) * (double)r4 / (double)L;
    cs = std::cos(th);
    sn = std::sin(th);
  } else {
    const double th = (M_PI / 2) * (double)(L - r4) / (double)L;
    cs = std::sin(th);
    sn = std::cos(th);
  }
  double C, S;
  switch (q) {
    case 0: C = cs; S = sn; break;
    case 1: C = -sn; S = cs; break;
    case 2: C = -cs; S = -sn; break;
    default: C = sn; S = -cs; break;
  }
  *c = C;
  *s = -S;
}

struct SpecKey {
  int lx, ly, lz;
  double dx, dy, dz, k0;
  int kind;   // 0: collocated dyadic spectra, 1: rooftop scalar spectrum and symbols
  bool operator<(const SpecKey& o) const {
    return std::tie(lx, ly, lz, dx, dy, dz, k0, kind) < std::tie(o.lx, o.ly, o.lz, o.dx, o.dy, o.dz, o.k0, o.kind);
  }
};

struct Spectra {
  DevBuf s64, s32;
  size_t bytes() const { return s64.bytes + s32.bytes; }
};

constexpr int kRing = 16;

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

struct Server;

struct vie_context {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  hipStream_t stream = nullptr;
  DevBuf tw64, tw32;
  vie::TwiddleSet<double> tws64{};
  vie::TwiddleSet<float> tws32{};
  std::mutex mu;
  std::map<SpecKey, std::weak_ptr<Spectra>> cache;
  size_t reserved = 0;   // bytes reserved by requests admitted to the server
  std::map<std::array<int, 8>, std::pair<int, std::array<float, vie::kZPassVariants>>> ztune;
  std::map<std::array<int, 8>, std::pair<int, std::array<float, vie::kPlaneVariants>>> ptune;
  std::unique_ptr<Server> server;
  std::mutex server_mu;
  double* far_scratch = nullptr;   // this device's copy of the far field's fixed scratch array
  ~vie_context();
};

namespace {

int64_t spectra_elems(int lx, int ly, int lz, int kind) {
  const int64_t oct = (int64_t)(lx / 2 + 1) * (ly / 2 + 1) * (lz / 2 + 1);
  return kind == 1 ? oct + lx + ly + lz : 6 * oct;
}

std::shared_ptr<Spectra> get_spectra(vie_context* ctx, int lx, int ly, int lz, double dx, double dy, double dz,
                                     double k0, hipStream_t s, int kind = 0) {
  SpecKey key{lx, ly, lz, dx, dy, dz, k0, kind};
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end())
      if (auto sp = it->second.lock()) return sp;
  }
  auto sp = std::make_shared<Spectra>();
  const int64_t ne = spectra_elems(lx, ly, lz, kind);
  sp->s64.alloc(ne * sizeof(c128));
  sp->s32.alloc(ne * sizeof(c64));
  DevBuf scratch((kind == 1 ? 1 : 6) * (size_t)lx * ly * lz * sizeof(c128));
  // embed with the largest box the lengths support: a box of n <= (L+1)/2
  // voxels touches only offsets |m| <= n - 1, all of which are present.
  if (kind == 1)
    vie::green_spectrum_rooftop((lx + 1) / 2, (ly + 1) / 2, (lz + 1) / 2, lx, ly, lz, dx, dy, dz, k0,
                                scratch.as<c128>(), sp->s64.as<c128>(), sp->s32.as<c64>(), ctx->tws64, s);
  else
    vie::green_spectra((lx + 1) / 2, (ly + 1) / 2, (lz + 1) / 2, lx, ly, lz, dx, dy, dz, k0, scratch.as<c128>(),
                       sp->s64.as<c128>(), sp->s32.as<c64>(), ctx->tws64, s);
  hip_check(hipStreamSynchronize(s), "spectra");
  std::lock_guard<std::mutex> g(ctx->mu);
  auto& slot = ctx->cache[key];
  if (auto other = slot.lock()) return other;   // built concurrently by another thread
  slot = sp;
  return sp;
}

// Krylov vectors of a batch of systems.
enum VecKind { V_B = 0, V_X, V_R, V_RHAT, V_P, V_V, V_S, V_T, V_Y, V_Z, V_TMP1, V_TMP2, V_COUNT };

struct Group {
  int bx, by, bz, lx, ly, lz, nsys;
  int64_t bnv, n;
  std::shared_ptr<Spectra> spec;
  DevBuf chi, work, vecs;
  DevBuf sys_origin;     // expanded blocks: box origin of each system (int4)
  int zvar[2] = {0, 0};  // tuned z-pass variant per precision ([0] FP64, [1] FP32)
  int pvar[2] = {0, 0};  // tuned plane-kernel variant per precision
  // systems from problems with different spacing or wavelength: each
  // system's spectra (kept alive here) and a device table of their addresses
  // ([0, nsys) FP64, [nsys, 2 nsys) FP32); empty when all share `spec`
  std::vector<std::shared_ptr<Spectra>> sys_spec;
  DevBuf spec_tab;
  c128* vec[8];  // B, X, R, RHAT, P, V, S, T
  int slot0;     // first entry in the problem's inner status/state arrays
  bool wg = false;  // small enough for the one-workgroup block solver
  std::vector<int> blocks;
  // the group's inner BiCGSTAB step captured as a HIP graph, per precision
  // ([0] FP64, [1] FP32); replayed until the group's systems have converged
  hipGraphExec_t graph[2] = {nullptr, nullptr};
};

// Streams on which the groups of blocks iterate side by side during a
// preconditioner application (one per group when there are several), with
// the events that fork them from and join them back to the solve's stream.
struct Branches {
  std::vector<hipStream_t> streams;   // one per group, or empty
  std::vector<hipEvent_t> events;     // [0] fork, [1 + g] join of group g
};

}  // namespace

// Host-side plan of a problem: 1/chi, block ids, the blocks' bounding boxes
// and their shape groups.  Its device footprint is known before anything
// is allocated (admission by memory), and build_problem() turns it into a
// vie_problem with set-up work on a caller-chosen stream.
struct GroupPlan {
  int lx, ly, lz;
  std::vector<int> blocks;
  bool wg = false;
  int bx = 1, by = 1, bz = 1;
};

struct ProblemPlan {
  vie_grid g{};
  int64_t nv = 0;
  int lx = 0, ly = 0, lz = 0;
  double k0 = 0;
  std::vector<c128> chi;      // 1/chi, 0 on vacuum (rooftop: per face, [3][nz][ny][nx])
  bool rooftop = false;       // staggered rooftop unknowns on cell faces
  std::vector<int32_t> bid3;  // rooftop with blocks: block owning each face [3][nz][ny][nx], -1 none
  bool has_blocks = false;
  int n_blocks = 0;
  std::vector<int32_t> bid;   // -1 on vacuum
  std::vector<int> lo, hi;    // bounding boxes of the solve sets [3 * n_blocks]
  std::vector<int64_t> cnt;   // voxels per block
  // expanded blocks (overlap > 0): block k is solved on its voxels dilated by
  // `overlap` in every axis within the scatterer; emask[k] marks that set on
  // the box lo..hi (x fastest)
  int overlap = 0;
  std::vector<std::vector<uint8_t>> emask;
  std::vector<GroupPlan> groups;   // batched groups first, then block-solver groups
  // blocks of several problems (vie_solve_many): dx, dy, dz, k0 of every
  // block's own problem (empty: the plan's grid and k0 for every block)
  std::vector<double> blk_phys;
};

struct vie_problem {
  vie_context* ctx = nullptr;
  vie_grid g{};
  int64_t nv = 0;
  bool rooftop = false;   // rooftop discretisation: 1/chi per face (3 nv entries), scalar spectrum
  int lx = 0, ly = 0, lz = 0;
  double k0 = 0;
  std::shared_ptr<Spectra> spec;
  DevBuf chi, work, vecs, partials, partials2, ntile, ostate, ostatus, scal;
  int64_t pstride = 0;
  int zvar[2] = {0, 0};
  float ztune_ms[2][vie::kZPassVariants] = {};
  int pvar[2] = {0, 0};
  float ptune_ms[2][vie::kPlaneVariants] = {};
  // inner systems of all groups: partials (per-system stride ipstride)
  DevBuf d_ipartials, d_ipartials2, d_intile;
  int64_t ipstride = 0;
  c128* vec[V_COUNT] = {};
  // blocks
  int n_blocks = 0, n_nonempty = 0;
  std::vector<Group> groups;
  DevBuf d_block_id, d_block_group, d_block_sys, d_block_origin, d_gbox, d_gptr, d_istatus, d_istate, d_slots;
  DevBuf d_acc, d_hist, d_count;
  int n_inner = 0;
  vie::BlockMap bmap{};
  // Groups are ordered batched first, then the block-solver groups; with the
  // block solver on, the batched groups own inner slots [0, n_batched_wg).
  int n_batched_wg = 0, n_wg_groups = 0;
  std::vector<hipStream_t> wg_streams;   // one per block-solver group
  std::vector<hipEvent_t> wg_events;     // [0] fork, [1 + i] join of group i
  Branches branches;   // per-group streams of the inner iterations
  // polling: ring 0 for the outer loop, ring 1 + g for the inner steps of
  // group g
  int* h_ring = nullptr;
  int* d_ring = nullptr;   // the device's address of h_ring (null: progress values are copied)
  std::vector<std::array<hipEvent_t, kRing>> ev;
  std::mutex mu;
  size_t footprint = 0;
  const std::atomic<bool>* cancel = nullptr;   // set by the server: stop after the current outer step
  // flexible GMRES storage, allocated by the first such solve (restart gm_m,
  // with the preconditioned vectors Z when gm_z)
  DevBuf gm_basis, gm_small, gm_part, gm_state;
  int gm_m = 0;
  bool gm_z = false;
  // batched right-hand sides (plain BiCGSTAB), allocated by the first batch
  // solve: kBatchVecs vectors, one FFT work buffer and the Krylov scalars per
  // right-hand side
  DevBuf mr_vecs, mr_work, mr_state, mr_status, mr_partials, mr_partials2, mr_ntile, mr_count;
  int mr_cap = 0;
  // host plan (kept for batches) and, for preconditioned batches, the blocks
  // of nrhs copies of the problem stacked along z (inner solves only)
  std::shared_ptr<const ProblemPlan> plan;
  int overlap = 0;   // expanded blocks: gather the dilated sets, scatter the own voxels
  std::unique_ptr<vie_problem> replica;
  int replica_nrhs = 0;
  size_t replica_bytes = 0;

  ~vie_problem() {
    ApiShared api;
    for (auto& G : groups)
      for (auto g : G.graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto b : wg_streams) (void)hipStreamDestroy(b);
    for (auto e : wg_events) (void)hipEventDestroy(e);
    for (auto b : branches.streams) (void)hipStreamDestroy(b);
    for (auto e : branches.events) (void)hipEventDestroy(e);
    for (auto& r : ev)
      for (auto& e : r)
        if (e) (void)hipEventDestroy(e);
    if (h_ring) (void)hipHostFree(h_ring);
  }
};

namespace {

// Progress checks that trail the enqueued work (pinned ring + events).
struct Poller {
  vie_problem& P;
  hipStream_t s;
  int ring;
  long n = 0;
  Poller(vie_problem& p, hipStream_t st, int which) : P(p), s(st), ring(which) {}
  long push(const int* dval) {
    const int slot = (int)(n % kRing);
    hip_check(hipMemcpyAsync(&P.h_ring[ring * kRing + slot], dval, sizeof(int), hipMemcpyDeviceToHost, s),
              "poll copy");
    hip_check(hipEventRecord(P.ev[ring][slot], s), "poll event");
    return n++;
  }
  // The end of a fused BiCGSTAB step of the batch k (k_step_end), with the
  // number of systems still ACTIVE as the next value (stored straight into
  // the pinned ring, or into this ring's device counter and copied).
  long push_step_end(const KBatch& k) {
    if (!P.d_ring) {
      int* dc = P.d_count.as<int>() + ring;
      vie::k_step_end(k, dc, s);
      return push(dc);
    }
    const int slot = (int)(n % kRing);
    vie::k_step_end(k, P.d_ring + ring * kRing + slot, s);
    hip_check(hipEventRecord(P.ev[ring][slot], s), "poll event");
    return n++;
  }
  // The number of ACTIVE entries of status[0..nsys) as the next value.  The
  // counting kernel stores it straight into the pinned ring (no copy launch
  // per inner step); without a device address for the ring it counts into
  // dtmp and the value is copied.
  long push_count(const int* status, int nsys, int* dtmp) {
    if (!P.d_ring) {
      vie::count_active(status, nsys, dtmp, s);
      return push(dtmp);
    }
    const int slot = (int)(n % kRing);
    vie::count_active(status, nsys, P.d_ring + ring * kRing + slot, s);
    hip_check(hipEventRecord(P.ev[ring][slot], s), "poll event");
    return n++;
  }
  int wait(long ticket) {
    const int slot = (int)(ticket % kRing);
    hip_check(hipEventSynchronize(P.ev[ring][slot]), "poll wait");
    return P.h_ring[ring * kRing + slot];
  }
};

// Device-to-host copy ordered on the solve's own (non-blocking) stream.  A
// synchronous hipMemcpy would go through the legacy stream, which HIP
// refuses while another server slot is capturing its inner-step graph.
void copy_out(void* dst, const void* src, size_t bytes, hipStream_t s, const char* what) {
  hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), what);
  hip_check(hipStreamSynchronize(s), what);
}

template <typename R>
const cx<R>* spec_ptr(const Spectra& s);
template <>
const cx<double>* spec_ptr<double>(const Spectra& s) {
  return s.s64.as<c128>();
}
template <>
const cx<float>* spec_ptr<float>(const Spectra& s) {
  return s.s32.as<c64>();
}
template <typename R>
const vie::TwiddleSet<R>* tw_set(vie_context* c);
template <>
const vie::TwiddleSet<double>* tw_set<double>(vie_context* c) {
  return &c->tws64;
}
template <>
const vie::TwiddleSet<float>* tw_set<float>(vie_context* c) {
  return &c->tws32;
}

template <typename R>
MvmBatch<R> outer_batch(vie_problem& P, bool gated) {
  MvmBatch<R> b{};
  b.nx = P.g.nx;
  b.ny = P.g.ny;
  b.nz = P.g.nz;
  b.lx = P.lx;
  b.ly = P.ly;
  b.lz = P.lz;
  b.nsys = 1;
  b.vstride = 3 * P.nv;
  b.cstride = P.rooftop ? 3 * P.nv : P.nv;
  b.rooftop = P.rooftop ? 1 : 0;
  b.wstride = 3 * (int64_t)P.g.nz * P.ly * P.lx;
  b.sstride = 0;
  b.chi_inv = P.chi.as<c128>();
  b.spec = spec_ptr<R>(*P.spec);
  b.work = P.work.as<cx<R>>();
  b.status = gated ? P.ostatus.as<int>() : nullptr;
  b.tw = tw_set<R>(P.ctx);
  b.zvariant = P.zvar[sizeof(R) == sizeof(float) ? 1 : 0];
  b.plane = vie::plane_supported(b.lx, b.ly) ? 1 : 0;
  b.pvariant = P.pvar[sizeof(R) == sizeof(float) ? 1 : 0];
  return b;
}

template <typename R>
MvmBatch<R> group_batch(vie_problem& P, Group& G, bool gated) {
  MvmBatch<R> b{};
  b.nx = G.bx;
  b.ny = G.by;
  b.nz = G.bz;
  b.lx = G.lx;
  b.ly = G.ly;
  b.lz = G.lz;
  b.nsys = G.nsys;
  b.vstride = G.n;
  b.cstride = P.rooftop ? 3 * G.bnv : G.bnv;
  b.rooftop = P.rooftop ? 1 : 0;
  b.wstride = 3 * (int64_t)G.bz * G.ly * G.lx;
  b.sstride = 0;
  b.chi_inv = G.chi.as<c128>();
  b.spec = spec_ptr<R>(*G.spec);
  b.work = G.work.as<cx<R>>();
  b.status = gated ? P.d_istatus.as<int>() + G.slot0 : nullptr;
  b.tw = tw_set<R>(P.ctx);
  b.zvariant = G.zvar[sizeof(R) == sizeof(float) ? 1 : 0];
  b.plane = vie::plane_supported(b.lx, b.ly) ? 1 : 0;
  b.pvariant = G.pvar[sizeof(R) == sizeof(float) ? 1 : 0];
  if (G.spec_tab.p)
    b.spec_tab = G.spec_tab.as<const cx<R>*>() + (sizeof(R) == sizeof(float) ? G.nsys : 0);
  return b;
}

// Entries of the problem's 1/chi per period: one per voxel, or one per face
// (three per voxel) for the rooftop discretisation.
int64_t chi_period(const vie_problem& P) { return P.rooftop ? 3 * P.nv : P.nv; }

KBatch outer_kbatch(vie_problem& P) {
  KBatch k{};
  k.nsys = 1;
  k.n = 3 * P.nv;
  k.status = P.ostatus.as<int>();
  k.st = P.ostate.as<KState>();
  k.partials = P.partials.as<double>();
  k.pstride = P.pstride;
  k.ntile = P.ntile.as<int>();
  k.partials2 = P.partials2.as<double>();
  return k;
}

// One group's systems (producers), within the problem's inner arrays.
KBatch group_kbatch(vie_problem& P, Group& G) {
  KBatch k{};
  k.nsys = G.nsys;
  k.n = G.n;
  k.status = P.d_istatus.as<int>() + G.slot0;
  k.st = P.d_istate.as<KState>() + G.slot0;
  k.partials = P.d_ipartials.as<double>() + (int64_t)G.slot0 * P.ipstride;
  k.pstride = P.ipstride;
  k.ntile = P.d_intile.as<int>() + G.slot0;
  k.partials2 = P.d_ipartials2.as<double>() + (int64_t)G.slot0 * P.ipstride;
  return k;
}

// Inner systems [0, nsys) of the problem (finalize kernels).
KBatch inner_all(vie_problem& P, int nsys) {
  KBatch k{};
  k.nsys = nsys;
  k.n = 0;
  k.status = P.d_istatus.as<int>();
  k.st = P.d_istate.as<KState>();
  k.partials = P.d_ipartials.as<double>();
  k.pstride = P.ipstride;
  k.ntile = P.d_intile.as<int>();
  k.partials2 = P.d_ipartials2.as<double>();
  return k;
}

// Vectors of one unpreconditioned BiCGSTAB batch (y = p, z = s).
struct StepVecs {
  c128 *x, *r, *rhat, *p, *v, *s, *t;
};

// One BiCGSTAB step with K = I (y = p, z = s) for a batch of systems, with
// the scalar work fused into the kernels: [p update + product + <rhat, v>]
// -> [alpha + s update + product + <t, s>, <t, t>, ||s||] -> [half-step
// test, omega, x, r update + <rhat, r>, ||r||]; k_step_end (run by the
// caller, Poller::push_step_end) finishes it with rho, beta and convergence.
// The product t = A s runs before the half-step test: a system that
// converges at the half step computes one product it does not use, and the
// step needs no launch between the products.
template <typename R>
void fused_step(const MvmBatch<R>& m, const KBatch& k, const StepVecs& v, hipStream_t s) {
  const vie::FuseArgs f1{1, 1, v.r, v.p, v.v, v.rhat, nullptr};
  vie::mvm_pass1<R>(m, &k, f1, nullptr, false, s);
  vie::mvm_mid<R>(m, s);
  vie::mvm_pass5<R>(m, &k, f1, v.p, v.v, s);
  const vie::FuseArgs f2{3, 4, v.r, v.s, v.v, nullptr, v.s};
  vie::mvm_pass1<R>(m, &k, f2, nullptr, false, s);
  vie::mvm_mid<R>(m, s);
  vie::mvm_pass5<R>(m, &k, f2, v.s, v.t, s);
  vie::k_update_xr_fused(k, v.x, v.p, v.s, v.r, v.s, v.t, v.rhat, s);
}

c128* const* gptr(vie_problem& P, int kind) { return P.d_gptr.as<c128*>() + (size_t)kind * P.groups.size(); }

// Groups solved by the batched kernels (all, or all but the block-solver
// groups) and their inner slot count.
bool batched(const Group& G, bool wg) { return !(wg && G.wg); }
int batched_slots(const vie_problem& P, bool wg) { return wg ? P.n_batched_wg : P.n_inner; }

// One inner BiCGSTAB step of every system of a group (the inner solves are
// unpreconditioned), without its step end.
template <typename R>
void group_step(vie_problem& P, Group& G, hipStream_t s) {
  const StepVecs v{G.vec[V_X], G.vec[V_R], G.vec[V_RHAT], G.vec[V_P], G.vec[V_V], G.vec[V_S], G.vec[V_T]};
  fused_step<R>(group_batch<R>(P, G, true), group_kbatch(P, G), v, s);
}

// The group's inner step captured once per precision as a HIP graph (all
// kernel arguments are fixed per problem), replayed every iteration.  The
// capture holds the process-wide API lock exclusively: other threads' HIP
// calls that a capture forbids wait for it.
template <typename R>
hipGraphExec_t group_graph(vie_problem& P, Group& G) {
  hipGraphExec_t& ex = G.graph[sizeof(R) == sizeof(float) ? 1 : 0];
  if (ex) return ex;
  std::unique_lock<std::shared_mutex> capture(vie::api_mutex());
  hipStream_t cs = nullptr;
  hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    hip_check(e, "begin capture");
  }
  try {
    group_step<R>(P, G, cs);
  } catch (...) {
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    throw;
  }
  e = hipStreamEndCapture(cs, &g);
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    ex = nullptr;
    hip_check(e, "graph capture");
  }
  return ex;
}

// A captured step spares the host its launches, but each replay's start and
// end cost the GPU more than the gaps between kernels launched one by one.
// Groups whose products transform at least 2^21 points per step keep the GPU
// busy long enough for the host to launch the step's kernels ahead of it, so
// they launch them one by one (the metasurface's pillar and slab groups:
// 2.27 against 2.36 s per mixed solve, same results); smaller groups replay
// the captured step.
constexpr int64_t kEagerStepPoints = int64_t(1) << 21;
bool replay_step(const Group& G) {
  return (int64_t)G.nsys * 3 * G.lx * G.ly * G.lz < kEagerStepPoints;
}

template <typename R>
vie::BlockSolveArgs wg_args(vie_problem& P, Group& G, const int* gate, double tol, int maxit) {
  vie::BlockSolveArgs a{};
  a.nsys = G.nsys;
  a.bx = G.bx;
  a.by = G.by;
  a.bz = G.bz;
  a.n = G.n;
  a.chi = G.chi.as<c128>();
  a.b = G.vec[V_B];
  a.x = G.vec[V_X];
  a.r = G.vec[V_R];
  a.rhat = G.vec[V_RHAT];
  a.p = G.vec[V_P];
  a.v = G.vec[V_V];
  a.s = G.vec[V_S];
  a.t = G.vec[V_T];
  a.work = G.work.p;
  a.spec = spec_ptr<R>(*G.spec);
  a.twx = tw_set<R>(P.ctx)->table[G.lx];
  a.twz = tw_set<R>(P.ctx)->table[G.lz];
  a.status = P.d_istatus.as<int>() + G.slot0;
  a.st = P.d_istate.as<KState>() + G.slot0;
  a.gate = gate;
  a.tol = tol;
  a.maxit = maxit;
  return a;
}

// y = K2^{-1} w: inner BiCGSTAB-FFT solves of every block (Sec. II-B).
// Block-solver groups (wg) run one launch each on their own streams while
// the batched groups iterate on s; s waits for both before the scatter.
template <typename R>
void precond_apply(vie_problem& P, const c128* w, c128* y, double tol, int maxit, const int* gate, int lag,
                   int32_t* hist, int64_t hist_cap, bool graphs, bool wg, hipStream_t s) {
  if (P.overlap == 0) {
    vie::block_gather(P.bmap, w, gptr(P, V_B), s);
  } else {   // expanded blocks overlap: each system gathers its own set
    for (auto& G : P.groups)
      vie::gather_sets(w, P.g.nx, P.g.ny, P.g.nz, G.bx, G.by, G.bz, G.nsys, G.sys_origin.as<int4>(),
                       G.chi.as<c128>(), G.vec[V_B], s);
  }
  const bool any_wg = wg && P.n_wg_groups > 0;
  if (any_wg) {
    hip_check(hipEventRecord(P.wg_events[0], s), "fork");
    int i = 0;
    for (auto& G : P.groups) {
      if (!G.wg) continue;
      hipStream_t ws = P.wg_streams[i];
      hip_check(hipStreamWaitEvent(ws, P.wg_events[0], 0), "fork wait");
      vie::block_solve<R>(wg_args<R>(P, G, gate, tol, maxit), G.lx, G.lz, ws);
      hip_check(hipEventRecord(P.wg_events[1 + i], ws), "join");
      ++i;
    }
  }
  const int nslots = batched_slots(P, wg);
  if (nslots > 0) {
    for (auto& G : P.groups) {
      if (!batched(G, wg)) continue;
      KBatch k = group_kbatch(P, G);
      vie::k_init(k, G.vec[V_B], G.vec[V_X], G.vec[V_R], G.vec[V_RHAT], gate, s);
    }
    vie::k_finalize(inner_all(P, nslots), vie::FIN_INIT, s, gate, tol, maxit);
    // Every batched group iterates on its own until its systems have
    // converged (its own stream when there are several, its own progress
    // ring): a group that finishes early stops costing launches.
    struct Run {
      size_t gi;
      hipStream_t st;
      hipGraphExec_t ex;
      Poller poll;
      bool active;
    };
    std::vector<size_t> bg;
    for (size_t gi = 0; gi < P.groups.size(); ++gi)
      if (batched(P.groups[gi], wg)) bg.push_back(gi);
    const bool split = bg.size() > 1 && P.branches.streams.size() == P.groups.size();
    if (split) {
      hip_check(hipEventRecord(P.branches.events[0], s), "fork");
      for (size_t gi : bg) hip_check(hipStreamWaitEvent(P.branches.streams[gi], P.branches.events[0], 0), "fork wait");
    }
    std::vector<Run> runs;
    for (size_t gi : bg) {
      hipStream_t gs = split ? P.branches.streams[gi] : s;
      runs.push_back(Run{gi, gs, graphs && replay_step(P.groups[gi]) ? group_graph<R>(P, P.groups[gi]) : nullptr,
                         Poller(P, gs, 1 + (int)gi),
                         true});
    }
    for (int it = 1; it <= maxit; ++it) {
      bool any = false;
      for (auto& r : runs) {
        if (!r.active) continue;
        any = true;
        Group& G = P.groups[r.gi];
        if (r.ex)
          hip_check(hipGraphLaunch(r.ex, r.st), "graph launch");
        else
          group_step<R>(P, G, r.st);
        const long t = r.poll.push_step_end(group_kbatch(P, G));
        if (t - lag >= 0 && r.poll.wait(t - lag) == 0) r.active = false;
      }
      if (!any) break;
    }
    if (split)
      for (size_t gi : bg) {
        hipEvent_t ev = P.branches.events[1 + gi];
        hip_check(hipEventRecord(ev, P.branches.streams[gi]), "join");
        hip_check(hipStreamWaitEvent(s, ev, 0), "join wait");
      }
  }
  if (any_wg)
    for (int i = 0; i < P.n_wg_groups; ++i) hip_check(hipStreamWaitEvent(s, P.wg_events[1 + i], 0), "join wait");
  vie::block_scatter(P.bmap, gptr(P, V_X), y, s);
  vie::record_inner(gate, P.d_istate.as<KState>(), P.d_slots.as<int>(), P.n_nonempty, P.d_acc.as<int64_t>(), hist,
                    hist_cap, s);
}

struct RunResult {
  KState st;
  int status;
};

// Right-preconditioned BiCGSTAB on the full grid: A x = rhs (Sec. II-B).
// R: precision of the full-grid products; RI: of the inner block solves.
template <typename R, typename RI = R>
RunResult run_bicgstab(vie_problem& P, const c128* rhs, c128* x, double tol, int maxit, bool prec, double tol_in,
                       int maxit_in, int lag, int32_t* hist, int64_t hist_cap, bool graphs, bool wg,
                       hipStream_t s) {
  KBatch k = outer_kbatch(P);
  MvmBatch<R> m = outer_batch<R>(P, true);
  c128** v = P.vec;
  const int* gate = P.ostatus.as<int>();
  vie::k_init(k, rhs, x, v[V_R], v[V_RHAT], nullptr, s);
  vie::k_finalize(k, vie::FIN_INIT, s, nullptr, tol, maxit);
  const StepVecs vv{x, v[V_R], v[V_RHAT], v[V_P], v[V_V], v[V_S], v[V_T]};
  Poller poll(P, s, 0);
  for (int it = 1; it <= maxit; ++it) {
    if (!prec) {
      fused_step<R>(m, k, vv, s);
      // progress value: the number of systems (0 or 1) still iterating
      const long t = poll.push_step_end(k);
      if (t - lag >= 0 && poll.wait(t - lag) == 0) break;
      if (P.cancel && P.cancel->load(std::memory_order_relaxed)) break;
      continue;
    } else {
      vie::k_update_p(k, v[V_R], v[V_V], v[V_P], s);
      precond_apply<RI>(P, v[V_P], v[V_Y], tol_in, maxit_in, gate, lag, hist, hist_cap, graphs, wg, s);
      const vie::FuseArgs fa{0, 1, nullptr, nullptr, nullptr, v[V_RHAT], nullptr};
      vie::mvm_pass1<R>(m, &k, fa, v[V_Y], false, s);
      vie::mvm_mid<R>(m, s);
      vie::mvm_pass5<R>(m, &k, fa, v[V_Y], v[V_V], s);
      vie::k_finalize(k, vie::FIN_ALPHA, s);
      vie::k_update_s(k, v[V_R], v[V_V], v[V_S], s);
      vie::k_finalize(k, vie::FIN_S, s);
      precond_apply<RI>(P, v[V_S], v[V_Z], tol_in, maxit_in, gate, lag, hist, hist_cap, graphs, wg, s);
      const vie::FuseArgs fo{0, 2, nullptr, nullptr, nullptr, nullptr, v[V_S]};
      vie::mvm_pass1<R>(m, &k, fo, v[V_Z], false, s);
      vie::mvm_mid<R>(m, s);
      vie::mvm_pass5<R>(m, &k, fo, v[V_Z], v[V_T], s);
      vie::k_finalize(k, vie::FIN_OMEGA, s);
      vie::k_update_xr(k, x, v[V_Y], v[V_Z], v[V_R], v[V_S], v[V_T], v[V_RHAT], s);
      vie::k_finalize(k, vie::FIN_XR, s);
    }
    const long t = poll.push(P.ostatus.as<int>());
    if (t - lag >= 0 && poll.wait(t - lag) != vie::ST_ACTIVE) break;
    if (P.cancel && P.cancel->load(std::memory_order_relaxed)) break;
  }
  hip_check(hipStreamSynchronize(s), "solve");
  RunResult r{};
  copy_out(&r.st, P.ostate.p, sizeof(KState), s, "state");
  copy_out(&r.status, P.ostatus.p, sizeof(int), s, "state");
  return r;
}

// Storage of flexible GMRES(m): m + 1 Arnoldi vectors, m preconditioned
// vectors (with a preconditioner), the small dense arrays and the partials.
// Allocated on first use and counted in the problem's footprint.
size_t gmres_small_bytes(int m) {
  return ((size_t)(m + 1) * m + 2 * (size_t)m + 3 * (size_t)(m + 1)) * sizeof(c128) + (size_t)m * sizeof(double);
}

void ensure_gmres(vie_problem& P, int m, bool prec) {
  if (P.gm_m == m && (P.gm_z || !prec)) return;
  const int64_t n = 3 * P.nv;
  const size_t basis = ((size_t)(m + 1) + (prec ? (size_t)m : 0)) * (size_t)n * sizeof(c128);
  const size_t part = (size_t)(m + 1) * (size_t)vie::gmres_chunks(n) * 2 * sizeof(double);
  const size_t total = basis + gmres_small_bytes(m) + part + sizeof(vie::GmresState);
  const size_t old = P.gm_basis.bytes + P.gm_small.bytes + P.gm_part.bytes + P.gm_state.bytes;
  vie_context* ctx = P.ctx;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const size_t others = ctx->used + ctx->reserved - std::min(ctx->used + ctx->reserved, old);
    if (ctx->budget && others + total > ctx->budget) fail(VIE_EBUSY, "GMRES storage exceeds the context's HBM budget");
    ctx->used = ctx->used - std::min(ctx->used, old) + total;
  }
  P.footprint = P.footprint - std::min(P.footprint, old) + total;
  P.gm_m = 0;
  P.gm_basis.reset();
  P.gm_small.reset();
  P.gm_part.reset();
  P.gm_state.reset();
  try {
    P.gm_basis.alloc(basis);
    P.gm_small.alloc(gmres_small_bytes(m));
    P.gm_part.alloc(part);
    P.gm_state.alloc(sizeof(vie::GmresState));
  } catch (...) {
    P.gm_basis.reset();
    P.gm_small.reset();
    P.gm_part.reset();
    P.gm_state.reset();
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= std::min(ctx->used, total);
    P.footprint -= std::min(P.footprint, total);
    throw;
  }
  P.gm_m = m;
  P.gm_z = prec;
}

vie::GmresDev gmres_dev(vie_problem& P) {
  vie::GmresDev d{};
  const int m = P.gm_m;
  const int64_t n = 3 * P.nv;
  d.V = P.gm_basis.as<c128>();
  d.Z = P.gm_z ? d.V + (int64_t)(m + 1) * n : nullptr;
  d.n = n;
  d.m = m;
  c128* q = P.gm_small.as<c128>();
  d.H = q;
  q += (int64_t)(m + 1) * m;
  d.sn = q;
  q += m;
  d.g = q;
  q += m + 1;
  d.y = q;
  q += m;
  d.h = q;
  q += m + 1;
  d.c = q;
  q += m + 1;
  d.cs = reinterpret_cast<double*>(q);
  d.part = P.gm_part.as<double>();
  d.nchunk = vie::gmres_chunks(n);
  d.scal = P.scal.as<double>();
  d.st = P.gm_state.as<vie::GmresState>();
  d.status = P.ostatus.as<int>();
  return d;
}

// Flexible GMRES(m) on the full grid, x0 = 0: a solver variant next to the
// BiCGSTAB of Sec. II-B.  Each Arnoldi step applies the block preconditioner
// of eq. (10) once and the product once; the preconditioned vectors are kept
// because the inexact inner solves make the preconditioner change from step
// to step.  Cycles of m steps end with x += Z y and a restart from the
// residual b - A x (in the product precision R; RI: inner block solves).
template <typename R, typename RI = R>
RunResult run_fgmres(vie_problem& P, const c128* rhs, c128* x, double tol, int maxit, int restart, bool prec,
                     double tol_in, int maxit_in, int lag, int32_t* hist, int64_t hist_cap, bool graphs, bool wg,
                     hipStream_t s) {
  ensure_gmres(P, restart, prec);
  const vie::GmresDev d = gmres_dev(P);
  const int64_t n = d.n;
  const MvmBatch<R> mg = outer_batch<R>(P, true);
  const MvmBatch<R> mu = outer_batch<R>(P, false);
  const int* gate = P.ostatus.as<int>();
  auto V = [&](int j) { return d.V + (int64_t)j * n; };
  auto Z = [&](int j) { return d.Z + (int64_t)j * n; };
  hip_check(hipMemsetAsync(x, 0, n * sizeof(c128), s), "x0");
  hip_check(hipMemcpyAsync(V(0), rhs, n * sizeof(c128), hipMemcpyDeviceToDevice, s), "r0");
  vie::norm2(V(0), n, P.partials.as<double>(), P.scal.as<double>(), s);
  vie::gmres_start(d, V(0), true, tol, maxit, s);
  int status = vie::ST_ACTIVE;
  for (;;) {
    Poller poll(P, s, 0);
    for (int j = 0; j < d.m; ++j) {
      const c128* src = V(j);
      if (prec) {
        precond_apply<RI>(P, V(j), Z(j), tol_in, maxit_in, gate, lag, hist, hist_cap, graphs, wg, s);
        src = Z(j);
      }
      vie::mvm<R>(mg, src, V(j + 1), false, s);
      vie::gmres_orthogonalise(d, V(j + 1), j, s);
      vie::norm2(V(j + 1), n, P.partials.as<double>(), P.scal.as<double>(), s);
      vie::gmres_arnoldi(d, V(j + 1), j, s);
      const long t = poll.push(P.ostatus.as<int>());
      if (t - lag >= 0 && poll.wait(t - lag) != vie::ST_ACTIVE) break;
      if (P.cancel && P.cancel->load(std::memory_order_relaxed)) break;
    }
    vie::gmres_update(d, x, prec ? d.Z : d.V, s);
    hip_check(hipMemcpyAsync(&status, P.ostatus.p, sizeof(int), hipMemcpyDeviceToHost, s), "status");
    hip_check(hipStreamSynchronize(s), "fgmres cycle");
    if (status != vie::ST_RESTART || (P.cancel && P.cancel->load())) break;
    // restart from the residual of the updated iterate
    vie::mvm<R>(mu, x, V(0), false, s);
    vie::sub_vec(rhs, V(0), V(0), n, s);
    vie::norm2(V(0), n, P.partials.as<double>(), P.scal.as<double>(), s);
    vie::gmres_start(d, V(0), false, tol, maxit, s);
  }
  vie::GmresState gs{};
  copy_out(&gs, d.st, sizeof(gs), s, "state");
  RunResult r{};
  r.st.nb = gs.nb;
  r.st.iters = gs.iters;
  r.st.rnorm = gs.relres;
  r.status = status == vie::ST_RESTART ? vie::ST_MAXIT : status;
  return r;
}

// Conjugate gradient squared (Sonneveld) on the full grid, x0 = 0: a solver
// variant that Sec. II-B names beside BiCGSTAB, right-preconditioned with the
// block preconditioner of eq. (10).  Each step applies the preconditioner
// twice (to p and to u + q) and the product twice (to K^{-1} p and to the new
// x: the residual is recomputed as b - A x and tested).  Vectors: u in V_S,
// q in V_T, v and A x in V_V, u + q in V_Z, K^{-1} p then K^{-1}(u + q) in
// V_Y; rhs and x may be V_TMP2 / V_TMP1 (refinement).
template <typename R, typename RI = R>
RunResult run_cgs(vie_problem& P, const c128* rhs, c128* x, double tol, int maxit, bool prec, double tol_in,
                  int maxit_in, int lag, int32_t* hist, int64_t hist_cap, bool graphs, bool wg, hipStream_t s) {
  KBatch k = outer_kbatch(P);
  MvmBatch<R> m = outer_batch<R>(P, true);
  c128** v = P.vec;
  const int* gate = P.ostatus.as<int>();
  c128 *r = v[V_R], *rhat = v[V_RHAT], *u = v[V_S], *q = v[V_T], *p = v[V_P], *av = v[V_V], *w = v[V_Z];
  c128* ph = prec ? v[V_Y] : p;    // K^{-1} p
  c128* uh = prec ? v[V_Y] : w;    // K^{-1} (u + q)
  vie::k_init(k, rhs, x, r, rhat, nullptr, s);
  vie::k_finalize(k, vie::FIN_INIT, s, nullptr, tol, maxit);
  const vie::FuseArgs fa{0, 1, nullptr, nullptr, nullptr, rhat, nullptr};
  Poller poll(P, s, 0);
  for (int it = 1; it <= maxit; ++it) {
    vie::cgs_update_up(k, r, u, q, p, s);
    if (prec) precond_apply<RI>(P, p, ph, tol_in, maxit_in, gate, lag, hist, hist_cap, graphs, wg, s);
    vie::mvm_pass1<R>(m, &k, fa, ph, false, s);
    vie::mvm_mid<R>(m, s);
    vie::mvm_pass5<R>(m, &k, fa, ph, av, s);
    vie::k_finalize(k, vie::FIN_ALPHA, s);
    vie::cgs_update_q(k, u, av, q, w, s);
    if (prec) precond_apply<RI>(P, w, uh, tol_in, maxit_in, gate, lag, hist, hist_cap, graphs, wg, s);
    vie::cgs_update_x(k, x, uh, s);
    vie::mvm<R>(m, x, av, false, s);
    vie::cgs_update_r(k, rhs, av, r, rhat, s);
    vie::k_finalize(k, vie::FIN_CGS, s);
    const long t = poll.push(P.ostatus.as<int>());
    if (t - lag >= 0 && poll.wait(t - lag) != vie::ST_ACTIVE) break;
    if (P.cancel && P.cancel->load(std::memory_order_relaxed)) break;
  }
  hip_check(hipStreamSynchronize(s), "solve");
  RunResult res{};
  copy_out(&res.st, P.ostate.p, sizeof(KState), s, "state");
  copy_out(&res.status, P.ostatus.p, sizeof(int), s, "state");
  return res;
}

double true_relres(vie_problem& P, const c128* rhs, const c128* x, c128* tmp_ax, c128* tmp_r, double nb,
                   hipStream_t s) {
  MvmBatch<double> m = outer_batch<double>(P, false);
  vie::mvm<double>(m, x, tmp_ax, false, s);
  vie::sub_vec(rhs, tmp_ax, tmp_r, 3 * P.nv, s);
  vie::norm2(tmp_r, 3 * P.nv, P.partials.as<double>(), P.scal.as<double>(), s);
  double r2 = 0;
  hip_check(hipMemcpyAsync(&r2, P.scal.p, sizeof(double), hipMemcpyDeviceToHost, s), "norm");
  hip_check(hipStreamSynchronize(s), "norm");
  return nb > 0 ? std::sqrt(r2) / nb : 0.0;
}

void validate_opts(const vie_opts* o, bool has_blocks) {
  if (!o) fail(VIE_EINVAL, "opts is NULL");
  if (!(o->tol_outer >= 0) || !is_finite(o->tol_outer)) fail(VIE_EINVAL, "tol_outer must be finite and >= 0");
  if (o->maxit_outer < 0 || o->maxit_outer > 1000000) fail(VIE_EINVAL, "maxit_outer out of range");
  if (o->precision != VIE_FP64 && o->precision != VIE_MIXED && o->precision != VIE_MIXED_INNER)
    fail(VIE_EINVAL, "unknown precision");
  if (o->poll_lag < 0 || o->poll_lag > kRing - 2) fail(VIE_EINVAL, "poll_lag out of range");
  if (o->max_refine < 0 || o->max_refine > 100) fail(VIE_EINVAL, "max_refine out of range");
  if (o->flags & ~(VIE_FLAG_NO_GRAPHS | VIE_FLAG_NO_BLOCK_KERNEL)) fail(VIE_EINVAL, "unknown flags");
  if (o->solver != VIE_SOLVER_BICGSTAB && o->solver != VIE_SOLVER_FGMRES && o->solver != VIE_SOLVER_CGS)
    fail(VIE_EINVAL, "unknown solver");
  if (o->solver == VIE_SOLVER_FGMRES && (o->restart < 1 || o->restart > 1000))
    fail(VIE_EINVAL, "restart must be in [1, 1000]");
  if (o->precondition) {
    if (!has_blocks) fail(VIE_EINVAL, "precondition requested but the problem has no blocks");
    if (!(o->tol_inner >= 0) || !is_finite(o->tol_inner)) fail(VIE_EINVAL, "tol_inner must be finite and >= 0");
    if (o->maxit_inner < 1 || o->maxit_inner > 1000000) fail(VIE_EINVAL, "maxit_inner out of range");
  }
}

void set_device(vie_context* ctx) { hip_check(hipSetDevice(ctx->device), "hipSetDevice"); }

// One solve.  With `solved`, the main iteration has already run (a batch of
// right-hand sides): V_B and V_X hold this system's rhs and iterate, and
// only the true residual, refinement, fields and statistics follow.
vie_status solve_impl(vie_problem* p, const c128* e_inc, const vie_opts* o, c128* e_tot, c128* pol,
                      vie_stats* stats, hipStream_t s, const RunResult* solved = nullptr) {
  auto t0 = std::chrono::steady_clock::now();
  vie_problem& P = *p;
  c128** v = P.vec;
  const bool prec = o->precondition != 0;
  const bool graphs = (o->flags & VIE_FLAG_NO_GRAPHS) == 0;
  const bool wg = (o->flags & VIE_FLAG_NO_BLOCK_KERNEL) == 0;
  int32_t* hist = nullptr;
  int64_t hist_cap = 0;
  if (stats && stats->inner_hist && stats->inner_hist_cap > 0 && prec) {
    P.d_hist.alloc((size_t)stats->inner_hist_cap * sizeof(int32_t));
    hist = P.d_hist.as<int32_t>();
    hist_cap = stats->inner_hist_cap;
  }
  if (prec) hip_check(hipMemsetAsync(P.d_acc.p, 0, 3 * sizeof(int64_t), s), "acc");
  if (!solved) vie::masked_copy(e_inc, P.chi.as<c128>(), v[V_B], P.nv, s, chi_period(P));
  RunResult rr;
  int refine = 0, refine_iters = 0;
  double relres_true = 0;
  const bool fgmres = o->solver == VIE_SOLVER_FGMRES;
  auto run = [&](auto tag, auto itag, const c128* rhs, c128* x, double tol) {
    using R = decltype(tag);
    using RI = decltype(itag);
    if (fgmres)
      return run_fgmres<R, RI>(P, rhs, x, tol, o->maxit_outer, o->restart, prec, o->tol_inner, o->maxit_inner,
                               o->poll_lag, hist, hist_cap, graphs, wg, s);
    if (o->solver == VIE_SOLVER_CGS)
      return run_cgs<R, RI>(P, rhs, x, tol, o->maxit_outer, prec, o->tol_inner, o->maxit_inner, o->poll_lag, hist,
                            hist_cap, graphs, wg, s);
    return run_bicgstab<R, RI>(P, rhs, x, tol, o->maxit_outer, prec, o->tol_inner, o->maxit_inner, o->poll_lag,
                               hist, hist_cap, graphs, wg, s);
  };
  if (o->precision == VIE_FP64 || o->precision == VIE_MIXED_INNER) {
    // FP64 full-grid products: the recursive residual stays accurate, no refinement
    if (solved)
      rr = *solved;
    else if (o->precision == VIE_FP64)
      rr = run(double{}, double{}, v[V_B], v[V_X], o->tol_outer);
    else
      rr = run(double{}, float{}, v[V_B], v[V_X], o->tol_outer);
    relres_true = true_relres(P, v[V_B], v[V_X], v[V_TMP1], v[V_TMP2], rr.st.nb, s);
  } else {
    rr = solved ? *solved : run(float{}, float{}, v[V_B], v[V_X], o->tol_outer);
    const double nb = rr.st.nb;
    relres_true = true_relres(P, v[V_B], v[V_X], v[V_TMP1], v[V_TMP2], nb, s);
    // iterative refinement: solve A d = b - A x with FP32 products, x += d
    while (rr.status != vie::ST_BREAKDOWN && relres_true > o->tol_outer && refine < o->max_refine && nb > 0 &&
           !(P.cancel && P.cancel->load())) {
      const double tol_c = std::min(0.5, o->tol_outer / relres_true);
      RunResult rc = run(float{}, float{}, v[V_TMP2], v[V_TMP1], tol_c);
      vie::add_vec(v[V_X], v[V_TMP1], 3 * P.nv, s);
      ++refine;
      refine_iters += rc.st.iters;
      relres_true = true_relres(P, v[V_B], v[V_X], v[V_TMP1], v[V_TMP2], nb, s);
    }
  }
  vie::total_field(v[V_X], P.chi.as<c128>(), e_tot, P.nv, 3, s, chi_period(P));
  if (pol) hip_check(hipMemcpyAsync(pol, v[V_X], 3 * P.nv * sizeof(c128), hipMemcpyDeviceToDevice, s), "pol");
  int64_t acc[3] = {0, 0, 0};
  if (prec) hip_check(hipMemcpyAsync(acc, P.d_acc.p, sizeof(acc), hipMemcpyDeviceToHost, s), "acc");
  hip_check(hipStreamSynchronize(s), "solve end");
  if (stats) {
    stats->outer_iters = rr.st.iters;
    stats->refine_steps = refine;
    stats->refine_iters = refine_iters;
    stats->inner_iters_total = acc[0];
    stats->precond_applies = acc[1];
    stats->relres_recursive = rr.st.rnorm;
    stats->relres_true = relres_true;
    stats->final_state = rr.status == vie::ST_BREAKDOWN ? 3 : (rr.status == vie::ST_CONVERGED ? 1 : 4);
    stats->inner_hist_len = 0;
    if (hist) {
      const int64_t len = std::min<int64_t>(acc[2], hist_cap);
      if (acc[2] <= hist_cap) {
        copy_out(stats->inner_hist, hist, len * sizeof(int32_t), s, "hist");
        stats->inner_hist_len = len;
      }
    }
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (P.cancel && P.cancel->load()) {
    g_last_error = "request cancelled";
    return VIE_ECANCELLED;
  }
  if (rr.status == vie::ST_BREAKDOWN) {
    g_last_error = fgmres                           ? "GMRES breakdown (last iterate written)"
                   : o->solver == VIE_SOLVER_CGS ? "CGS breakdown (last iterate written)"
                                                 : "BiCGSTAB breakdown (last iterate written)";
    return VIE_EBREAKDOWN;
  }
  // mixed: the refinement may reach the tolerance after the main loop's cap
  const bool refined_ok = o->precision == VIE_MIXED && refine > 0 && relres_true <= o->tol_outer;
  if (rr.status == vie::ST_CONVERGED || rr.status == vie::ST_HALF || refined_ok) {
    if (o->precision == VIE_MIXED && relres_true > o->tol_outer) {
      g_last_error = "mixed-precision solve stopped above tol_outer after refinement";
      return VIE_NOT_CONVERGED;
    }
    return VIE_OK;
  }
  g_last_error = "iteration cap reached";
  return VIE_NOT_CONVERGED;
}

// Vectors of a batch of right-hand sides: B, X, R, RHAT, P, V, S, T, Y, Z,
// and two in the stacked layout (preconditioner input and output).
constexpr int kBatchVecs = 12;
enum BatchVec { BV_B = 0, BV_X, BV_R, BV_RHAT, BV_P, BV_V, BV_S, BV_T, BV_Y, BV_Z, BV_WI, BV_WO };

void ensure_batch(vie_problem& P, int nrhs) {
  if (P.mr_cap >= nrhs) return;
  const int64_t n = 3 * P.nv;
  const size_t vecs = (size_t)kBatchVecs * nrhs * n * sizeof(c128);
  const size_t work = (size_t)nrhs * 3 * P.g.nz * P.ly * P.lx * sizeof(c128);
  const size_t small = (size_t)nrhs * (sizeof(KState) + 2 * sizeof(int) + 2 * (size_t)P.pstride * sizeof(double)) +
                       sizeof(int);
  const size_t total = vecs + work + small;
  const size_t old = P.mr_vecs.bytes + P.mr_work.bytes + P.mr_state.bytes + P.mr_status.bytes +
                     P.mr_partials.bytes + P.mr_partials2.bytes + P.mr_ntile.bytes + P.mr_count.bytes;
  vie_context* ctx = P.ctx;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    const size_t others = ctx->used + ctx->reserved - std::min(ctx->used + ctx->reserved, old);
    if (ctx->budget && others + total > ctx->budget) fail(VIE_EBUSY, "batch storage exceeds the context's HBM budget");
    ctx->used = ctx->used - std::min(ctx->used, old) + total;
  }
  P.footprint = P.footprint - std::min(P.footprint, old) + total;
  P.mr_cap = 0;
  DevBuf* bufs[] = {&P.mr_vecs,     &P.mr_work,     &P.mr_state, &P.mr_status,
                    &P.mr_partials, &P.mr_partials2, &P.mr_ntile, &P.mr_count};
  for (DevBuf* b : bufs) b->reset();
  try {
    P.mr_vecs.alloc(vecs);
    P.mr_work.alloc(work);
    P.mr_state.alloc((size_t)nrhs * sizeof(KState));
    P.mr_status.alloc((size_t)nrhs * sizeof(int));
    P.mr_partials.alloc((size_t)nrhs * P.pstride * sizeof(double));
    P.mr_partials2.alloc((size_t)nrhs * P.pstride * sizeof(double));
    P.mr_ntile.alloc((size_t)nrhs * sizeof(int));
    P.mr_count.alloc(sizeof(int));
  } catch (...) {
    for (DevBuf* b : bufs) b->reset();
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= std::min(ctx->used, total);
    P.footprint -= std::min(P.footprint, total);
    throw;
  }
  P.mr_cap = nrhs;
}

c128* batch_vec(vie_problem& P, int kind, int nrhs) {
  return P.mr_vecs.as<c128>() + (int64_t)kind * nrhs * 3 * P.nv;
}

// nrhs systems with the full-grid operator: shared 1/chi and spectra, one
// work buffer, vector and status per system.
template <typename R>
MvmBatch<R> batch_mvm(vie_problem& P, int nrhs) {
  MvmBatch<R> b = outer_batch<R>(P, true);
  b.nsys = nrhs;
  b.cstride = 0;
  b.work = P.mr_work.as<cx<R>>();
  b.status = P.mr_status.as<int>();
  return b;
}

KBatch batch_kbatch(vie_problem& P, int nrhs) {
  KBatch k{};
  k.nsys = nrhs;
  k.n = 3 * P.nv;
  k.status = P.mr_status.as<int>();
  k.st = P.mr_state.as<KState>();
  k.partials = P.mr_partials.as<double>();
  k.pstride = P.pstride;
  k.ntile = P.mr_ntile.as<int>();
  k.partials2 = P.mr_partials2.as<double>();
  return k;
}

// The Krylov state of a batch of systems that share the full grid's shape
// (right-hand sides of one problem, or several problems): vectors
// kBatchVecs x [nsys][3 nv], per-system state and status, the replica that
// holds the blocks of every system stacked along z (preconditioned solves)
// and the problem whose outer progress ring (ring 0) the loop polls.
struct BatchSet {
  vie_problem& poll;
  vie_problem* replica;
  int nsys;
  int64_t nv;
  c128* vecs;
  KBatch k;
  int* status;
  int* count;
  c128* vec(int kind) const { return vecs + (int64_t)kind * nsys * 3 * nv; }
};

// BiCGSTAB of the batch's systems (x0 = 0): every launch covers all
// systems, each stops on its own status (same per-system arithmetic as a
// single solve).  Rhs in batch vector B, iterates in X.  With the
// preconditioner, each application solves the blocks of all systems
// together on the replica (R: outer products, RI: inner).
template <typename R, typename RI = R>
void run_batch(const BatchSet& B, const MvmBatch<R>& m, double tol, int maxit, int lag, bool prec, double tol_in,
               int maxit_in, bool graphs, bool wg, hipStream_t s) {
  const KBatch& k = B.k;
  const int nsys = B.nsys;
  auto vec = [&](int kind) { return B.vec(kind); };
  vie::k_init(k, vec(BV_B), vec(BV_X), vec(BV_R), vec(BV_RHAT), nullptr, s);
  vie::k_finalize(k, vie::FIN_INIT, s, nullptr, tol, maxit);
  const StepVecs vv{vec(BV_X), vec(BV_R), vec(BV_RHAT), vec(BV_P), vec(BV_V), vec(BV_S), vec(BV_T)};
  // y = K2^{-1} w for every system: to the stacked layout (systems that no
  // longer iterate give zero right-hand sides, which the inner solves
  // skip), one application on the replica, back
  auto apply = [&](const c128* w, c128* y) {
    vie::batch_to_stacked(w, vec(BV_WI), nsys, B.nv, B.status, s);
    precond_apply<RI>(*B.replica, vec(BV_WI), vec(BV_WO), tol_in, maxit_in, nullptr, lag, nullptr, 0, graphs, wg, s);
    vie::stacked_to_batch(vec(BV_WO), y, nsys, B.nv, s);
  };
  Poller poll(B.poll, s, 0);
  for (int it = 1; it <= maxit; ++it) {
    if (!prec) {
      fused_step<R>(m, k, vv, s);
      const long t = poll.push_step_end(k);
      if (t - lag >= 0 && poll.wait(t - lag) == 0) break;
      continue;
    } else {
      vie::k_update_p(k, vec(BV_R), vec(BV_V), vec(BV_P), s);
      apply(vec(BV_P), vec(BV_Y));
      const vie::FuseArgs fa{0, 1, nullptr, nullptr, nullptr, vec(BV_RHAT), nullptr};
      vie::mvm_pass1<R>(m, &k, fa, vec(BV_Y), false, s);
      vie::mvm_mid<R>(m, s);
      vie::mvm_pass5<R>(m, &k, fa, vec(BV_Y), vec(BV_V), s);
      vie::k_finalize(k, vie::FIN_ALPHA, s);
      vie::k_update_s(k, vec(BV_R), vec(BV_V), vec(BV_S), s);
      vie::k_finalize(k, vie::FIN_S, s);
      apply(vec(BV_S), vec(BV_Z));
      const vie::FuseArgs fo{0, 2, nullptr, nullptr, nullptr, nullptr, vec(BV_S)};
      vie::mvm_pass1<R>(m, &k, fo, vec(BV_Z), false, s);
      vie::mvm_mid<R>(m, s);
      vie::mvm_pass5<R>(m, &k, fo, vec(BV_Z), vec(BV_T), s);
      vie::k_finalize(k, vie::FIN_OMEGA, s);
      vie::k_update_xr(k, vec(BV_X), vec(BV_Y), vec(BV_Z), vec(BV_R), vec(BV_S), vec(BV_T), vec(BV_RHAT), s);
      vie::k_finalize(k, vie::FIN_XR, s);
    }
    const long t = poll.push_count(B.status, nsys, B.count);
    if (t - lag >= 0 && poll.wait(t - lag) == 0) break;
  }
  hip_check(hipStreamSynchronize(s), "batch solve");
}

// nrhs right-hand sides of one problem in one batch.
template <typename R, typename RI = R>
void run_bicgstab_batch(vie_problem& P, int nrhs, double tol, int maxit, int lag, bool prec, double tol_in,
                        int maxit_in, bool graphs, bool wg, hipStream_t s) {
  const BatchSet B{P, P.replica.get(), nrhs, P.nv, P.mr_vecs.as<c128>(), batch_kbatch(P, nrhs),
                   P.mr_status.as<int>(), P.mr_count.as<int>()};
  run_batch<R, RI>(B, batch_mvm<R>(P, nrhs), tol, maxit, lag, prec, tol_in, maxit_in, graphs, wg, s);
}

// The plan of nrhs copies of a problem stacked along z, with block ids
// offset per copy and the original shape groups (so every block is solved
// with the same transform lengths and box as in the problem itself).
// Rooftop plans stacked along z: the per-face 1/chi and owners are
// component-major ([3][copies x nz][ny][nx], the layout batch_to_stacked
// gives the vectors), copy r's block ids shifted by off[r].  Faces between
// copies carry no unknown: every copy's first and last z layer is vacuum.
void stack_faces(ProblemPlan& sp, const std::vector<const ProblemPlan*>& pls, const std::vector<int>& off) {
  sp.rooftop = true;
  sp.chi.clear();
  sp.bid3.clear();
  sp.chi.reserve(3 * (size_t)sp.nv);
  sp.bid3.reserve(3 * (size_t)sp.nv);
  for (int c = 0; c < 3; ++c)
    for (size_t r = 0; r < pls.size(); ++r) {
      const ProblemPlan& pl = *pls[r];
      sp.chi.insert(sp.chi.end(), pl.chi.begin() + (size_t)c * pl.nv, pl.chi.begin() + (size_t)(c + 1) * pl.nv);
      for (int64_t i = 0; i < pl.nv; ++i) {
        const int32_t b = pl.bid3[(size_t)c * pl.nv + i];
        sp.bid3.push_back(b < 0 ? -1 : b + off[r]);
      }
    }
}

ProblemPlan stacked_plan(const ProblemPlan& pl, int nrhs) {
  ProblemPlan sp;
  sp.g = pl.g;
  sp.g.nz = pl.g.nz * nrhs;
  sp.nv = pl.nv * nrhs;
  sp.k0 = pl.k0;
  sp.has_blocks = pl.has_blocks;
  sp.overlap = pl.overlap;
  const int nb = pl.n_blocks;
  sp.n_blocks = nb * nrhs;
  sp.chi.reserve((size_t)sp.nv);
  sp.bid.reserve((size_t)sp.nv);
  for (int r = 0; r < nrhs; ++r) {
    sp.chi.insert(sp.chi.end(), pl.chi.begin(), pl.chi.end());
    for (int32_t b : pl.bid) sp.bid.push_back(b < 0 ? -1 : b + r * nb);
    for (int k = 0; k < nb; ++k) {
      for (int a = 0; a < 3; ++a) {
        sp.lo.push_back(pl.lo[3 * k + a] + (a == 2 ? r * pl.g.nz : 0));
        sp.hi.push_back(pl.hi[3 * k + a] + (a == 2 ? r * pl.g.nz : 0));
      }
    }
    sp.cnt.insert(sp.cnt.end(), pl.cnt.begin(), pl.cnt.end());
    if (pl.overlap > 0) sp.emask.insert(sp.emask.end(), pl.emask.begin(), pl.emask.end());
  }
  for (const auto& gp : pl.groups) {
    GroupPlan g2 = gp;
    g2.blocks.clear();
    for (int r = 0; r < nrhs; ++r)
      for (int k : gp.blocks) g2.blocks.push_back(k + r * nb);
    sp.groups.push_back(std::move(g2));
  }
  if (pl.rooftop) {
    std::vector<const ProblemPlan*> pls(nrhs, &pl);
    std::vector<int> off(nrhs);
    for (int r = 0; r < nrhs; ++r) off[r] = r * nb;
    stack_faces(sp, pls, off);
  }
  return sp;
}

std::unique_ptr<vie_problem> build_problem(vie_context* ctx, const ProblemPlan& pl, hipStream_t s,
                                           bool inner_only = false);

// Device memory of an inner-only problem built from plan sp (block
// vectors, work buffers and state; spectra are the context's).
size_t replica_bytes(const ProblemPlan& sp) {
  size_t foot = 0;
  for (const auto& gp : sp.groups) {
    const size_t nsys = gp.blocks.size(), bnv = (size_t)gp.bx * gp.by * gp.bz;
    foot += nsys * (sp.rooftop ? 3 : 1) * bnv * sizeof(c128) + nsys * 3 * (size_t)gp.bz * gp.ly * gp.lx * sizeof(c128) +
            8 * nsys * 3 * bnv * sizeof(c128) + nsys * (sizeof(KState) + 2 * sizeof(int));
  }
  foot += (size_t)sp.nv * (sizeof(int32_t) + 4 * sizeof(int));   // block map
  return foot;
}

// The replica problem for preconditioned batches of nrhs right-hand sides
// (rebuilt when nrhs changes; counted in the problem's footprint).
void ensure_replica(vie_problem& P, int nrhs, hipStream_t s) {
  if (P.replica && P.replica_nrhs == nrhs) return;
  if (!P.plan) fail(VIE_EINVAL, "this problem keeps no plan for batched preconditioned solves");
  vie_context* ctx = P.ctx;
  const size_t old = P.replica_bytes;
  P.replica.reset();
  P.replica_nrhs = 0;
  P.replica_bytes = 0;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= std::min(ctx->used, old);
  }
  P.footprint -= std::min(P.footprint, old);
  const ProblemPlan sp = stacked_plan(*P.plan, nrhs);
  const size_t foot = replica_bytes(sp);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->budget && ctx->used + ctx->reserved + foot > ctx->budget)
      fail(VIE_EBUSY, "batch replica exceeds the context's HBM budget");
    ctx->used += foot;
  }
  try {
    P.replica = build_problem(ctx, sp, s, true);
  } catch (...) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= std::min(ctx->used, foot);
    throw;
  }
  P.replica_nrhs = nrhs;
  P.replica_bytes = foot;
  P.footprint += foot;
}

// Several problems of one grid shape in one batch (vie_solve_many): their
// blocks stacked along z in problem order (block ids offset per problem),
// regrouped across problems by box shape and FFT lengths, every block with
// its own problem's spacing and k0 (its spectra); all groups batched.
ProblemPlan fleet_plan(const std::vector<vie_problem*>& ps) {
  const ProblemPlan& p0 = *ps[0]->plan;
  ProblemPlan sp;
  sp.g = p0.g;
  sp.g.nz = p0.g.nz * (int)ps.size();
  sp.nv = p0.nv * (int64_t)ps.size();
  sp.k0 = p0.k0;
  sp.lx = p0.lx;
  sp.ly = p0.ly;
  sp.lz = p0.lz;
  sp.has_blocks = true;
  sp.overlap = p0.overlap;
  std::map<std::array<int, 6>, size_t> key_group;
  int off = 0;
  for (size_t r = 0; r < ps.size(); ++r) {
    const ProblemPlan& pl = *ps[r]->plan;
    const int nb = pl.n_blocks;
    sp.chi.insert(sp.chi.end(), pl.chi.begin(), pl.chi.end());
    for (int32_t b : pl.bid) sp.bid.push_back(b < 0 ? -1 : b + off);
    for (int k = 0; k < nb; ++k) {
      for (int a = 0; a < 3; ++a) {
        sp.lo.push_back(pl.lo[3 * k + a] + (a == 2 ? (int)r * p0.g.nz : 0));
        sp.hi.push_back(pl.hi[3 * k + a] + (a == 2 ? (int)r * p0.g.nz : 0));
      }
      sp.blk_phys.insert(sp.blk_phys.end(), {pl.g.dx, pl.g.dy, pl.g.dz, pl.k0});
    }
    sp.cnt.insert(sp.cnt.end(), pl.cnt.begin(), pl.cnt.end());
    if (pl.overlap > 0) sp.emask.insert(sp.emask.end(), pl.emask.begin(), pl.emask.end());
    for (const auto& gp : pl.groups) {
      const std::array<int, 6> key{gp.lx, gp.ly, gp.lz, gp.bx, gp.by, gp.bz};
      auto it = key_group.find(key);
      if (it == key_group.end()) {
        GroupPlan g2 = gp;
        g2.blocks.clear();
        g2.wg = false;
        it = key_group.emplace(key, sp.groups.size()).first;
        sp.groups.push_back(std::move(g2));
      }
      for (int k : gp.blocks) sp.groups[it->second].blocks.push_back(k + off);
    }
    off += nb;
  }
  sp.n_blocks = off;
  if (p0.rooftop) {
    std::vector<const ProblemPlan*> pls;
    std::vector<int> offs;
    int o = 0;
    for (vie_problem* q : ps) {
      pls.push_back(q->plan.get());
      offs.push_back(o);
      o += q->plan->n_blocks;
    }
    stack_faces(sp, pls, offs);
  }
  return sp;
}

// The batch state of a vie_solve_many call: 1/chi of every problem,
// per-problem spectrum tables, work buffer, vectors, Krylov state and the
// replica; counted against the context's budget while it lives.
struct Fleet {
  vie_context* ctx;
  size_t bytes = 0;
  DevBuf chi, tab, work, vecs, state, status, partials, partials2, ntile, count;
  std::unique_ptr<vie_problem> replica;
  explicit Fleet(vie_context* c) : ctx(c) {}
  ~Fleet() {
    replica.reset();
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= std::min(ctx->used, bytes);
  }
};

template <typename R>
MvmBatch<R> fleet_mvm(vie_problem& P0, Fleet& F, int n) {
  MvmBatch<R> b = outer_batch<R>(P0, true);   // the first problem's shape and kernel variants
  b.nsys = n;
  b.cstride = chi_period(P0);
  b.chi_inv = F.chi.as<c128>();
  b.spec_tab = F.tab.as<const cx<R>*>() + (sizeof(R) == sizeof(float) ? n : 0);
  b.work = F.work.as<cx<R>>();
  b.status = F.status.as<int>();
  return b;
}

// ------------------------------------------------------------------ problem set-up
// Expanded blocks: the set of block k grows by `m` voxels in every axis (a
// (2m+1)^3 cube dilation, separable into three 1-D running maxima) and is
// cut to the scatterer; lo/hi become the set's tight bounding box.
void expand_blocks(ProblemPlan& pl, int m) {
  const vie_grid& g = pl.g;
  const int n_blocks = pl.n_blocks;
  pl.overlap = m;
  pl.emask.assign(n_blocks, {});
  for (int k = 0; k < n_blocks; ++k) {
    if (pl.cnt[k] == 0) continue;
    int b0[3], ext[3];
    const int dims[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
      b0[a] = std::max(0, pl.lo[3 * k + a] - m);
      ext[a] = std::min(dims[a] - 1, pl.hi[3 * k + a] + m) - b0[a] + 1;
    }
    const int64_t bn = (int64_t)ext[0] * ext[1] * ext[2];
    auto at = [&](int x, int y, int z) { return ((int64_t)z * ext[1] + y) * ext[0] + x; };
    std::vector<uint8_t> cur(bn, 0), nxt(bn, 0);
    for (int z = 0; z < ext[2]; ++z)
      for (int y = 0; y < ext[1]; ++y)
        for (int x = 0; x < ext[0]; ++x) {
          const int64_t v = ((int64_t)(b0[2] + z) * g.ny + (b0[1] + y)) * g.nx + (b0[0] + x);
          cur[at(x, y, z)] = pl.bid[v] == k;
        }
    for (int a = 0; a < 3; ++a) {   // running max of radius m along axis a
      for (int z = 0; z < ext[2]; ++z)
        for (int y = 0; y < ext[1]; ++y)
          for (int x = 0; x < ext[0]; ++x) {
            const int c[3] = {x, y, z};
            uint8_t v = 0;
            for (int d = -m; d <= m && !v; ++d) {
              int q[3] = {x, y, z};
              q[a] = c[a] + d;
              if (q[a] < 0 || q[a] >= ext[a]) continue;
              v = cur[at(q[0], q[1], q[2])];
            }
            nxt[at(x, y, z)] = v;
          }
      std::swap(cur, nxt);
    }
    int lo[3] = {ext[0], ext[1], ext[2]}, hi[3] = {-1, -1, -1};
    for (int z = 0; z < ext[2]; ++z)
      for (int y = 0; y < ext[1]; ++y)
        for (int x = 0; x < ext[0]; ++x) {
          const int64_t v = ((int64_t)(b0[2] + z) * g.ny + (b0[1] + y)) * g.nx + (b0[0] + x);
          uint8_t& e = cur[at(x, y, z)];
          e = e && (pl.chi[v].x != 0.0 || pl.chi[v].y != 0.0);
          if (!e) continue;
          const int c[3] = {x, y, z};
          for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], c[a]);
            hi[a] = std::max(hi[a], c[a]);
          }
        }
    std::vector<uint8_t>& em = pl.emask[k];
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    em.assign((size_t)ex * ey * ez, 0);
    for (int z = 0; z < ez; ++z)
      for (int y = 0; y < ey; ++y)
        for (int x = 0; x < ex; ++x) em[((size_t)z * ey + y) * ex + x] = cur[at(lo[0] + x, lo[1] + y, lo[2] + z)];
    for (int a = 0; a < 3; ++a) {
      pl.lo[3 * k + a] = b0[a] + lo[a];
      pl.hi[3 * k + a] = b0[a] + hi[a];
    }
  }
}

// rooftop: every block's box grows by one cell per side (the cells whose
// faces and charges the block's face unknowns touch), and no group uses the
// one-workgroup block solver (its kernels are collocated only).
ProblemPlan make_plan(const vie_grid& g, const double* eps_r, const int32_t* block_id, int32_t n_blocks,
                      int overlap = 0, bool rooftop = false) {
  if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > 256 || g.ny > 256 || g.nz > 256)
    fail(VIE_EINVAL, "grid sizes must be in [1, 256]");
  if (!(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0) || !(g.wavelength > 0) || !is_finite(g.dx) || !is_finite(g.dy) ||
      !is_finite(g.dz) || !is_finite(g.wavelength))
    fail(VIE_EINVAL, "spacing and wavelength must be finite and > 0");
  if (block_id && n_blocks < 1) fail(VIE_EINVAL, "n_blocks must be >= 1 when block_id is given");
  if (n_blocks < 0) fail(VIE_EINVAL, "n_blocks must be >= 0");
  ProblemPlan pl;
  pl.g = g;
  const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
  pl.nv = nv;
  // 1/chi on the host
  pl.chi.resize(nv);
  for (int64_t i = 0; i < nv; ++i) {
    const double er = eps_r[2 * i], ei = eps_r[2 * i + 1];
    if (!is_finite(er) || !is_finite(ei)) fail(VIE_EINVAL, "eps_r has non-finite entries");
    if (er == 1.0 && ei == 0.0) {
      pl.chi[i] = mk<double>(0.0, 0.0);
    } else {
      const std::complex<double> c = 1.0 / (std::complex<double>(er, ei) - 1.0);
      pl.chi[i] = mk<double>(c.real(), c.imag());
    }
  }
  pl.lx = vie::smallest_fft_length(2 * g.nx - 1, true);
  pl.ly = vie::smallest_fft_length(2 * g.ny - 1, true);
  pl.lz = vie::smallest_fft_length(2 * g.nz - 1);
  if (pl.lx < 0 || pl.ly < 0 || pl.lz < 0) fail(VIE_EINVAL, "grid too large for the compiled FFT lengths");
  pl.k0 = 2.0 * M_PI / g.wavelength;
  if (!block_id) return pl;
  pl.has_blocks = true;
  pl.n_blocks = n_blocks;
  pl.bid.assign(nv, -1);
  for (int64_t i = 0; i < nv; ++i) {
    const bool vac = pl.chi[i].x == 0.0 && pl.chi[i].y == 0.0;
    if (vac) continue;
    const int32_t k = block_id[i];
    if (k < 0 || k >= n_blocks) fail(VIE_EINVAL, "block id out of range on a scatterer voxel");
    pl.bid[i] = k;
  }
  // tight bounding box of every block
  auto& lo = pl.lo;
  auto& hi = pl.hi;
  auto& cnt = pl.cnt;
  lo.assign(3 * n_blocks, 1 << 30);
  hi.assign(3 * n_blocks, -1);
  cnt.assign(n_blocks, 0);
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const int k = pl.bid[((int64_t)z * g.ny + y) * g.nx + x];
        if (k < 0) continue;
        cnt[k]++;
        const int c[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
          lo[3 * k + a] = std::min(lo[3 * k + a], c[a]);
          hi[3 * k + a] = std::max(hi[3 * k + a], c[a]);
        }
      }
  if (overlap > 0) expand_blocks(pl, overlap);
  if (rooftop) {
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < n_blocks; ++k)
      if (cnt[k] > 0)
        for (int a = 0; a < 3; ++a) {
          lo[3 * k + a] = std::max(0, lo[3 * k + a] - 1);
          hi[3 * k + a] = std::min(n[a] - 1, hi[3 * k + a] + 1);
        }
  }
  // group blocks by circulant lengths of their bounding boxes
  std::vector<GroupPlan> plans;
  {
    std::map<std::tuple<int, int, int>, std::vector<int>> bylen;
    for (int k = 0; k < n_blocks; ++k) {
      if (cnt[k] == 0) continue;
      const int ex = hi[3 * k] - lo[3 * k] + 1, ey = hi[3 * k + 1] - lo[3 * k + 1] + 1,
                ez = hi[3 * k + 2] - lo[3 * k + 2] + 1;
      bylen[{vie::smallest_fft_length(2 * ex - 1, true), vie::smallest_fft_length(2 * ey - 1, true),
             vie::smallest_fft_length(2 * ez - 1)}]
          .push_back(k);
    }
    for (auto& kv : bylen) {
      GroupPlan gp;
      gp.lx = std::get<0>(kv.first);
      gp.ly = std::get<1>(kv.first);
      gp.lz = std::get<2>(kv.first);
      gp.blocks = kv.second;
      plans.push_back(std::move(gp));
    }
  }
  // Shapes the one-workgroup block solver handles stay separate groups
  // (one launch per group and application, whatever the group size).
  std::vector<GroupPlan> wg_plans;
  {
    std::vector<GroupPlan> rest;
    for (auto& gp : plans) {
      int bz = 1;
      for (int k : gp.blocks) bz = std::max(bz, hi[3 * k + 2] - lo[3 * k + 2] + 1);
      gp.wg = !rooftop && vie::block_solver_supported(gp.lx, gp.ly, gp.lz, bz);
      (gp.wg ? wg_plans : rest).push_back(std::move(gp));
    }
    plans = std::move(rest);
  }
  // Merge shape groups while it lowers the modelled cost of one inner
  // iteration: a fixed per-group overhead (its kernel launches) plus
  // work proportional to the padded transform volume of its systems.
  // A merged group takes the largest lengths of both (a box of n <=
  // (L+1)/2 voxels embeds in any longer L).
  {
    // ~11 launches of >= 5 us per group and step, against ~50 ps per padded
    // point and step (two products and the vector updates) on MI355X
    const double kGroupOverhead = 1.2e6;  // padded points per group-iteration overhead
    auto cost = [&](int lx, int ly, int lz, size_t nsys) { return kGroupOverhead + (double)nsys * lx * ly * lz; };
    for (;;) {
      double best = 0;
      int bi = -1, bj = -1;
      for (size_t i = 0; i < plans.size(); ++i)
        for (size_t j = i + 1; j < plans.size(); ++j) {
          const GroupPlan &a = plans[i], &b = plans[j];
          const int lx = std::max(a.lx, b.lx), ly = std::max(a.ly, b.ly), lz = std::max(a.lz, b.lz);
          const double d = cost(lx, ly, lz, a.blocks.size() + b.blocks.size()) -
                           cost(a.lx, a.ly, a.lz, a.blocks.size()) - cost(b.lx, b.ly, b.lz, b.blocks.size());
          if (d < best) {
            best = d;
            bi = (int)i;
            bj = (int)j;
          }
        }
      if (bi < 0) break;
      GroupPlan& a = plans[bi];
      GroupPlan& b = plans[bj];
      a.lx = std::max(a.lx, b.lx);
      a.ly = std::max(a.ly, b.ly);
      a.lz = std::max(a.lz, b.lz);
      a.blocks.insert(a.blocks.end(), b.blocks.begin(), b.blocks.end());
      std::sort(a.blocks.begin(), a.blocks.end());
      plans.erase(plans.begin() + bj);
    }
  }
  for (auto& gp : wg_plans) plans.push_back(std::move(gp));
  for (auto& gp : plans)
    for (int k : gp.blocks) {
      gp.bx = std::max(gp.bx, hi[3 * k] - lo[3 * k] + 1);
      gp.by = std::max(gp.by, hi[3 * k + 1] - lo[3 * k + 1] + 1);
      gp.bz = std::max(gp.bz, hi[3 * k + 2] - lo[3 * k + 2] + 1);
    }
  pl.groups = std::move(plans);
  return pl;
}

// Rooftop discretisation (Sec. II-A, eq. (5)): the unknowns are the normal
// components of P on the faces between cells.  Face c + e_i / 2 (index c of
// component i) joins cells c and c + e_i; the normal flux density is
// continuous across it, so the face's field is D times the mean m of 1/eps
// of the two cells, and P = D - E gives the face contrast chi_f = (1 - m) / m,
// stored as 1/chi_f = m / (1 - m).  Faces between two vacuum cells, faces
// past the grid's last layer and faces with m = 1 carry no unknown
// (1/chi_f = 0).  The first and last cell layers of every axis must be
// vacuum: every face with an unknown then lies inside the grid, and the
// cell divergence and the face gradient need no boundary terms.
ProblemPlan make_plan_rooftop(const vie_grid& g, const double* eps_r, const int32_t* block_id, int32_t n_blocks) {
  // sizes, finiteness, FFT lengths, block ids and boxes
  ProblemPlan pl = make_plan(g, eps_r, block_id, n_blocks, 0, true);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int64_t nv = pl.nv;
  auto vac = [&](int64_t i) { return eps_r[2 * i] == 1.0 && eps_r[2 * i + 1] == 0.0; };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const bool edge = x == 0 || y == 0 || z == 0 || x == nx - 1 || y == ny - 1 || z == nz - 1;
        if (edge && !vac(((int64_t)z * ny + y) * nx + x))
          fail(VIE_EINVAL, "rooftop problems need vacuum in the first and last cell layer of every axis");
      }
  auto inv_eps = [&](int64_t i) {
    return vac(i) ? std::complex<double>(1.0, 0.0) : 1.0 / std::complex<double>(eps_r[2 * i], eps_r[2 * i + 1]);
  };
  std::vector<c128> chi(3 * (size_t)nv, mk<double>(0.0, 0.0));
  const int64_t step[3] = {1, nx, (int64_t)nx * ny};
  for (int c = 0; c < 3; ++c)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int pos[3] = {x, y, z}, n[3] = {nx, ny, nz};
          if (pos[c] == n[c] - 1) continue;
          const int64_t i = ((int64_t)z * ny + y) * nx + x, j = i + step[c];
          if (vac(i) && vac(j)) continue;
          const std::complex<double> m = 0.5 * (inv_eps(i) + inv_eps(j));
          if (m == 1.0) continue;
          const std::complex<double> v = m / (1.0 - m);
          chi[(size_t)c * nv + i] = mk<double>(v.real(), v.imag());
        }
  pl.chi = std::move(chi);
  pl.rooftop = true;
  if (pl.has_blocks) {
    // a face belongs to the block of its lower cell when that cell is a
    // scatterer cell, else to the block of its upper cell (eq. (10)
    // partitions the unknowns; the blocks are sets of cells)
    pl.bid3.assign(3 * (size_t)nv, -1);
    for (int c = 0; c < 3; ++c)
      for (int64_t i = 0; i < nv; ++i) {
        const c128 f = pl.chi[(size_t)c * nv + i];
        if (f.x == 0.0 && f.y == 0.0) continue;
        pl.bid3[(size_t)c * nv + i] = pl.bid[i] >= 0 ? pl.bid[i] : pl.bid[i + step[c]];
      }
  }
  return pl;
}

size_t spectra_bytes(int lx, int ly, int lz, int kind = 0) {
  return (size_t)spectra_elems(lx, ly, lz, kind) * (sizeof(c128) + sizeof(c64));
}

bool spectra_cached(vie_context* ctx, int lx, int ly, int lz, const vie_grid& g, double k0, int kind = 0) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->cache.find(SpecKey{lx, ly, lz, g.dx, g.dy, g.dz, k0, kind});
  return it != ctx->cache.end() && !it->second.expired();
}

// Device bytes a problem built from `pl` holds.  Spectra already in the
// context's cache are shared and not counted, unless `all_spectra` (a
// request's reservation: the cache holds weak references, so spectra cached
// at submission may be gone when the request is built).
size_t plan_footprint(vie_context* ctx, const ProblemPlan& pl, bool all_spectra = false) {
  const auto& g = pl.g;
  const size_t nv = (size_t)pl.nv;
  size_t foot = (pl.rooftop ? 3 : 1) * nv * sizeof(c128)                 // 1/chi
                + 3 * (size_t)g.nz * pl.ly * pl.lx * sizeof(c128)       // work
                + V_COUNT * 3 * nv * sizeof(c128)                       // Krylov vectors
                + 2 * 4 * (size_t)std::max(vie::krylov_chunks(3 * (int64_t)nv), vie::mvm_row_tiles(pl.lx, g.nz, g.ny)) *
                      sizeof(double);   // two partial buffers
  std::set<std::tuple<int, int, int>> seen;
  const int kind = pl.rooftop ? 1 : 0;
  auto spec = [&](int lx, int ly, int lz) {
    if (seen.insert({lx, ly, lz}).second && (all_spectra || !spectra_cached(ctx, lx, ly, lz, g, pl.k0, kind)))
      foot += spectra_bytes(lx, ly, lz, kind);
  };
  spec(pl.lx, pl.ly, pl.lz);
  int64_t ipstride = 0, slots = 0;
  for (const auto& gp : pl.groups) {
    const size_t nsys = gp.blocks.size(), bnv = (size_t)gp.bx * gp.by * gp.bz;
    foot += nsys * (pl.rooftop ? 3 : 1) * bnv * sizeof(c128) + nsys * 3 * (size_t)gp.bz * gp.ly * gp.lx * sizeof(c128) +
            8 * nsys * 3 * bnv * sizeof(c128);
    spec(gp.lx, gp.ly, gp.lz);
    ipstride = std::max<int64_t>(ipstride, 4 * std::max(vie::krylov_chunks(3 * (int64_t)bnv),
                                                        vie::mvm_row_tiles(gp.lx, gp.bz, gp.by)));
    slots += (int64_t)nsys;
  }
  foot += 2 * (size_t)std::max<int64_t>(1, slots) * ipstride * sizeof(double);   // two partial buffers
  return foot;
}

// z-pass variant for a batch shape: tuned once per context, shape and
// precision, so every problem of that shape uses the same kernels.
template <typename R>
int cached_zvariant(vie_context* ctx, const MvmBatch<R>& b, hipStream_t s, float* ms) {
  const std::array<int, 8> key{(int)sizeof(R) + 64 * b.rooftop, b.nx, b.ny, b.nz, b.lx, b.ly, b.lz, b.nsys};
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->ztune.find(key);
    if (it != ctx->ztune.end()) {
      if (ms)
        for (int v = 0; v < vie::kZPassVariants; ++v) ms[v] = it->second.second[v];
      return it->second.first;
    }
  }
  std::array<float, vie::kZPassVariants> t{};
  const int v = vie::tune_zpass<R>(b, s, t.data());
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->ztune.emplace(key, std::make_pair(v, t)).first;   // first tuning wins
  if (ms)
    for (int q = 0; q < vie::kZPassVariants; ++q) ms[q] = it->second.second[q];
  return it->second.first;
}

// Plane-kernel variant for a batch shape, tuned once per context, shape and
// precision as the z pass; x and y: device vectors of the batch that hold
// no data yet (clobbered).
template <typename R>
int cached_pvariant(vie_context* ctx, const MvmBatch<R>& b, const c128* x, c128* y, hipStream_t s, float* ms) {
  const std::array<int, 8> key{(int)sizeof(R) + 64 * b.rooftop, b.nx, b.ny, b.nz, b.lx, b.ly, b.lz, b.nsys};
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->ptune.find(key);
    if (it != ctx->ptune.end()) {
      if (ms)
        for (int v = 0; v < vie::kPlaneVariants; ++v) ms[v] = it->second.second[v];
      return it->second.first;
    }
  }
  std::array<float, vie::kPlaneVariants> t{};
  const int v = vie::tune_plane<R>(b, x, y, s, t.data());
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->ptune.emplace(key, std::make_pair(v, t)).first;   // first tuning wins
  if (ms)
    for (int q = 0; q < vie::kPlaneVariants; ++q) ms[q] = it->second.second[q];
  return it->second.first;
}

// inner_only: the blocks and their inner solves only (no full-grid operator:
// no outer spectra, work buffer or Krylov vectors); used for the stacked
// replica of preconditioned batches.
std::unique_ptr<vie_problem> build_problem(vie_context* ctx, const ProblemPlan& pl, hipStream_t s,
                                           bool inner_only) {
  const vie_grid& g = pl.g;
  const int64_t nv = pl.nv;
  auto P = std::make_unique<vie_problem>();
  P->ctx = ctx;
  P->g = g;
  P->nv = nv;
  P->lx = pl.lx;
  P->ly = pl.ly;
  P->lz = pl.lz;
  P->k0 = pl.k0;
  P->overlap = pl.overlap;
  P->rooftop = pl.rooftop;
  if (!inner_only) {
    P->spec = get_spectra(ctx, P->lx, P->ly, P->lz, g.dx, g.dy, g.dz, P->k0, s, pl.rooftop ? 1 : 0);
    upload(P->chi, pl.chi, s);
    P->work.alloc(3 * (size_t)g.nz * P->ly * P->lx * sizeof(c128));
    P->work.zero(s);
    P->vecs.alloc(V_COUNT * 3 * (size_t)nv * sizeof(c128));
    P->vecs.zero(s);
    for (int k = 0; k < V_COUNT; ++k) P->vec[k] = P->vecs.as<c128>() + (size_t)k * 3 * nv;
    P->pstride = 4 * std::max(vie::krylov_chunks(3 * nv), vie::mvm_row_tiles(P->lx, g.nz, g.ny));
    P->partials.alloc(P->pstride * sizeof(double));
    P->partials2.alloc(P->pstride * sizeof(double));
  }
  P->ntile.alloc(sizeof(int));
  P->ntile.zero(s);
  P->ostate.alloc(sizeof(KState));
  P->ostate.zero(s);
  P->ostatus.alloc(sizeof(int));
  P->ostatus.zero(s);
  P->scal.alloc(64);
  const int rings = 1 + (int)pl.groups.size();   // outer loop, then one per group
  P->d_count.alloc(rings * sizeof(int));
  P->d_acc.alloc(3 * sizeof(int64_t));
  P->d_acc.zero(s);
  {
    ApiShared api;
    hip_check(hipHostMalloc((void**)&P->h_ring, (size_t)rings * kRing * sizeof(int)), "pinned ring");
  }
  {
    void* dv = nullptr;
    if (hipHostGetDevicePointer(&dv, P->h_ring, 0) == hipSuccess && dv)
      P->d_ring = static_cast<int*>(dv);
    else
      (void)hipGetLastError();
  }
  {
    ApiShared api;
    P->ev.resize(rings);
    for (auto& r : P->ev) r.fill(nullptr);
    for (auto& r : P->ev)
      for (auto& e : r) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  }

  if (pl.has_blocks) {
    const int n_blocks = pl.n_blocks;
    const auto& lo = pl.lo;
    const auto& bid = pl.bid;
    P->n_blocks = n_blocks;
    std::vector<int> block_group(n_blocks, -1), block_sys(n_blocks, -1);
    std::vector<int4> origin(n_blocks, int4{0, 0, 0, 0}), gbox;
    int slot = 0;
    for (const auto& gp : pl.groups) {
      Group G{};
      G.lx = gp.lx;
      G.ly = gp.ly;
      G.lz = gp.lz;
      G.blocks = gp.blocks;
      G.wg = gp.wg;
      G.nsys = (int)G.blocks.size();
      G.bx = gp.bx;
      G.by = gp.by;
      G.bz = gp.bz;
      G.bnv = (int64_t)G.bx * G.by * G.bz;
      G.n = 3 * G.bnv;
      const int gi = (int)P->groups.size();
      const int ncc = pl.rooftop ? 3 : 1;   // 1/chi entries per box voxel
      std::vector<c128> gchi((size_t)G.nsys * ncc * G.bnv, mk<double>(0.0, 0.0));
      std::vector<int4> sorg(G.nsys);
      for (int q = 0; q < G.nsys; ++q) {
        const int k = G.blocks[q];
        block_group[k] = gi;
        block_sys[k] = q;
        origin[k] = int4{lo[3 * k], lo[3 * k + 1], lo[3 * k + 2], 0};
        sorg[q] = origin[k];
        const int ex = pl.hi[3 * k] - lo[3 * k] + 1, ey = pl.hi[3 * k + 1] - lo[3 * k + 1] + 1;
        for (int z = 0; z < G.bz; ++z)
          for (int y = 0; y < G.by; ++y)
            for (int x = 0; x < G.bx; ++x) {
              const int X = lo[3 * k] + x, Y = lo[3 * k + 1] + y, Z = lo[3 * k + 2] + z;
              if (X >= g.nx || Y >= g.ny || Z >= g.nz) continue;
              const int64_t v = ((int64_t)Z * g.ny + Y) * g.nx + X;
              // the block's solve set: its own voxels, or the expanded set
              bool in = bid[v] == k;
              if (pl.overlap > 0)
                in = X <= pl.hi[3 * k] && Y <= pl.hi[3 * k + 1] && Z <= pl.hi[3 * k + 2] &&
                     pl.emask[k][((size_t)z * ey + y) * ex + x] != 0;
              const int64_t loc = ((int64_t)z * G.by + y) * G.bx + x;
              if (pl.rooftop) {   // the faces block k owns
                for (int c = 0; c < 3; ++c)
                  if (pl.bid3[(size_t)c * nv + v] == k)
                    gchi[((size_t)q * 3 + c) * G.bnv + loc] = pl.chi[(size_t)c * nv + v];
              } else if (in) {
                gchi[(size_t)q * G.bnv + loc] = pl.chi[v];
              }
            }
      }
      gbox.push_back(int4{G.bx, G.by, G.bz, 0});
      upload(G.chi, gchi, s);
      if (pl.overlap > 0) upload(G.sys_origin, sorg, s);
      if (pl.blk_phys.empty()) {
        G.spec = get_spectra(ctx, G.lx, G.ly, G.lz, g.dx, g.dy, g.dz, P->k0, s, pl.rooftop ? 1 : 0);
      } else {
        bool same = true;
        for (int q = 0; q < G.nsys; ++q) {
          const double* ph = &pl.blk_phys[4 * (size_t)G.blocks[q]];
          G.sys_spec.push_back(get_spectra(ctx, G.lx, G.ly, G.lz, ph[0], ph[1], ph[2], ph[3], s, pl.rooftop ? 1 : 0));
          same = same && G.sys_spec.back() == G.sys_spec.front();
        }
        G.spec = G.sys_spec.front();
        if (same) {
          G.sys_spec.clear();
        } else {
          std::vector<const void*> tab(2 * (size_t)G.nsys);
          for (int q = 0; q < G.nsys; ++q) {
            tab[q] = spec_ptr<double>(*G.sys_spec[q]);
            tab[G.nsys + q] = spec_ptr<float>(*G.sys_spec[q]);
          }
          upload(G.spec_tab, tab, s);
        }
      }
      G.work.alloc((size_t)G.nsys * 3 * G.bz * G.ly * G.lx * sizeof(c128));
      G.work.zero(s);
      G.vecs.alloc(8 * (size_t)G.nsys * G.n * sizeof(c128));
      G.vecs.zero(s);
      for (int q = 0; q < 8; ++q) G.vec[q] = G.vecs.as<c128>() + (size_t)q * G.nsys * G.n;
      P->ipstride =
          std::max<int64_t>(P->ipstride, 4 * std::max(vie::krylov_chunks(G.n), vie::mvm_row_tiles(G.lx, G.bz, G.by)));
      G.slot0 = slot;
      slot += G.nsys;
      P->groups.push_back(std::move(G));
    }
    P->n_inner = slot;
    for (auto& G : P->groups) {
      if (G.wg)
        ++P->n_wg_groups;
      else
        P->n_batched_wg += G.nsys;
    }
    std::vector<int> slots;
    for (int k = 0; k < n_blocks; ++k)
      if (pl.cnt[k] > 0) slots.push_back(P->groups[block_group[k]].slot0 + block_sys[k]);
    P->n_nonempty = (int)slots.size();
    upload(P->d_block_id, pl.rooftop ? pl.bid3 : bid, s);
    upload(P->d_block_group, block_group, s);
    upload(P->d_block_sys, block_sys, s);
    upload(P->d_block_origin, origin, s);
    upload(P->d_gbox, gbox, s);
    upload(P->d_slots, slots, s);
    std::vector<c128*> ptrs(8 * P->groups.size());
    for (size_t gi = 0; gi < P->groups.size(); ++gi)
      for (int q = 0; q < 8; ++q) ptrs[q * P->groups.size() + gi] = P->groups[gi].vec[q];
    upload(P->d_gptr, ptrs, s);
    P->d_istatus.alloc(std::max(1, slot) * sizeof(int));
    P->d_istatus.zero(s);
    P->d_istate.alloc(std::max(1, slot) * sizeof(KState));
    P->d_istate.zero(s);
    P->d_ipartials.alloc((size_t)std::max(1, slot) * P->ipstride * sizeof(double));
    P->d_ipartials2.alloc((size_t)std::max(1, slot) * P->ipstride * sizeof(double));
    P->d_intile.alloc(std::max(1, slot) * sizeof(int));
    P->d_intile.zero(s);
    // pick the faster z-pass kernel per batch shape and precision (tuning
    // clobbers the work buffers, which hold no data yet)
    for (auto& G : P->groups) {
      G.zvar[0] = cached_zvariant<double>(ctx, group_batch<double>(*P, G, false), s, nullptr);
      G.zvar[1] = cached_zvariant<float>(ctx, group_batch<float>(*P, G, false), s, nullptr);
      G.pvar[0] = cached_pvariant<double>(ctx, group_batch<double>(*P, G, false), G.vec[0], G.vec[1], s, nullptr);
      G.pvar[1] = cached_pvariant<float>(ctx, group_batch<float>(*P, G, false), G.vec[0], G.vec[1], s, nullptr);
    }
    if (P->groups.size() > 1) {
      ApiShared api;
      const size_t G = P->groups.size();
      P->branches.streams.resize(G, nullptr);
      for (auto& b : P->branches.streams) hip_check(hipStreamCreateWithFlags(&b, hipStreamNonBlocking), "stream");
      P->branches.events.resize(G + 1, nullptr);
      for (auto& e : P->branches.events) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    }
    if (P->n_wg_groups > 0) {
      ApiShared api;
      P->wg_streams.resize(P->n_wg_groups, nullptr);
      for (auto& b : P->wg_streams) hip_check(hipStreamCreateWithFlags(&b, hipStreamNonBlocking), "stream");
      P->wg_events.resize(1 + P->n_wg_groups, nullptr);
      for (auto& e : P->wg_events) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    }
    vie::BlockMap& m = P->bmap;
    m.nblocks = n_blocks;
    m.ngroups = (int)P->groups.size();
    m.block_id = P->d_block_id.as<int>();
    m.block_group = P->d_block_group.as<int>();
    m.block_sys = P->d_block_sys.as<int>();
    m.block_origin = P->d_block_origin.as<int4>();
    m.gbox = P->d_gbox.as<int4>();
    m.nx = g.nx;
    m.ny = g.ny;
    m.nz = g.nz;
    m.faces = pl.rooftop ? 1 : 0;
  }
  if (!inner_only) {
    P->zvar[0] = cached_zvariant<double>(ctx, outer_batch<double>(*P, false), s, P->ztune_ms[0]);
    P->zvar[1] = cached_zvariant<float>(ctx, outer_batch<float>(*P, false), s, P->ztune_ms[1]);
    P->pvar[0] = cached_pvariant<double>(ctx, outer_batch<double>(*P, false), P->vec[V_B], P->vec[V_TMP1], s,
                                         P->ptune_ms[0]);
    P->pvar[1] = cached_pvariant<float>(ctx, outer_batch<float>(*P, false), P->vec[V_B], P->vec[V_TMP1], s,
                                        P->ptune_ms[1]);
  }
  hip_check(hipStreamSynchronize(s), "problem set-up");
  return P;
}

}  // namespace

// ------------------------------------------------------------------ serving
struct vie_request {
  enum State { QUEUED, RUNNING, DONE };
  ProblemPlan plan;
  std::vector<double> e_inc;
  vie_opts opts{};
  size_t footprint = 0;
  // result
  State state = QUEUED;
  vie_status status = VIE_OK;
  std::string error;
  std::vector<double> e_tot;
  vie_stats stats{};
  std::atomic<bool> cancel{false};
  std::chrono::steady_clock::time_point t_submit, t_start, t_solve, t_end;
  struct Server* server = nullptr;
};

// Worker threads (one HIP stream each) taking requests from a FIFO queue.
struct Server {
  vie_context* ctx = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<vie_request*> queue;
  std::set<vie_request*> running;
  std::vector<std::thread> workers;
  int queue_cap = 0;
  int64_t outstanding = 0;   // tickets not yet passed to vie_wait
  bool stop = false;

  // Front request fits the memory budget next to everything running.
  bool admissible() {
    if (queue.empty()) return false;
    if (ctx->budget == 0) return true;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return ctx->used + ctx->reserved + g_unfreed_bytes.load() + queue.front()->footprint <= ctx->budget;
  }

  void run(vie_request* r, hipStream_t s) {
    t_free_failed = false;
    vie_status st = guarded([&]() -> vie_status {
      set_device(ctx);
      auto P = build_problem(ctx, r->plan, s);
      P->footprint = r->footprint;
      P->cancel = &r->cancel;
      r->t_solve = std::chrono::steady_clock::now();
      const int64_t n = 3 * P->nv;
      DevBuf din(n * sizeof(c128)), dout(n * sizeof(c128));
      hip_check(hipMemcpyAsync(din.p, r->e_inc.data(), n * sizeof(c128), hipMemcpyHostToDevice, s), "upload e_inc");
      const vie_status code = solve_impl(P.get(), din.as<c128>(), &r->opts, dout.as<c128>(), nullptr, &r->stats, s);
      if (code != VIE_ECANCELLED) {
        r->e_tot.resize(2 * n);
        hip_check(hipMemcpyAsync(r->e_tot.data(), dout.p, n * sizeof(c128), hipMemcpyDeviceToHost, s), "download");
      }
      hip_check(hipStreamSynchronize(s), "request");
      return code;
    });
    r->status = st;
    if (st != VIE_OK) r->error = vie_last_error_str();
    if (t_free_failed && st >= 0) {
      // the request's problem is gone, but some of its device memory could
      // not be freed (it stays counted against the budget)
      r->status = VIE_EDEVICE;
      r->error = "device memory of the request could not be freed";
    }
  }

  void worker() {
    hipStream_t s = nullptr;
    (void)hipSetDevice(ctx->device);
    {
      ApiShared api;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    }
    for (;;) {
      vie_request* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || admissible(); });
        if (stop) break;
        r = queue.front();
        queue.pop_front();
        running.insert(r);
        r->state = vie_request::RUNNING;
        r->t_start = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lc(ctx->mu);
        ctx->reserved += r->footprint;
      }
      cv_work.notify_all();   // the next request may fit as well
      if (s)
        run(r, s);
      else {
        r->status = VIE_EDEVICE;
        r->error = "worker stream could not be created";
      }
      r->t_end = std::chrono::steady_clock::now();
      {
        std::lock_guard<std::mutex> lk(mu);
        {
          std::lock_guard<std::mutex> lc(ctx->mu);
          ctx->reserved -= std::min(ctx->reserved, r->footprint);
        }
        running.erase(r);
        r->state = vie_request::DONE;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (s) {
      ApiShared api;
      (void)hipStreamDestroy(s);
    }
  }

  void start(int slots, int cap) {
    queue_cap = cap;
    for (int i = 0; i < slots; ++i) workers.emplace_back([this] { worker(); });
  }

  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
      for (auto* r : queue) {
        r->status = VIE_ECANCELLED;
        r->error = "server stopped";
        r->state = vie_request::DONE;
      }
      queue.clear();
      for (auto* r : running) r->cancel.store(true);
    }
    cv_work.notify_all();
    for (auto& t : workers) t.join();
    cv_done.notify_all();
  }
};

vie_context::~vie_context() { server.reset(); }


// =================================================================== C ABI
extern "C" {

int32_t vie_abi_version(void) { return VIE_ABI_VERSION; }

const char* vie_last_error(void) { return g_last_error.c_str(); }

vie_status vie_context_create(int32_t device, size_t hbm_budget_bytes, vie_context** out) {
  return guarded([&]() -> vie_status {
    if (!out) fail(VIE_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) fail(VIE_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) fail(VIE_EDEVICE, "device index out of range");
    auto ctx = std::make_unique<vie_context>();
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    set_device(ctx.get());
    {
      ApiShared api;
      hip_check(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking), "stream");
    }
    // twiddle tables for every supported length, both precisions
    size_t total = 0;
    for (int L : vie::kFftLengths) total += L;
    std::vector<c128> h64(total);
    std::vector<c64> h32(total);
    size_t off = 0;
    for (int L : vie::kFftLengths) {
      for (int t = 0; t < L; ++t) {
        double c, sn;
        cis_neg(t, L, &c, &sn);
        h64[off + t] = mk<double>(c, sn);
        h32[off + t] = mk<float>((float)c, (float)sn);
      }
      off += L;
    }
    upload(ctx->tw64, h64, ctx->stream);
    upload(ctx->tw32, h32, ctx->stream);
    off = 0;
    for (int L : vie::kFftLengths) {
      ctx->tws64.table[L] = ctx->tw64.as<c128>() + off;
      ctx->tws32.table[L] = ctx->tw32.as<c64>() + off;
      off += L;
    }
    // the device address of the fixed scratch array, with this device current
    try {
      ctx->far_scratch = static_cast<double*>(vie::far_field_scratch_address());
    } catch (const std::exception& e) {
      fail(VIE_EDEVICE, e.what());
    }
    *out = ctx.release();
    return VIE_OK;
  });
}

vie_status vie_context_destroy(vie_context* ctx) {
  return guarded([&]() -> vie_status {
    if (!ctx) return VIE_OK;
    if (ctx->server) {
      {
        std::lock_guard<std::mutex> lk(ctx->server->mu);
        if (ctx->server->outstanding > 0) fail(VIE_EBUSY, "tickets are outstanding (pass each to vie_wait first)");
      }
      ctx->server.reset();
    }
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) {
      ApiShared api;
      (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
    return VIE_OK;
  });
}

// overlap < 0: the rooftop discretisation (no blocks)
static vie_status problem_create(vie_context* ctx, const vie_grid* grid, const double* eps_r,
                                 const int32_t* block_id, int32_t n_blocks, int32_t overlap, vie_problem** out) {
  return guarded([&]() -> vie_status {
    if (!out) fail(VIE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !grid || !eps_r) fail(VIE_EINVAL, "ctx, grid and eps_r are required");
    if (overlap < -1 || overlap > 256) fail(VIE_EINVAL, "overlap must be in [0, 256]");
    ProblemPlan plan = overlap < 0 ? make_plan_rooftop(*grid, eps_r, block_id, n_blocks)
                                   : make_plan(*grid, eps_r, block_id, n_blocks, block_id ? overlap : 0);
    set_device(ctx);
    const size_t foot = plan_footprint(ctx, plan);
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (ctx->budget && ctx->used + ctx->reserved + g_unfreed_bytes.load() + foot > ctx->budget)
        fail(VIE_EBUSY, "problem exceeds the context's HBM budget");
      ctx->used += foot;
    }
    try {
      auto P = build_problem(ctx, plan, ctx->stream);
      P->footprint = foot;
      P->plan = std::make_shared<const ProblemPlan>(std::move(plan));
      *out = P.release();
    } catch (...) {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->used -= std::min(ctx->used, foot);
      throw;
    }
    return VIE_OK;
  });
}

vie_status vie_problem_create(vie_context* ctx, const vie_grid* grid, const double* eps_r, const int32_t* block_id,
                              int32_t n_blocks, vie_problem** out) {
  return problem_create(ctx, grid, eps_r, block_id, n_blocks, 0, out);
}

vie_status vie_problem_create_overlap(vie_context* ctx, const vie_grid* grid, const double* eps_r,
                                      const int32_t* block_id, int32_t n_blocks, int32_t overlap, vie_problem** out) {
  if (overlap < 0) {
    if (out) *out = nullptr;
    return guarded([]() -> vie_status { fail(VIE_EINVAL, "overlap must be in [0, 256]"); });
  }
  return problem_create(ctx, grid, eps_r, block_id, n_blocks, overlap, out);
}

vie_status vie_problem_create_rooftop(vie_context* ctx, const vie_grid* grid, const double* eps_r,
                                      const int32_t* block_id, int32_t n_blocks, vie_problem** out) {
  return problem_create(ctx, grid, eps_r, block_id, n_blocks, -1, out);
}

vie_status vie_problem_destroy(vie_problem* p) {
  return guarded([&]() -> vie_status {
    if (!p) return VIE_OK;
    (void)hipSetDevice(p->ctx->device);
    {
      ApiShared api;
      (void)hipDeviceSynchronize();
    }
    vie_context* ctx = p->ctx;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->used -= std::min(ctx->used, p->footprint);
    }
    delete p;
    {
      // queued requests may fit now
      std::lock_guard<std::mutex> lk(ctx->server_mu);
      if (ctx->server) ctx->server->cv_work.notify_all();
    }
    return VIE_OK;
  });
}

vie_status vie_problem_set_zpass(vie_problem* p, int32_t precision, int32_t variant) {
  return guarded([&]() -> vie_status {
    if (!p) fail(VIE_EINVAL, "problem is NULL");
    if (precision != VIE_FP64 && precision != VIE_MIXED) fail(VIE_EINVAL, "unknown precision");
    if (variant < -1 || variant >= vie::kZPassVariants) fail(VIE_EINVAL, "z-pass variant out of range");
    if (variant == 1 && p->rooftop) fail(VIE_EINVAL, "rooftop problems have no mirror-column z pass (variant 1)");
    set_device(p->ctx);
    {
      ApiShared api;
      hip_check(hipDeviceSynchronize(), "synchronise");
    }
    std::lock_guard<std::mutex> lk(p->mu);
    const int q = precision == VIE_MIXED ? 1 : 0;
    hipStream_t s = p->ctx->stream;
    // the problem, and the replica of its blocks used by preconditioned batches
    for (vie_problem* x : {p, p->replica.get()}) {
      if (!x) continue;
      const bool outer = x->spec != nullptr;
      if (variant >= 0) {
        x->zvar[q] = variant;
        for (auto& G : x->groups) G.zvar[q] = variant;
      } else if (q == 0) {
        if (outer) x->zvar[0] = cached_zvariant<double>(x->ctx, outer_batch<double>(*x, false), s, nullptr);
        for (auto& G : x->groups)
          G.zvar[0] = cached_zvariant<double>(x->ctx, group_batch<double>(*x, G, false), s, nullptr);
      } else {
        if (outer) x->zvar[1] = cached_zvariant<float>(x->ctx, outer_batch<float>(*x, false), s, nullptr);
        for (auto& G : x->groups)
          G.zvar[1] = cached_zvariant<float>(x->ctx, group_batch<float>(*x, G, false), s, nullptr);
      }
      // captured inner steps hold the old kernels
      ApiShared api;
      for (auto& G : x->groups)
        if (G.graph[q]) {
          (void)hipGraphExecDestroy(G.graph[q]);
          G.graph[q] = nullptr;
        }
    }
    return VIE_OK;
  });
}

vie_status vie_problem_set_plane(vie_problem* p, int32_t precision, int32_t variant) {
  return guarded([&]() -> vie_status {
    if (!p) fail(VIE_EINVAL, "problem is NULL");
    if (precision != VIE_FP64 && precision != VIE_MIXED) fail(VIE_EINVAL, "unknown precision");
    if (variant < -1 || variant >= vie::kPlaneVariants) fail(VIE_EINVAL, "plane-kernel variant out of range");
    set_device(p->ctx);
    {
      ApiShared api;
      hip_check(hipDeviceSynchronize(), "synchronise");
    }
    std::lock_guard<std::mutex> lk(p->mu);
    const int q = precision == VIE_MIXED ? 1 : 0;
    for (vie_problem* x : {p, p->replica.get()}) {
      if (!x) continue;
      if (variant >= 0) {
        x->pvar[q] = variant;
        for (auto& G : x->groups) G.pvar[q] = variant;
      } else {
        // the choices cached at set-up (tuned once per shape)
        std::lock_guard<std::mutex> ck(x->ctx->mu);
        auto tuned = [&](int sz, int nx, int ny, int nz, int lx, int ly, int lz, int nsys) {
          auto it = x->ctx->ptune.find({sz, nx, ny, nz, lx, ly, lz, nsys});
          return it == x->ctx->ptune.end() ? 0 : it->second.first;
        };
        const int sz = q == 1 ? (int)sizeof(float) : (int)sizeof(double);
        if (x->spec) x->pvar[q] = tuned(sz, x->g.nx, x->g.ny, x->g.nz, x->lx, x->ly, x->lz, 1);
        for (auto& G : x->groups) G.pvar[q] = tuned(sz, G.bx, G.by, G.bz, G.lx, G.ly, G.lz, G.nsys);
      }
      // captured inner steps hold the old kernels
      ApiShared api;
      for (auto& G : x->groups)
        if (G.graph[q]) {
          (void)hipGraphExecDestroy(G.graph[q]);
          G.graph[q] = nullptr;
        }
    }
    return VIE_OK;
  });
}

vie_status vie_problem_get_info(const vie_problem* p, vie_problem_info* info) {
  return guarded([&]() -> vie_status {
    if (!p || !info) fail(VIE_EINVAL, "problem and info are required");
    info->lx = p->lx;
    info->ly = p->ly;
    info->lz = p->lz;
    info->n_blocks = p->n_nonempty;
    info->n_groups = (int32_t)p->groups.size();
    info->footprint_bytes = (int64_t)p->footprint;
    info->n_block_solver_groups = p->n_wg_groups;
    static_assert(vie::kZPassVariants == 5, "vie_problem_info holds 5 z-pass timings");
    static_assert(vie::kPlaneVariants == 3, "vie_problem_info holds 3 plane-kernel timings");
    for (int q = 0; q < 2; ++q) {
      info->zpass_variant[q] = p->zvar[q];
      for (int v = 0; v < vie::kZPassVariants; ++v) info->zpass_tune_ms[q][v] = p->ztune_ms[q][v];
      info->plane_variant[q] = p->pvar[q];
      for (int v = 0; v < vie::kPlaneVariants; ++v) info->plane_tune_ms[q][v] = p->ptune_ms[q][v];
    }
    return VIE_OK;
  });
}

vie_status vie_plan(const vie_grid* grid, const double* eps_r, const int32_t* block_id, int32_t n_blocks,
                    int32_t overlap, vie_problem_info* info, vie_group_plan* groups, int32_t groups_cap,
                    int32_t* block_group) {
  return guarded([&]() -> vie_status {
    if (!grid || !eps_r || !info) fail(VIE_EINVAL, "grid, eps_r and info are required");
    if (overlap < 0 || overlap > 256) fail(VIE_EINVAL, "overlap must be in [0, 256]");
    if (groups_cap < 0 || (groups_cap > 0 && !groups)) fail(VIE_EINVAL, "groups_cap needs a groups array");
    const ProblemPlan pl = make_plan(*grid, eps_r, block_id, n_blocks, block_id ? overlap : 0);
    vie_problem_info d{};
    d.lx = pl.lx;
    d.ly = pl.ly;
    d.lz = pl.lz;
    for (int64_t c : pl.cnt) d.n_blocks += c > 0 ? 1 : 0;
    d.n_groups = (int32_t)pl.groups.size();
    for (const auto& gp : pl.groups) d.n_block_solver_groups += gp.wg ? 1 : 0;
    d.footprint_bytes = (int64_t)plan_footprint(nullptr, pl, true);
    d.zpass_variant[0] = d.zpass_variant[1] = -1;
    for (auto& row : d.zpass_tune_ms)
      for (auto& v : row) v = -1.0f;
    d.plane_variant[0] = d.plane_variant[1] = -1;
    for (auto& row : d.plane_tune_ms)
      for (auto& v : row) v = -1.0f;
    for (int32_t i = 0; i < groups_cap && i < (int32_t)pl.groups.size(); ++i) {
      const GroupPlan& gp = pl.groups[i];
      groups[i] = vie_group_plan{gp.lx, gp.ly, gp.lz, gp.bx, gp.by, gp.bz, (int32_t)gp.blocks.size(), gp.wg ? 1 : 0};
    }
    if (block_group && block_id) {
      for (int32_t k = 0; k < n_blocks; ++k) block_group[k] = -1;
      for (size_t gi = 0; gi < pl.groups.size(); ++gi)
        for (int k : pl.groups[gi].blocks) block_group[k] = (int32_t)gi;
    }
    *info = d;
    return VIE_OK;
  });
}

// faces: component c sampled half a cell further along axis c (the face
// centres of the rooftop unknowns)
static vie_status plane_wave(const vie_grid* grid, const double kdir[3], const double pol[6], double* e_inc,
                             bool faces) {
  return guarded([&]() -> vie_status {
    if (!grid || !kdir || !pol || !e_inc) fail(VIE_EINVAL, "all arguments are required");
    const vie_grid g = *grid;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) fail(VIE_EINVAL, "grid sizes must be >= 1");
    if (!(g.wavelength > 0) || !is_finite(g.wavelength) || !is_finite(g.dx) || !is_finite(g.dy) || !is_finite(g.dz))
      fail(VIE_EINVAL, "bad spacing or wavelength");
    const double kn = std::sqrt(kdir[0] * kdir[0] + kdir[1] * kdir[1] + kdir[2] * kdir[2]);
    if (!(std::fabs(kn - 1.0) <= 1e-12)) fail(VIE_EINVAL, "kdir must be a unit vector");
    for (int i = 0; i < 6; ++i)
      if (!is_finite(pol[i])) fail(VIE_EINVAL, "pol has non-finite entries");
    const double k0 = 2.0 * M_PI / g.wavelength;
    const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
    for (int z = 0; z < g.nz; ++z)
      for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; ++x) {
          const double rx = (x - 0.5 * (g.nx - 1)) * g.dx, ry = (y - 0.5 * (g.ny - 1)) * g.dy,
                       rz = (z - 0.5 * (g.nz - 1)) * g.dz;
          const int64_t v = ((int64_t)z * g.ny + y) * g.nx + x;
          for (int c = 0; c < 3; ++c) {
            const double sx = faces && c == 0 ? 0.5 * g.dx : 0.0, sy = faces && c == 1 ? 0.5 * g.dy : 0.0,
                         sz = faces && c == 2 ? 0.5 * g.dz : 0.0;
            const double ph = -k0 * (kdir[0] * (rx + sx) + kdir[1] * (ry + sy) + kdir[2] * (rz + sz));
            const std::complex<double> val = std::complex<double>(pol[2 * c], pol[2 * c + 1]) * std::polar(1.0, ph);
            e_inc[2 * (c * nv + v)] = val.real();
            e_inc[2 * (c * nv + v) + 1] = val.imag();
          }
        }
    return VIE_OK;
  });
}

vie_status vie_plane_wave(const vie_grid* grid, const double kdir[3], const double pol[6], double* e_inc) {
  return plane_wave(grid, kdir, pol, e_inc, false);
}

vie_status vie_plane_wave_faces(const vie_grid* grid, const double kdir[3], const double pol[6], double* e_inc) {
  return plane_wave(grid, kdir, pol, e_inc, true);
}

vie_status vie_matvec(vie_problem* p, int32_t precision, const void* x_dev, void* y_dev, void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !x_dev || !y_dev) fail(VIE_EINVAL, "problem, x and y are required");
    if (x_dev == y_dev) fail(VIE_EINVAL, "x and y must not overlap");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = (hipStream_t)stream;
    if (precision == VIE_FP64)
      vie::mvm<double>(outer_batch<double>(*p, false), (const c128*)x_dev, (c128*)y_dev, true, s);
    else if (precision == VIE_MIXED)
      vie::mvm<float>(outer_batch<float>(*p, false), (const c128*)x_dev, (c128*)y_dev, true, s);
    else
      fail(VIE_EINVAL, "unknown precision");
    return VIE_OK;
  });
}

extern "C++" {
template <typename R>
static void total_field_box(vie_problem* p, const c128* pol, const c128* e_inc, c128* e_box, hipStream_t s) {
  const MvmBatch<R> m = outer_batch<R>(*p, false);
  const vie::FuseArgs none{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
  const vie::FuseArgs field{0, 3, nullptr, nullptr, nullptr, e_inc, nullptr};
  vie::mvm_pass1<R>(m, nullptr, none, pol, true, s);
  vie::mvm_mid<R>(m, s);
  vie::mvm_pass5<R>(m, nullptr, field, pol, e_box, s);
  if (p->rooftop) vie::zero_outer_faces(e_box, p->g.nx, p->g.ny, p->g.nz, s);
}
}  // extern "C++"

vie_status vie_total_field_box(vie_problem* p, int32_t precision, const void* pol_dev, const void* e_inc_dev,
                               void* e_box_dev, void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !pol_dev || !e_inc_dev || !e_box_dev) fail(VIE_EINVAL, "problem, pol, e_inc and e_box are required");
    if (e_box_dev == pol_dev || e_box_dev == e_inc_dev) fail(VIE_EINVAL, "e_box must not overlap the inputs");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = (hipStream_t)stream;
    if (precision == VIE_FP64)
      total_field_box<double>(p, (const c128*)pol_dev, (const c128*)e_inc_dev, (c128*)e_box_dev, s);
    else if (precision == VIE_MIXED)
      total_field_box<float>(p, (const c128*)pol_dev, (const c128*)e_inc_dev, (c128*)e_box_dev, s);
    else
      fail(VIE_EINVAL, "unknown precision");
    return VIE_OK;
  });
}

extern "C++" {
static void far_field_host(vie_problem* p, const void* pol_dev, int32_t n_dir, const double* rhat,
                           std::vector<c128>& F, hipStream_t s) {
  if (!p || !pol_dev || !rhat) fail(VIE_EINVAL, "problem, pol and rhat are required");
  if (n_dir < 1 || n_dir > 1000000) fail(VIE_EINVAL, "n_dir out of range");
  for (int32_t d = 0; d < n_dir; ++d) {
    const double* r = rhat + 3 * d;
    if (!is_finite(r[0]) || !is_finite(r[1]) || !is_finite(r[2])) fail(VIE_EINVAL, "rhat has non-finite entries");
    const double nrm = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(std::fabs(nrm - 1.0) <= 1e-12)) fail(VIE_EINVAL, "rhat entries must be unit vectors");
  }
  set_device(p->ctx);
  const vie_grid& g = p->g;
  const int64_t nchunk = vie::far_field_chunks(p->nv);
  DevBuf dr(3 * (size_t)n_dir * sizeof(double)), part(6 * (size_t)n_dir * nchunk * sizeof(double)),
      dF(3 * (size_t)n_dir * sizeof(c128));
  hip_check(hipMemcpyAsync(dr.p, rhat, dr.bytes, hipMemcpyHostToDevice, s), "upload rhat");
  vie::far_field((const c128*)pol_dev, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, p->k0, dr.as<double>(), n_dir,
                 part.as<double>(), dF.as<c128>(), s, p->rooftop);
  F.resize(3 * (size_t)n_dir);
  hip_check(hipMemcpyAsync(F.data(), dF.p, dF.bytes, hipMemcpyDeviceToHost, s), "download F");
  hip_check(hipStreamSynchronize(s), "far field");
}
}  // extern "C++"

vie_status vie_far_field(vie_problem* p, const void* pol_dev, int32_t n_dir, const double* rhat, double* f_out,
                         void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !f_out) fail(VIE_EINVAL, "problem and f_out are required");
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<c128> F;
    far_field_host(p, pol_dev, n_dir, rhat, F, (hipStream_t)stream);
    std::memcpy(f_out, F.data(), F.size() * sizeof(c128));
    return VIE_OK;
  });
}

vie_status vie_far_field_noalloc(vie_problem* p, const void* pol_dev, int32_t n_dir, const void* rhat_dev,
                                 void* f_dev, void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !pol_dev || !rhat_dev || !f_dev) fail(VIE_EINVAL, "problem, pol, rhat and f are required");
    if (n_dir < 1) fail(VIE_EINVAL, "n_dir must be >= 1");
    const int64_t nchunk = vie::far_field_chunks(p->nv);
    if ((int64_t)n_dir * nchunk * 6 > vie::far_field_scratch_doubles())
      fail(VIE_EINVAL, "n_dir * ceil(nx ny nz / 2048) * 6 exceeds the fixed scratch of 1048576 doubles (use "
                       "vie_far_field, or fewer directions per call)");
    if (!p->ctx->far_scratch) fail(VIE_EDEVICE, "far-field scratch not set up");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    const vie_grid& g = p->g;
    vie::far_field((const c128*)pol_dev, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, p->k0, (const double*)rhat_dev, n_dir,
                   p->ctx->far_scratch, (c128*)f_dev, (hipStream_t)stream, p->rooftop);
    return VIE_OK;
  });
}

vie_status vie_rcs(vie_problem* p, const void* pol_dev, int32_t n_dir, const double* rhat, double* sigma_out,
                   void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !sigma_out) fail(VIE_EINVAL, "problem and sigma_out are required");
    std::lock_guard<std::mutex> lk(p->mu);
    std::vector<c128> F;
    far_field_host(p, pol_dev, n_dir, rhat, F, (hipStream_t)stream);
    const double k4 = std::pow(p->k0, 4) / (4.0 * M_PI);
    for (int32_t d = 0; d < n_dir; ++d) {
      double a = 0;
      for (int q = 0; q < 3; ++q) a += F[3 * d + q].x * F[3 * d + q].x + F[3 * d + q].y * F[3 * d + q].y;
      sigma_out[d] = k4 * a;
    }
    return VIE_OK;
  });
}

vie_status vie_matvec_profile(vie_problem* p, int32_t precision, const void* x_dev, void* y_dev, void* stream,
                              int32_t reps, double* pass_ms) {
  return guarded([&]() -> vie_status {
    if (!p || !x_dev || !y_dev || !pass_ms) fail(VIE_EINVAL, "problem, x, y and pass_ms are required");
    if (x_dev == y_dev) fail(VIE_EINVAL, "x and y must not overlap");
    if (reps < 1 || reps > 100000) fail(VIE_EINVAL, "reps out of range");
    if (precision != VIE_FP64 && precision != VIE_MIXED) fail(VIE_EINVAL, "unknown precision");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[6];
    {
      ApiShared api;
      for (auto& e : ev) hip_check(hipEventCreate(&e), "event");
    }
    auto destroy = [&] {
      ApiShared api;
      for (auto& e : ev) (void)hipEventDestroy(e);
    };
    double acc[5] = {0, 0, 0, 0, 0};
    try {
      for (int r = 0; r < reps; ++r) {
        if (precision == VIE_FP64)
          vie::mvm<double>(outer_batch<double>(*p, false), (const c128*)x_dev, (c128*)y_dev, false, s, ev);
        else
          vie::mvm<float>(outer_batch<float>(*p, false), (const c128*)x_dev, (c128*)y_dev, false, s, ev);
        hip_check(hipEventSynchronize(ev[5]), "profile");
        for (int i = 0; i < 5; ++i) {
          float ms = 0;
          hip_check(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "elapsed");
          acc[i] += ms;
        }
      }
    } catch (...) {
      destroy();
      throw;
    }
    destroy();
    for (int i = 0; i < 5; ++i) pass_ms[i] = acc[i] / reps;
    return VIE_OK;
  });
}

vie_status vie_group_profile(vie_problem* p, int32_t precision, int32_t group, int32_t n_active, int32_t reps,
                             void* stream, double* pass_ms) {
  return guarded([&]() -> vie_status {
    if (!p || !pass_ms) fail(VIE_EINVAL, "problem and pass_ms are required");
    if (group < 0 || group >= (int32_t)p->groups.size()) fail(VIE_EINVAL, "group out of range");
    if (precision != VIE_FP64 && precision != VIE_MIXED) fail(VIE_EINVAL, "unknown precision");
    if (reps < 1 || reps > 100000) fail(VIE_EINVAL, "reps out of range");
    Group& G = p->groups[group];
    if (n_active < 0 || n_active > G.nsys) fail(VIE_EINVAL, "n_active out of range");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = (hipStream_t)stream;
    std::vector<int> st(G.nsys, vie::ST_CONVERGED);
    for (int q = 0; q < n_active; ++q) st[q] = vie::ST_ACTIVE;
    hip_check(hipMemcpyAsync(p->d_istatus.as<int>() + G.slot0, st.data(), st.size() * sizeof(int),
                             hipMemcpyHostToDevice, s),
              "profile status");
    hip_check(hipStreamSynchronize(s), "profile status");
    hipEvent_t ev[6];
    {
      ApiShared api;
      for (auto& e : ev) hip_check(hipEventCreate(&e), "event");
    }
    auto destroy = [&] {
      ApiShared api;
      for (auto& e : ev) (void)hipEventDestroy(e);
    };
    double acc[5] = {0, 0, 0, 0, 0};
    try {
      for (int r = 0; r < reps; ++r) {
        if (precision == VIE_FP64)
          vie::mvm<double>(group_batch<double>(*p, G, true), G.vec[V_P], G.vec[V_V], false, s, ev);
        else
          vie::mvm<float>(group_batch<float>(*p, G, true), G.vec[V_P], G.vec[V_V], false, s, ev);
        hip_check(hipEventSynchronize(ev[5]), "profile");
        for (int i = 0; i < 5; ++i) {
          float ms = 0;
          hip_check(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "elapsed");
          acc[i] += ms;
        }
      }
    } catch (...) {
      destroy();
      throw;
    }
    destroy();
    for (int i = 0; i < 5; ++i) pass_ms[i] = acc[i] / reps;
    return VIE_OK;
  });
}

vie_status vie_block_matvec(vie_problem* p, int32_t precision, const void* x_dev, void* y_dev, void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !x_dev || !y_dev) fail(VIE_EINVAL, "problem, x and y are required");
    if (x_dev == y_dev) fail(VIE_EINVAL, "x and y must not overlap");
    if (p->groups.empty()) fail(VIE_EINVAL, "problem has no blocks");
    if (precision != VIE_FP64 && precision != VIE_MIXED) fail(VIE_EINVAL, "unknown precision");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = (hipStream_t)stream;
    vie::block_gather(p->bmap, (const c128*)x_dev, gptr(*p, V_B), s);
    for (auto& G : p->groups) {
      if (precision == VIE_FP64)
        vie::mvm<double>(group_batch<double>(*p, G, false), G.vec[V_B], G.vec[V_V], false, s);
      else
        vie::mvm<float>(group_batch<float>(*p, G, false), G.vec[V_B], G.vec[V_V], false, s);
    }
    vie::block_scatter(p->bmap, gptr(*p, V_V), (c128*)y_dev, s);
    return VIE_OK;
  });
}

vie_status vie_precond_apply(vie_problem* p, int32_t precision, double tol_inner, int32_t maxit_inner,
                             int32_t flags, const void* w_dev, void* y_dev, void* stream, int64_t* inner_iters) {
  return guarded([&]() -> vie_status {
    if (!p || !w_dev || !y_dev) fail(VIE_EINVAL, "problem, w and y are required");
    if (w_dev == y_dev) fail(VIE_EINVAL, "w and y must not overlap");
    if (p->groups.empty()) fail(VIE_EINVAL, "problem has no blocks");
    if (!(tol_inner >= 0) || !is_finite(tol_inner)) fail(VIE_EINVAL, "tol_inner must be finite and >= 0");
    if (maxit_inner < 1) fail(VIE_EINVAL, "maxit_inner must be >= 1");
    if (flags & ~(VIE_FLAG_NO_GRAPHS | VIE_FLAG_NO_BLOCK_KERNEL)) fail(VIE_EINVAL, "unknown flags");
    const bool graphs = (flags & VIE_FLAG_NO_GRAPHS) == 0, wg = (flags & VIE_FLAG_NO_BLOCK_KERNEL) == 0;
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = (hipStream_t)stream;
    hip_check(hipMemsetAsync(p->d_acc.p, 0, 3 * sizeof(int64_t), s), "acc");
    if (precision == VIE_FP64)
      precond_apply<double>(*p, (const c128*)w_dev, (c128*)y_dev, tol_inner, maxit_inner, nullptr, 1, nullptr, 0, graphs,
                            wg, s);
    else if (precision == VIE_MIXED)
      precond_apply<float>(*p, (const c128*)w_dev, (c128*)y_dev, tol_inner, maxit_inner, nullptr, 1, nullptr, 0, graphs,
                           wg, s);
    else
      fail(VIE_EINVAL, "unknown precision");
    if (inner_iters) {
      int64_t acc[3];
      hip_check(hipMemcpyAsync(acc, p->d_acc.p, sizeof(acc), hipMemcpyDeviceToHost, s), "acc");
      hip_check(hipStreamSynchronize(s), "precond");
      *inner_iters = acc[0];
    }
    return VIE_OK;
  });
}

vie_status vie_solve_device(vie_problem* p, const void* e_inc_dev, const vie_opts* opts, void* e_tot_dev,
                            void* pol_dev, vie_stats* stats, void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !e_inc_dev || !e_tot_dev) fail(VIE_EINVAL, "problem, e_inc and e_tot are required");
    validate_opts(opts, !p->groups.empty());
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    return solve_impl(p, (const c128*)e_inc_dev, opts, (c128*)e_tot_dev, (c128*)pol_dev, stats, (hipStream_t)stream);
  });
}

vie_status vie_solve_batch(vie_problem* p, int32_t nrhs, const void* e_inc_dev, const vie_opts* opts,
                           void* e_tot_dev, void* pol_dev, vie_stats* stats, void* stream) {
  return guarded([&]() -> vie_status {
    if (!p || !e_inc_dev || !e_tot_dev) fail(VIE_EINVAL, "problem, e_inc and e_tot are required");
    if (nrhs < 1 || nrhs > 4096) fail(VIE_EINVAL, "nrhs must be in [1, 4096]");
    validate_opts(opts, !p->groups.empty());
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    vie_problem& P = *p;
    const int64_t n = 3 * P.nv;
    const c128* ein = (const c128*)e_inc_dev;
    c128* eout = (c128*)e_tot_dev;
    c128* pol = (c128*)pol_dev;
    // the first error, else a warning, else OK
    vie_status worst = VIE_OK;
    auto keep = [&](vie_status st) {
      if (worst >= 0 && (st < 0 || st > worst)) worst = st;
    };
    const bool batched = nrhs > 1 && opts->solver == VIE_SOLVER_BICGSTAB;
    const bool prec = opts->precondition != 0;
    const bool graphs = (opts->flags & VIE_FLAG_NO_GRAPHS) == 0;
    const bool wgk = (opts->flags & VIE_FLAG_NO_BLOCK_KERNEL) == 0;
    if (!batched) {
      for (int r = 0; r < nrhs; ++r)
        keep(solve_impl(p, ein + r * n, opts, eout + r * n, pol ? pol + r * n : nullptr, stats ? &stats[r] : nullptr,
                        s));
      return worst;
    }
    ensure_batch(P, nrhs);
    if (prec) {
      ensure_replica(P, nrhs, s);
      hip_check(hipMemsetAsync(P.replica->d_acc.p, 0, 3 * sizeof(int64_t), s), "acc");
    }
    for (int r = 0; r < nrhs; ++r)
      vie::masked_copy(ein + r * n, P.chi.as<c128>(), batch_vec(P, BV_B, nrhs) + r * n, P.nv, s, chi_period(P));
    const double ti = opts->tol_inner;
    const int mi = opts->maxit_inner, lag = opts->poll_lag;
    if (opts->precision == VIE_MIXED)
      run_bicgstab_batch<float, float>(P, nrhs, opts->tol_outer, opts->maxit_outer, lag, prec, ti, mi, graphs, wgk, s);
    else if (opts->precision == VIE_MIXED_INNER)
      run_bicgstab_batch<double, float>(P, nrhs, opts->tol_outer, opts->maxit_outer, lag, prec, ti, mi, graphs, wgk,
                                        s);
    else
      run_bicgstab_batch<double, double>(P, nrhs, opts->tol_outer, opts->maxit_outer, lag, prec, ti, mi, graphs,
                                         wgk, s);
    int64_t acc[3] = {0, 0, 0};
    if (prec) copy_out(acc, P.replica->d_acc.p, sizeof(acc), s, "acc");
    std::vector<KState> st(nrhs);
    std::vector<int> status(nrhs);
    copy_out(st.data(), P.mr_state.p, nrhs * sizeof(KState), s, "batch state");
    copy_out(status.data(), P.mr_status.p, nrhs * sizeof(int), s, "batch status");
    const double batch_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // per system: true residual, refinement (mixed), fields, statistics
    for (int r = 0; r < nrhs; ++r) {
      hip_check(hipMemcpyAsync(P.vec[V_B], batch_vec(P, BV_B, nrhs) + r * n, n * sizeof(c128),
                               hipMemcpyDeviceToDevice, s),
                "batch rhs");
      hip_check(hipMemcpyAsync(P.vec[V_X], batch_vec(P, BV_X, nrhs) + r * n, n * sizeof(c128),
                               hipMemcpyDeviceToDevice, s),
                "batch iterate");
      const RunResult rr{st[r], status[r]};
      keep(solve_impl(p, nullptr, opts, eout + r * n, pol ? pol + r * n : nullptr, stats ? &stats[r] : nullptr, s,
                      &rr));
      if (stats) {
        stats[r].seconds += batch_s;
        stats[r].inner_iters_total += acc[0];   // the batch's totals (all right-hand sides)
        stats[r].precond_applies += acc[1];
      }
    }
    return worst;
  });
}

vie_status vie_solve_many(int32_t n, vie_problem* const* problems, const void* const* e_inc_dev,
                          const vie_opts* opts, void* const* e_tot_dev, void* const* pol_dev, vie_stats* stats,
                          void* stream) {
  return guarded([&]() -> vie_status {
    if (n < 1 || n > 4096) fail(VIE_EINVAL, "n must be in [1, 4096]");
    if (!problems || !e_inc_dev || !e_tot_dev) fail(VIE_EINVAL, "problems, e_inc_dev and e_tot_dev are required");
    std::vector<vie_problem*> ps(problems, problems + n);
    for (int r = 0; r < n; ++r)
      if (!ps[r] || !e_inc_dev[r] || !e_tot_dev[r]) fail(VIE_EINVAL, "a problem, e_inc or e_tot entry is NULL");
    if (std::set<vie_problem*>(ps.begin(), ps.end()).size() != ps.size()) fail(VIE_EINVAL, "a problem appears twice");
    vie_problem& P0 = *ps[0];
    const bool prec = opts && opts->precondition != 0;
    for (vie_problem* q : ps) {
      if (q->rooftop != P0.rooftop) fail(VIE_EINVAL, "vie_solve_many: rooftop and collocated problems mixed");
      if (q->ctx != P0.ctx) fail(VIE_EINVAL, "problems belong to different contexts");
      if (q->g.nx != P0.g.nx || q->g.ny != P0.g.ny || q->g.nz != P0.g.nz || q->lx != P0.lx || q->ly != P0.ly ||
          q->lz != P0.lz)
        fail(VIE_EINVAL, "problems differ in grid shape or FFT lengths");
      validate_opts(opts, !q->groups.empty());
      if (prec && (!q->plan || q->plan->overlap != P0.plan->overlap))
        fail(VIE_EINVAL, "preconditioned problems need their plans and one overlap");
    }
    // every problem's lock, in address order
    std::vector<vie_problem*> order = ps;
    std::sort(order.begin(), order.end());
    std::vector<std::unique_lock<std::mutex>> locks;
    for (vie_problem* q : order) locks.emplace_back(q->mu);
    set_device(P0.ctx);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    vie_status worst = VIE_OK;
    auto keep = [&](vie_status st) {
      if (worst >= 0 && (st < 0 || st > worst)) worst = st;
    };
    const int64_t nv = P0.nv, n3 = 3 * nv;
    auto ein = [&](int r) { return (const c128*)e_inc_dev[r]; };
    auto eout = [&](int r) { return (c128*)e_tot_dev[r]; };
    auto pol = [&](int r) { return pol_dev ? (c128*)pol_dev[r] : nullptr; };
    if (n == 1 || opts->solver != VIE_SOLVER_BICGSTAB) {
      for (int r = 0; r < n; ++r) keep(solve_impl(ps[r], ein(r), opts, eout(r), pol(r), stats ? &stats[r] : nullptr, s));
      return worst;
    }
    const bool graphs = (opts->flags & VIE_FLAG_NO_GRAPHS) == 0;
    Fleet F(P0.ctx);
    ProblemPlan fp;
    if (prec) fp = fleet_plan(ps);
    const size_t small = (size_t)n * (sizeof(KState) + 2 * sizeof(int) + 2 * (size_t)P0.pstride * sizeof(double)) +
                         2 * (size_t)n * sizeof(void*) + sizeof(int);
    const int64_t cper = chi_period(P0);   // 1/chi entries per problem
    const size_t bytes = (size_t)n * cper * sizeof(c128) + (size_t)n * 3 * P0.g.nz * P0.ly * P0.lx * sizeof(c128) +
                         (size_t)kBatchVecs * n * n3 * sizeof(c128) + small + (prec ? replica_bytes(fp) : 0);
    {
      std::lock_guard<std::mutex> lk(P0.ctx->mu);
      if (P0.ctx->budget && P0.ctx->used + P0.ctx->reserved + g_unfreed_bytes.load() + bytes > P0.ctx->budget)
        fail(VIE_EBUSY, "the batch exceeds the context's HBM budget");
      P0.ctx->used += bytes;
      F.bytes = bytes;
    }
    F.chi.alloc((size_t)n * cper * sizeof(c128));
    F.work.alloc((size_t)n * 3 * P0.g.nz * P0.ly * P0.lx * sizeof(c128));
    F.vecs.alloc((size_t)kBatchVecs * n * n3 * sizeof(c128));
    F.vecs.zero(s);
    F.state.alloc((size_t)n * sizeof(KState));
    F.status.alloc((size_t)n * sizeof(int));
    F.partials.alloc((size_t)n * P0.pstride * sizeof(double));
    F.partials2.alloc((size_t)n * P0.pstride * sizeof(double));
    F.ntile.alloc((size_t)n * sizeof(int));
    F.count.alloc(sizeof(int));
    std::vector<const void*> tab(2 * (size_t)n);
    for (int r = 0; r < n; ++r) {
      hip_check(hipMemcpyAsync(F.chi.as<c128>() + r * cper, ps[r]->chi.p, cper * sizeof(c128),
                               hipMemcpyDeviceToDevice, s),
                "batch 1/chi");
      tab[r] = spec_ptr<double>(*ps[r]->spec);
      tab[n + r] = spec_ptr<float>(*ps[r]->spec);
    }
    upload(F.tab, tab, s);
    if (prec) {
      F.replica = build_problem(P0.ctx, fp, s, true);
      hip_check(hipMemsetAsync(F.replica->d_acc.p, 0, 3 * sizeof(int64_t), s), "acc");
    }
    KBatch k{};
    k.nsys = n;
    k.n = n3;
    k.status = F.status.as<int>();
    k.st = F.state.as<KState>();
    k.partials = F.partials.as<double>();
    k.pstride = P0.pstride;
    k.ntile = F.ntile.as<int>();
    k.partials2 = F.partials2.as<double>();
    const BatchSet B{P0, F.replica.get(), n, nv, F.vecs.as<c128>(), k, F.status.as<int>(), F.count.as<int>()};
    for (int r = 0; r < n; ++r)
      vie::masked_copy(ein(r), ps[r]->chi.as<c128>(), B.vec(BV_B) + r * n3, nv, s, chi_period(*ps[r]));
    const double ti = opts->tol_inner, to = opts->tol_outer;
    const int mi = opts->maxit_inner, mo = opts->maxit_outer, lag = opts->poll_lag;
    if (opts->precision == VIE_MIXED)
      run_batch<float, float>(B, fleet_mvm<float>(P0, F, n), to, mo, lag, prec, ti, mi, graphs, false, s);
    else if (opts->precision == VIE_MIXED_INNER)
      run_batch<double, float>(B, fleet_mvm<double>(P0, F, n), to, mo, lag, prec, ti, mi, graphs, false, s);
    else
      run_batch<double, double>(B, fleet_mvm<double>(P0, F, n), to, mo, lag, prec, ti, mi, graphs, false, s);
    int64_t acc[3] = {0, 0, 0};
    if (prec) copy_out(acc, F.replica->d_acc.p, sizeof(acc), s, "acc");
    std::vector<KState> st(n);
    std::vector<int> status(n);
    copy_out(st.data(), F.state.p, n * sizeof(KState), s, "batch state");
    copy_out(status.data(), F.status.p, n * sizeof(int), s, "batch status");
    const double batch_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // per problem: true residual, refinement (mixed), fields, statistics
    for (int r = 0; r < n; ++r) {
      vie_problem& P = *ps[r];
      hip_check(hipMemcpyAsync(P.vec[V_B], B.vec(BV_B) + r * n3, n3 * sizeof(c128), hipMemcpyDeviceToDevice, s),
                "batch rhs");
      hip_check(hipMemcpyAsync(P.vec[V_X], B.vec(BV_X) + r * n3, n3 * sizeof(c128), hipMemcpyDeviceToDevice, s),
                "batch iterate");
      const RunResult rr{st[r], status[r]};
      keep(solve_impl(&P, nullptr, opts, eout(r), pol(r), stats ? &stats[r] : nullptr, s, &rr));
      if (stats) {
        stats[r].seconds += batch_s;
        stats[r].inner_iters_total += acc[0];   // the batch's totals (all problems)
        stats[r].precond_applies += acc[1];
      }
    }
    return worst;
  });
}

vie_status vie_solve(vie_problem* p, const double* e_inc, const vie_opts* opts, double* e_tot_out, double* pol_out,
                     vie_stats* stats) {
  return guarded([&]() -> vie_status {
    if (!p || !e_inc || !e_tot_out) fail(VIE_EINVAL, "problem, e_inc and e_tot_out are required");
    validate_opts(opts, !p->groups.empty());
    const int64_t n = 3 * p->nv;
    for (int64_t i = 0; i < 2 * n; ++i)
      if (!is_finite(e_inc[i])) fail(VIE_EINVAL, "e_inc has non-finite entries");
    std::lock_guard<std::mutex> lk(p->mu);
    set_device(p->ctx);
    hipStream_t s = p->ctx->stream;
    DevBuf din(n * sizeof(c128)), dout(n * sizeof(c128)), dpol;
    if (pol_out) dpol.alloc(n * sizeof(c128));
    hip_check(hipMemcpyAsync(din.p, e_inc, n * sizeof(c128), hipMemcpyHostToDevice, s), "upload e_inc");
    vie_status st = solve_impl(p, din.as<c128>(), opts, dout.as<c128>(), pol_out ? dpol.as<c128>() : nullptr, stats, s);
    hip_check(hipMemcpyAsync(e_tot_out, dout.p, n * sizeof(c128), hipMemcpyDeviceToHost, s), "download e_tot");
    if (pol_out) hip_check(hipMemcpyAsync(pol_out, dpol.p, n * sizeof(c128), hipMemcpyDeviceToHost, s), "download pol");
    hip_check(hipStreamSynchronize(s), "download");
    return st;
  });
}

static void start_server(vie_context* ctx, int slots, int cap) {
  auto srv = std::make_unique<Server>();
  srv->ctx = ctx;
  srv->start(slots, cap);
  ctx->server = std::move(srv);
}

vie_status vie_server_start(vie_context* ctx, int32_t slots, int32_t queue_cap) {
  return guarded([&]() -> vie_status {
    if (!ctx) fail(VIE_EINVAL, "ctx is NULL");
    if (slots < 1 || slots > 64) fail(VIE_EINVAL, "slots must be in [1, 64]");
    if (queue_cap < 1) fail(VIE_EINVAL, "queue_cap must be >= 1");
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (ctx->server) fail(VIE_EBUSY, "server already running");
    start_server(ctx, slots, queue_cap);
    return VIE_OK;
  });
}

// Set-up scratch of the spectra (6 full kernels in FP64, one length set at
// a time) for lengths not cached (all of them with `all_spectra`).
static size_t transient_bytes(vie_context* ctx, const ProblemPlan& pl, bool all_spectra = false) {
  size_t t = 0;
  auto one = [&](int lx, int ly, int lz) {
    if (all_spectra || !spectra_cached(ctx, lx, ly, lz, pl.g, pl.k0))
      t = std::max(t, 6 * (size_t)lx * ly * lz * sizeof(c128));
  };
  one(pl.lx, pl.ly, pl.lz);
  for (const auto& gp : pl.groups) one(gp.lx, gp.ly, gp.lz);
  return t;
}

vie_status vie_footprint(vie_context* ctx, const vie_grid* grid, const double* eps_r, const int32_t* block_id,
                         int32_t n_blocks, size_t* bytes) {
  return guarded([&]() -> vie_status {
    if (!ctx || !grid || !eps_r || !bytes) fail(VIE_EINVAL, "ctx, grid, eps_r and bytes are required");
    const ProblemPlan pl = make_plan(*grid, eps_r, block_id, n_blocks);
    *bytes = plan_footprint(ctx, pl) + transient_bytes(ctx, pl);
    return VIE_OK;
  });
}

vie_status vie_submit(vie_context* ctx, const vie_grid* grid, const double* eps_r, const int32_t* block_id,
                      int32_t n_blocks, const double* e_inc, const vie_opts* opts, vie_ticket* out) {
  return guarded([&]() -> vie_status {
    if (!out) fail(VIE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !grid || !eps_r || !e_inc || !opts) fail(VIE_EINVAL, "ctx, grid, eps_r, e_inc and opts are required");
    auto r = std::make_unique<vie_request>();
    r->plan = make_plan(*grid, eps_r, block_id, n_blocks);
    r->opts = *opts;
    validate_opts(opts, !r->plan.groups.empty());
    if (opts->solver != VIE_SOLVER_BICGSTAB) fail(VIE_EINVAL, "the request server runs BiCGSTAB solves only");
    const int64_t n = 2 * 3 * r->plan.nv;
    r->e_inc.assign(e_inc, e_inc + n);
    for (double v : r->e_inc)
      if (!is_finite(v)) fail(VIE_EINVAL, "e_inc has non-finite entries");
    set_device(ctx);
    // reserved whatever the cache holds now, plus the request's own incident
    // and result buffers on the device
    r->footprint = plan_footprint(ctx, r->plan, true) + transient_bytes(ctx, r->plan, true) +
                   2 * 3 * (size_t)r->plan.nv * sizeof(c128);
    if (ctx->budget && r->footprint > ctx->budget) fail(VIE_EINVAL, "request needs more memory than the context budget");
    {
      std::lock_guard<std::mutex> lk(ctx->server_mu);
      if (!ctx->server) start_server(ctx, 4, 1024);
    }
    Server& S = *ctx->server;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      if ((int)S.queue.size() >= S.queue_cap) fail(VIE_EBUSY, "request queue is full");
      r->t_submit = std::chrono::steady_clock::now();
      r->server = &S;
      S.queue.push_back(r.get());
      ++S.outstanding;
    }
    *out = r.release();
    S.cv_work.notify_all();
    return VIE_OK;
  });
}

vie_status vie_wait(vie_ticket t, double timeout_s, double* e_tot_out, vie_stats* stats, double* times) {
  return guarded([&]() -> vie_status {
    if (!t) fail(VIE_EINVAL, "ticket is NULL");
    vie_request* r = t;
    Server* S = nullptr;
    // the request's server is the one whose queue or workers hold it; every
    // request was submitted to a context whose server outlives its tickets
    S = r->server;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto done = [&] { return r->state == vie_request::DONE; };
      if (timeout_s < 0)
        S->cv_done.wait(lk, done);
      else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
        fail(VIE_ETIMEDOUT, "request not finished");
      --S->outstanding;
    }
    std::unique_ptr<vie_request> own(r);
    if (e_tot_out && !r->e_tot.empty()) std::memcpy(e_tot_out, r->e_tot.data(), r->e_tot.size() * sizeof(double));
    if (stats) {
      int32_t* hist = stats->inner_hist;
      const int64_t cap = stats->inner_hist_cap;
      *stats = r->stats;
      stats->inner_hist = hist;
      stats->inner_hist_cap = cap;
      stats->inner_hist_len = 0;
    }
    if (times) {
      using d = std::chrono::duration<double>;
      const bool ran = r->t_start.time_since_epoch().count() != 0;
      const bool solved = r->t_solve.time_since_epoch().count() != 0;
      times[0] = ran ? d(r->t_start - r->t_submit).count() : d(r->t_end - r->t_submit).count();
      times[1] = solved ? d(r->t_solve - r->t_start).count() : 0.0;
      times[2] = solved ? d(r->t_end - r->t_solve).count() : 0.0;
    }
    if (r->status != VIE_OK) g_last_error = r->error;
    return r->status;
  });
}

vie_status vie_cancel(vie_ticket t) {
  return guarded([&]() -> vie_status {
    if (!t) fail(VIE_EINVAL, "ticket is NULL");
    vie_request* r = t;
    Server* S = r->server;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      r->cancel.store(true);
      if (r->state == vie_request::QUEUED) {
        auto it = std::find(S->queue.begin(), S->queue.end(), r);
        if (it != S->queue.end()) S->queue.erase(it);
        r->status = VIE_ECANCELLED;
        r->error = "request cancelled";
        r->t_end = std::chrono::steady_clock::now();
        r->state = vie_request::DONE;
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    return VIE_OK;
  });
}

}  // extern "C"
