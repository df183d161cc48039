// C ABI of the two-grid algebraic multiscale preconditioner (see include/amsp.h):
// handle lifetime, device setup orchestration, the preconditioner apply and
// the preconditioned CG driver.  All arithmetic runs in the HIP kernels;
// this file moves data, launches kernels and reads back status words.
#include <hip/hip_bf16.h>

#include <cfloat>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/amsp.h"
#include "amsp_internal.h"
#include "amsp_plan.h"
#include "amsp_tree.h"

using namespace amsp;

namespace {

thread_local std::string g_setup_error;

// Device allocations of one handle (thread-safe: the coupling-plan thread
// allocates while the main thread runs the setup).
// Device blocks of 1 MiB and more are recycled across handles in this
// process (up to kDevCacheCap): large hipMalloc / hipFree calls cost up to a
// few milliseconds each, and a setup makes dozens of them.  A block enters
// the cache only after a device-wide synchronisation (as hipFree would do),
// so that no queued work can still touch it when it is handed out again.
constexpr size_t kDevCacheMin = size_t(1) << 20;
constexpr size_t kDevCacheCap = size_t(8) << 30;
void release_dev_cache();
struct DevCache {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void *> free_blocks;  // (device, size) -> block
  size_t held = 0;
  static DevCache &get() {
    // never destroyed (handles may outlive statics); the free blocks are
    // released at exit, before the HIP runtime tears down (handlers run in
    // reverse order of registration, and this one is registered after the
    // runtime's first use)
    static DevCache *c = [] {
      std::atexit(release_dev_cache);
      return new DevCache();
    }();
    return *c;
  }
  // a cached block of at least `size` bytes (at most a quarter more), with
  // its real size in *got; null when there is none
  void *take(int dev, size_t size, size_t *got) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = free_blocks.lower_bound({dev, size});
    if (it == free_blocks.end() || it->first.first != dev || it->first.second > size + size / 4)
      return nullptr;
    void *p = it->second;
    *got = it->first.second;
    held -= *got;
    free_blocks.erase(it);
    return p;
  }
  bool put(int dev, size_t size, void *p) {  // false: over the cap, caller frees
    std::lock_guard<std::mutex> lk(mu);
    if (held + size > kDevCacheCap) return false;
    free_blocks.emplace(std::make_pair(dev, size), p);
    held += size;
    return true;
  }
  // hipFree every cached block on its own device (none is in use: a block
  // enters the cache only after a device-wide synchronisation)
  void release() {
    std::lock_guard<std::mutex> lk(mu);
    if (free_blocks.empty()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : free_blocks) {
      (void)hipSetDevice(kv.first.first);
      (void)hipFree(kv.second);
    }
    (void)hipSetDevice(cur);
    free_blocks.clear();
    held = 0;
  }
};
void release_dev_cache() { DevCache::get().release(); }

struct DevArena {
  struct Blk {
    void *p;
    size_t size;  // allocated size (a cached block may be larger than asked)
    int dev;
  };
  std::mutex mu;
  std::vector<Blk> blks;
  size_t bytes = 0;
  ~DevArena() { release(); }
  static void give_back(const Blk &b) {
    if (b.size < kDevCacheMin || !DevCache::get().put(b.dev, b.size, b.p)) (void)hipFree(b.p);
  }
  void release() {
    std::lock_guard<std::mutex> lk(mu);
    if (!blks.empty()) (void)hipDeviceSynchronize();
    for (const Blk &b : blks) give_back(b);
    blks.clear();
    bytes = 0;
  }
  template <typename T>
  T *alloc(size_t count) {
    if (count == 0) count = 1;
    size_t size = count * sizeof(T);
    int dev = 0;
    (void)hipGetDevice(&dev);
    void *p = nullptr;
    size_t got = size;
    if (size >= kDevCacheMin) {
      size = (size + kDevCacheMin - 1) & ~(kDevCacheMin - 1);
      got = size;
      p = DevCache::get().take(dev, size, &got);
    }
    if (!p && hipMalloc(&p, size) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    blks.push_back({p, got, dev});
    bytes += count * sizeof(T);
    return static_cast<T *>(p);
  }
  void free_one(void *p) {
    std::lock_guard<std::mutex> lk(mu);
    for (size_t k = 0; k < blks.size(); ++k)
      if (blks[k].p == p) {
        (void)hipDeviceSynchronize();
        give_back(blks[k]);
        blks.erase(blks.begin() + k);
        return;
      }
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

constexpr size_t kStageBytes = size_t(4) << 20;

struct amsp_handle {
  amsp_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;  // the device current at setup (holds every buffer)
  int n = 0, N = 0, nev = 0, nc = 0, T0 = 0;
  int64_t nnz = 0;
  HostPlan hp;
  DevArena mem;
  // matrix
  int *rowptr = nullptr, *col = nullptr;
  double *val = nullptr;
  // sliced copy for the CG matrix product (64-row slices, column-major)
  long long *sptr = nullptr;
  int *scol = nullptr;
  double *sval = nullptr;
  // plan
  Plan plan{};
  CoarsePlan cplan{};
  int *inv_ptr = nullptr, *inv_sd = nullptr, *inv_loc = nullptr;
  int *inv_x = nullptr;  // scatter: index of each copy in the local outputs
  int ntilerows = 0;
  // local factors and basis
  double *sdiag = nullptr;
  double *fac64 = nullptr;  // tile pool of the local factors (setup only)
  // the apply's local factors: packed inverse diagonal tiles and the envelope
  // (row and column forms), in the apply's precision
  double *dg64 = nullptr, *erow64 = nullptr, *ecol64 = nullptr;  // FP64 form
  float *fst32 = nullptr, *bst32 = nullptr;  // mixed forms: per-sweep streams
  long long nst_f = 0, nst_b = 0;            // stream lengths (entries)
  double *phi64 = nullptr;
  void *phi_lo = nullptr;  // float or bf16 copy used by the mixed apply
  void *phi_nat = nullptr; // the apply's basis in ascending-index layout, by columns
  double *lam = nullptr;   // N*(nev+1)
  // coarse
  double *a0keep = nullptr;  // copy of A0 tiles before factorisation (introspection)
  // multiplicative cycle: work vectors and the smoother weight
  double *mq = nullptr, *mt = nullptr, *mc = nullptr;
  double omega = 1.0;
  int max_mult = 1;
  // several right-hand sides per pass (allocated on first use): gathered and
  // solved blocks, region outputs, coarse vectors, and for the mixed forms
  // the f32 factor in the block solve's layout
  double *bX = nullptr, *bY = nullptr, *bXN = nullptr, *bC = nullptr, *bT = nullptr,
         *bC2 = nullptr, *bPart = nullptr;
  float *dg32 = nullptr, *er32 = nullptr, *ec32 = nullptr;
  int *loc_scratch = nullptr;  // local CSR build, large regions only
  int *inv_work = nullptr, *max_mult_dev = nullptr;  // inverse map build
  double *W0 = nullptr;
  float *W0f = nullptr;
  // sparse coarse factorisation (coarse_solver 2): plan, its device tables,
  // the fronts' X in the apply's precision, own-row and update vectors
  bool tree = false;
  TreePlan tp;
  TreeDev td{};
  double *X64 = nullptr;
  float *X32 = nullptr;
  double *ty = nullptr, *tv = nullptr;
  // apply scratch
  double *xloc = nullptr, *cvec = nullptr, *t1 = nullptr, *tvec = nullptr, *trmv_part = nullptr;
  // pcg scratch
  double *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
  // partial sums (MAX_PARTIALS each): a = p.q and scratch, b = r.z (scatter),
  // c = r.z_old (flexible) and scratch, d = r.r
  double *part_a = nullptr, *part_b = nullptr, *part_c = nullptr, *part_d = nullptr;
  double *scal = nullptr;
  PcgState *st = nullptr;
  PcgState *st_host = nullptr;               // two pinned slots for state copies
  hipEvent_t st_ev[2] = {nullptr, nullptr};  // completion of each slot's copy
  double *gm_host = nullptr;                 // GMRES: two pinned slots of 129 coefficients
  hipEvent_t gm_ev[2] = {nullptr, nullptr};
  double *hist = nullptr;  // recursive residual history of the last PCG call
  int hist_cap = 0, hist_len = 0;
  double hist_f2 = 0.0;
  amsp_setup_info sinfo{};
  std::string err;
  // per-launch HIP-event timing of the PCG kernels (opt.timing)
  std::vector<hipEvent_t> evs;
  size_t ev_used = 0;
  // timed launches: class, index of the start event, and the CG segment and
  // step they belong to (steps at or after the segment's converged count
  // return at once and are left out of the averages)
  struct EvRec {
    int cls, idx, seg, t;
  };
  std::vector<EvRec> ev_rec;
  int cur_seg = 0, cur_t = -1;  // launch context set by the CG driver
  std::vector<int> seg_cut;     // completed CG steps of each finished segment
  bool timing_active = false;
  int ev_count[5] = {0, 0, 0, 0, 0};  // launches per class seen by tstart (for the stride)
  // page-locked staging area for the setup's small uploads (a block of the
  // planner's cache): copies from pageable memory can stall the host for
  // milliseconds in the runtime; staged ones are plain DMA
  char *stage = nullptr;
  size_t stage_off = 0;
  ~amsp_handle() {
    if (stage) plan_free(stage, kStageBytes);
    for (hipEvent_t e : evs) hipEventDestroy(e);
    for (hipEvent_t e : st_ev)
      if (e) hipEventDestroy(e);
    for (hipEvent_t e : gm_ev)
      if (e) hipEventDestroy(e);
    if (st_host) hipHostFree(st_host);
    if (gm_host) hipHostFree(gm_host);
  }
};

static hipEvent_t next_event(amsp_handle *h) {
  if (h->ev_used == h->evs.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->evs.push_back(e);
  }
  return h->evs[h->ev_used++];
}

static int tstart(amsp_handle *h, int cls) {
  if (!h->timing_active || !(h->opt.timing & (1 << cls))) return -1;
  const int k = h->ev_count[cls]++;
  if (k % std::max(1, h->opt.timing_stride) != 0) return -1;
  const int idx = (int)h->ev_used;
  hipEvent_t e = next_event(h);
  if (!e) return -1;
  hipEventRecord(e, h->stream);
  return idx;
}

// Like tstart, but for a single kernel launched with its own start/stop
// events (hipExtLaunchKernelGGL): returns both events unrecorded, or nulls.
static int tpair(amsp_handle *h, int cls, hipEvent_t *e0, hipEvent_t *e1) {
  *e0 = *e1 = nullptr;
  if (!h->timing_active || !(h->opt.timing & (1 << cls))) return -1;
  const int k = h->ev_count[cls]++;
  if (k % std::max(1, h->opt.timing_stride) != 0) return -1;
  const int idx = (int)h->ev_used;
  *e0 = next_event(h);
  *e1 = next_event(h);
  if (!*e0 || !*e1) {
    *e0 = *e1 = nullptr;
    return -1;
  }
  return idx;
}

static void tpair_done(amsp_handle *h, int cls, int idx) {
  if (idx >= 0) h->ev_rec.push_back({cls, idx, h->cur_seg, h->cur_t});
}

static void tstop(amsp_handle *h, int cls, int idx) {
  if (idx < 0) return;
  hipEvent_t e = next_event(h);
  if (!e) return;
  hipEventRecord(e, h->stream);
  h->ev_rec.push_back({cls, idx, h->cur_seg, h->cur_t});
}

#define HIP_TRY(expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      h->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return AMSP_ERR_HIP;                                                \
    }                                                                     \
  } while (0)

#define ALLOC(dst, T, count)                                              \
  do {                                                                    \
    dst = h->mem.alloc<T>(count);                                         \
    if (!dst) {                                                           \
      h->err = std::string("device allocation failed: " #dst ": ") +       \
               hipGetErrorString(hipGetLastError());                      \
      return AMSP_ERR_OOM;                                                \
    }                                                                     \
  } while (0)

// Source of an upload of `bytes` from host memory `src` on the handle's
// stream: a copy in the staging area when the data is small and fits (the
// area is reused only after the stream has been synchronised:
// stage_release), else src itself.
static const void *stage_src(amsp_handle *h, hipStream_t stream, const void *src, size_t bytes) {
  if (stream != h->stream || bytes == 0 || bytes > kStageBytes / 4) return src;
  if (!h->stage) {
    h->stage = static_cast<char *>(plan_alloc(kStageBytes));
    if (!h->stage) return src;
  }
  const size_t at = (h->stage_off + 255) & ~size_t(255);
  if (at + bytes > kStageBytes) return src;
  std::memcpy(h->stage + at, src, bytes);
  h->stage_off = at + bytes;
  return h->stage + at;
}
// The stream has been synchronised: every staged copy has completed.
static void stage_release(amsp_handle *h) { h->stage_off = 0; }

template <typename V>
static typename V::value_type *upload_on(amsp_handle *h, hipStream_t stream, const V &v, bool &ok) {
  using T = typename V::value_type;
  T *d = h->mem.alloc<T>(v.size());
  if (!d) {
    ok = false;
    return nullptr;
  }
  const size_t bytes = v.size() * sizeof(T);
  if (!v.empty() && hipMemcpyAsync(d, stage_src(h, stream, v.data(), bytes), bytes,
                                   hipMemcpyHostToDevice, stream) != hipSuccess) {
    ok = false;
    return nullptr;
  }
  return d;
}

template <typename V>
static typename V::value_type *upload(amsp_handle *h, const V &v, bool &ok) {
  return upload_on(h, h->stream, v, ok);
}

extern "C" void amsp_default_options(amsp_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->overlap = 1;
  opt->precision = AMSP_FP64;
  opt->pou = 0;
  opt->local_order = AMSP_ORDER_RCM;
  opt->dense_tiles = 0;
  opt->eig_tol = 0.0;  // 0: 1e-12 (FP64) or 1e-4 (mixed forms)
  opt->eig_maxit = 80;
  opt->eig_shift = 1e-4;
  opt->chunk = 8;
  opt->flexible = -1;  // -1: on for the mixed forms
  opt->keep_a0 = 0;
  opt->timing = 0;
  opt->timing_stride = 1;
  opt->stream = nullptr;
  opt->singular = 0;
}

static amsp_status sync_status(amsp_handle *h, const int *dstatus, int N, int mask, int &first_bad) {
  std::vector<int> st(N);
  HIP_TRY(hipMemcpyAsync(st.data(), dstatus, N * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  first_bad = -1;
  for (int i = 0; i < N; ++i)
    if (st[i] & mask) {
      first_bad = i;
      break;
    }
  return AMSP_OK;
}

// Device copies of the coupling plan (filled by the coupling thread, copied
// into the handle's plans at the join).
struct CouplingDev {
  int *ext_ptr = nullptr, *ext_rowptr = nullptr, *ext_src = nullptr, *ext_loc = nullptr;
  int npairs = 0;
  int *pair_i = nullptr, *pair_j = nullptr, *pair_ptr = nullptr, *pair_l = nullptr,
      *pair_e = nullptr;
};

static bool upload_coupling(amsp_handle *h, hipStream_t stream, CouplingDev &d);

// Second planning phase (multiplicities, inverse map, extended regions,
// coupled pairs) on a host thread while the device extracts, factors and
// solves the local eigenproblems.  The thread also uploads the result on a
// stream of its own and waits for the copies, so the join hands over
// resident device arrays.
struct CouplingTask {
  std::thread th;
  int status = AMSP_OK;
  std::string msg;
  bool joined = true;
  double run_ms = 0.0, wait_ms = 0.0;
  CouplingDev dev;
  void start(amsp_handle *h, const amsp_csr *A, HostPlan *P, hipStream_t stream, int device) {
    joined = false;
    const amsp_options opt = h->opt;
    th = std::thread([this, h, A, opt, P, stream, device]() {
      const double t = now_ms();
      try {
        status = build_plan_coupling(A, opt, *P, msg);
        if (status == AMSP_OK) {
          if (hipSetDevice(device) != hipSuccess || !upload_coupling(h, stream, dev) ||
              hipStreamSynchronize(stream) != hipSuccess) {
            status = AMSP_ERR_OOM;
            msg = "device allocation or upload failed (coupling plan)";
          }
        }
      } catch (const std::bad_alloc &) {
        status = AMSP_ERR_OOM;
        msg = "host allocation failed during planning";
      }
      run_ms = now_ms() - t;
    });
  }
  int join() {
    if (!joined) {
      const double t = now_ms();
      th.join();
      wait_ms = now_ms() - t;
      joined = true;
    }
    return status;
  }
  ~CouplingTask() { join(); }
};

// A second stream (default priority) with two events, released on scope exit
// after the stream has drained.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t create() {
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e0, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
    return e;
  }
  ~SideStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Entries of one local factor set: the off-diagonal tiles, then one packed
// lower-triangular diagonal tile (DE entries) per tile row.
static size_t factor_elems(const HostPlan &P) {
  return (size_t)P.noff * TE + (size_t)P.trow_ptr.back() * DE;
}

// Sparse coarse factorisation (see amsp_tree.h): symbolic plan on the host
// from the coupled pairs, then on the device the pair blocks of A0, their
// assembly into the fronts, and level by level the children's Schur
// complements, the tile Cholesky of the own columns and the fronts' X.  With
// keep_a0 the dense A0 is also formed (introspection only).
static amsp_status tree_coarse_setup(amsp_handle *h, const HostPlan &P) {
  const bool mixed = h->opt.precision != AMSP_FP64;
  const double t5 = now_ms();
  TreePlan &tp = h->tp;
  {
    std::string msg;
    if (!build_tree_plan(h->N, P.mi, P.coff, P.pair_i, P.pair_j, tp, msg)) {
      h->err = msg;
      return AMSP_ERR_ARG;
    }
  }
  bool ok = true;
  TreeDev &t = h->td;
  t.nfront = tp.nfront;
  t.K = upload(h, tp.K, ok);
  t.T = upload(h, tp.T, ok);
  t.kdof = upload(h, tp.kdof, ok);
  t.udof = upload(h, tp.udof, ok);
  t.dbase = upload(h, tp.dbase, ok);
  t.rbase = upload(h, tp.rbase, ok);
  t.vbase = upload(h, tp.vbase, ok);
  t.parent = upload(h, tp.parent, ok);
  t.fbase = upload(h, tp.fbase, ok);
  t.xbase = upload(h, tp.xbase, ok);
  t.row_coarse = upload(h, tp.row_coarse, ok);
  t.gptr = upload(h, tp.gptr, ok);
  t.gsrc = upload(h, tp.gsrc, ok);
  t.ea_row = upload(h, tp.ea_row, ok);
  t.ch_front = upload(h, tp.ch_front, ok);
  t.as_pair = upload(h, tp.as_pair, ok);
  t.as_rev = upload(h, tp.as_rev, ok);
  t.as_front = upload(h, tp.as_front, ok);
  t.as_ri = upload(h, tp.as_ri, ok);
  t.as_rj = upload(h, tp.as_rj, ok);
  t.pair_i = h->cplan.pair_i;
  t.pair_j = h->cplan.pair_j;
  if (!ok) {
    h->err = "device allocation or upload failed (coarse tree)";
    return AMSP_ERR_OOM;
  }
  const Plan &p = h->plan;
  const CoarsePlan &c = h->cplan;
  const int nn = h->nev * h->nev;
  double *W, *pb, *F, *dinv;
  int *cstat;
  ALLOC(W, double, (size_t)P.ext_ptr.back() * h->nev);
  ALLOC(pb, double, std::max<size_t>((size_t)c.npairs * nn, 1));
  ALLOC(F, double, (size_t)tp.ftiles * TE);
  ALLOC(h->X64, double, (size_t)tp.xtiles * TE);
  ALLOC(dinv, double, (size_t)std::max(tp.dtiles, 1) * TE);
  ALLOC(cstat, int, 1);
  ALLOC(h->ty, double, std::max(h->nc, 1));
  ALLOC(h->tv, double, std::max(tp.nvec, 1));
  HIP_TRY(hipMemsetAsync(cstat, 0, sizeof(int), h->stream));
  launch_fill(h->stream, (size_t)tp.ftiles * TE, F, 0.0);
  launch_fill(h->stream, (size_t)tp.xtiles * TE, h->X64, 0.0);
  launch_tree_init(h->stream, t, tp.nfront, tp.max_T, F, h->X64);
  launch_apply_A_to_basis(h->stream, p, c, h->val, h->phi64, W);
  launch_pair_blocks(h->stream, p, c, h->phi64, W, pb);
  launch_tree_assemble(h->stream, p, t, (int)tp.as_pair.size(), pb, F);
  HIP_TRY(hipGetLastError());
  if (h->opt.keep_a0) {  // the dense A0 for amsp_get_coarse_matrix
    const int T0 = h->T0;
    double *A0t;
    ALLOC(A0t, double, (size_t)T0 * T0 * TE);
    launch_fill(h->stream, (size_t)T0 * T0 * TE, A0t, 0.0);
    launch_pair_products(h->stream, p, c, h->phi64, W, A0t, T0);
    launch_symmetrize_tiles(h->stream, A0t, T0, h->nc);
    h->a0keep = A0t;
  }
  const int MS = std::max(tp.max_slots, 1);
  for (int lv = 0; lv < tp.nlevel; ++lv) {
    const int f0 = tp.lvl_ptr[lv], f1 = tp.lvl_ptr[lv + 1];
    for (int cs = 0; cs < tp.max_slots; ++cs) {
      const int a = tp.ch_ptr[(size_t)lv * MS + cs], b = tp.ch_ptr[(size_t)lv * MS + cs + 1];
      int maxU = 0;
      for (int q = a; q < b; ++q) {
        const int ch = tp.ch_front[q], U = tp.T[ch] - tp.K[ch];
        maxU = std::max(maxU, U * (U + 1) / 2);
      }
      launch_tree_extend_add(h->stream, t, t.ch_front + a, b - a, maxU, F);
    }
    for (int k = 0; k < tp.lvl_maxK[lv]; ++k)
      launch_tree_factor_step(h->stream, t, f0, f1, tp.lvl_maxT[lv], k, F, dinv, cstat);
    for (int k = 0; k < tp.lvl_maxK[lv]; ++k)
      launch_tree_inverse_step(h->stream, t, f0, f1, tp.lvl_maxT[lv], k, F, dinv, h->X64);
    HIP_TRY(hipGetLastError());
  }
  int cs = 0;
  HIP_TRY(hipMemcpyAsync(&cs, cstat, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  stage_release(h);
  if (cs) {
    h->err = "coarse matrix A0 not SPD";
    return AMSP_ERR_COARSE_NOT_SPD;
  }
  h->mem.free_one(W);
  h->mem.free_one(pb);
  h->mem.free_one(F);
  h->mem.free_one(dinv);
  h->mem.free_one(cstat);
  if (mixed) {
    ALLOC(h->X32, float, (size_t)tp.xtiles * TE);
    launch_tree_x_to_f32(h->stream, h->X64, h->X32, tp.xtiles);
    HIP_TRY(hipGetLastError());
    h->mem.free_one(h->X64);  // waits for the stream
    h->X64 = nullptr;
  }
  h->sinfo.coarse_fronts = tp.nfront;
  h->sinfo.coarse_levels = tp.nlevel;
  h->sinfo.coarse_gflop = tp.flops * 1e-9;
  h->sinfo.coarse_factor_mb = (double)tp.xtiles * TE * (mixed ? 4 : 8) * 1e-6;
  h->sinfo.phase_ms[6] = now_ms() - t5;
  return AMSP_OK;
}

// The coarse solve x = A0^{-1} c through the handle's factorisation.
static void coarse_solve_tree(amsp_handle *h, hipStream_t s, const double *c, double *x,
                              const int *done) {
  const TreePlan &tp = h->tp;
  if (h->X32)
    launch_tree_solve<float>(s, h->td, tp.lvl_ptr, tp.lvl_maxT, tp.lvl_maxK, tp.max_K, tp.max_T,
                             h->X32, c, h->ty, h->tv, x, done);
  else
    launch_tree_solve<double>(s, h->td, tp.lvl_ptr, tp.lvl_maxT, tp.lvl_maxK, tp.max_K, tp.max_T,
                              h->X64, c, h->ty, h->tv, x, done);
}

static amsp_status device_setup(amsp_handle *h, const amsp_csr *A) {
  HostPlan &P = h->hp;
  const bool mixed = h->opt.precision != AMSP_FP64;
  double t0 = now_ms();
  bool ok = true;
  // device blocks whose last reader is still queued: returned to the
  // arena after the final synchronisation instead of after a wait of their own
  std::vector<void *> deferred;
  SideStream up;  // declared before the task: outlives the thread that uses it
  HIP_TRY(up.create());
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  CouplingTask coupling;
  coupling.start(h, A, &P, up.s, device);
  auto join_coupling = [&]() -> amsp_status {
    const int cs = coupling.join();
    h->sinfo.coupling_ms = coupling.run_ms;
    h->sinfo.coupling_wait_ms = coupling.wait_ms;
    if (cs != AMSP_OK) {
      h->err = coupling.msg;
      return (amsp_status)cs;
    }
    const CouplingDev &d = coupling.dev;
    Plan &pl = h->plan;
    CoarsePlan &cp = h->cplan;
    cp.ext_ptr = d.ext_ptr;
    cp.ext_rowptr = d.ext_rowptr;
    cp.ext_src = d.ext_src;
    cp.ext_loc = d.ext_loc;
    cp.npairs = d.npairs;
    cp.pair_i = d.pair_i;
    cp.pair_j = d.pair_j;
    cp.pair_ptr = d.pair_ptr;
    cp.pair_l = d.pair_l;
    cp.pair_e = d.pair_e;
    return AMSP_OK;
  };
  const double host_plan_ms = h->sinfo.phase_ms[0];
  // --- upload matrix and plan
  double ta, tb;
  {
    // 32-bit row pointers and the sliced copy's slice starts, on the
    // planner's threads (64 chunks of rows; 64-row slices)
    const int n = h->n, ns = (n + 63) / 64;
    ivec rp32;
    rp32.resize(n + 1);
    std::vector<long long> sp(ns + 1);
    sp[0] = 0;
    plan_parallel_for(64, [&](int c) {
      const int s0 = (int)((long long)ns * c / 64), s1 = (int)((long long)ns * (c + 1) / 64);
      for (int sl = s0; sl < s1; ++sl) {
        int w = 0;
        for (int i = 64 * sl; i < std::min(n, 64 * sl + 64); ++i) {
          rp32[i] = (int)A->row_ptr[i];
          w = std::max(w, (int)(A->row_ptr[i + 1] - A->row_ptr[i]));
        }
        sp[sl + 1] = 64LL * w;  // widths first, then the running sum
      }
    });
    rp32[n] = (int)A->row_ptr[n];
    for (int sl = 0; sl < ns; ++sl) sp[sl + 1] += sp[sl];
    ta = now_ms();
    h->rowptr = upload(h, rp32, ok);
    h->col = h->mem.alloc<int>(h->nnz);
    h->val = h->mem.alloc<double>(h->nnz);
    if (!ok || !h->col || !h->val) {
      h->err = std::string("device allocation failed (matrix): ") + hipGetErrorString(hipGetLastError());
      return AMSP_ERR_OOM;
    }
    HIP_TRY(hipMemcpyAsync(h->col, A->col_idx, h->nnz * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->val, A->val, h->nnz * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    tb = now_ms();
    // sliced copy for the CG matrix product
    h->sptr = upload(h, sp, ok);
    h->scol = h->mem.alloc<int>(std::max<long long>(1, sp[ns]));
    h->sval = h->mem.alloc<double>(std::max<long long>(1, sp[ns]));
    if (!ok || !h->scol || !h->sval) {
      h->err = "device allocation failed (sliced matrix)";
      return AMSP_ERR_OOM;
    }
    launch_csr_to_sell(h->stream, h->n, h->rowptr, h->col, h->val, h->sptr, h->scol, h->sval);
    HIP_TRY(hipGetLastError());
  }
  Plan &p = h->plan;
  p.N = h->N;
  p.nev = h->nev;
  p.sd_ptr = upload(h, P.sd_ptr, ok);
  p.sd_dofs = upload(h, P.sd_dofs, ok);
  p.nat = upload(h, P.nat, ok);
  p.vp_ptr = upload(h, P.vp_ptr, ok);
  p.trow_ptr = upload(h, P.trow_ptr, ok);
  p.tfirst = upload(h, P.tfirst, ok);
  p.toff = upload(h, P.toff, ok);
  p.noff = P.noff;
  p.eptr = upload(h, P.eptr, ok);
  p.uptr = upload(h, P.uptr, ok);
  p.ebase = upload(h, P.ebase, ok);
  {
    // per-sweep streams of the mixed form's factor: start of every 64-row
    // block inside its region's stream, and of every region's stream
    const int ntr = P.trow_ptr.back();
    std::vector<int> sfb(ntr), sbb(ntr);
    std::vector<long long> sfr(h->N + 1, 0), sbr(h->N + 1, 0);
    for (int i = 0; i < h->N; ++i) {
      const int g0 = P.trow_ptr[i], nt = P.trow_ptr[i + 1] - g0;
      const int *ep = P.eptr.data() + P.vp_ptr[i] + i, *up = P.uptr.data() + P.vp_ptr[i] + i;
      long long of = 0, ob = 0;
      for (int I = 0; I < nt; ++I) {
        sfb[g0 + I] = (int)of;
        of += ((ep[I * TS + TS] - ep[I * TS] + 3) & ~3) + DE;
      }
      for (int J = nt - 1; J >= 0; --J) {
        sbb[g0 + J] = (int)ob;
        ob += ((up[J * TS + TS] - up[J * TS] + 3) & ~3) + DE;
      }
      if (of > INT_MAX || ob > INT_MAX) {
        h->err = "region " + std::to_string(i) + " too large for the local apply's stream";
        return AMSP_ERR_ARG;
      }
      sfr[i + 1] = sfr[i] + of;
      sbr[i + 1] = sbr[i] + ob;
    }
    p.sfb = upload(h, sfb, ok);
    p.sbb = upload(h, sbb, ok);
    p.sfr = upload(h, sfr, ok);
    p.sbr = upload(h, sbr, ok);
    h->nst_f = sfr[h->N];
    h->nst_b = sbr[h->N];
  }
  p.loc_rowptr = upload(h, P.loc_rowptr, ok);
  {  // the entries of the local CSR are built here from A's device CSR
    int *lc = nullptr, *ls = nullptr, *gs = nullptr;
    ALLOC(lc, int, std::max<long long>(P.nloc, 1));
    ALLOC(ls, int, std::max<long long>(P.nloc, 1));
    if (local_csr_lds_bytes(P.max_ni) > LOCAL_CSR_LDS_MAX)
      ALLOC(gs, int, std::max<size_t>((size_t)2 * P.sd_ptr.back(), 1));
    p.loc_col = lc;
    p.loc_src = ls;
    h->loc_scratch = gs;
    launch_local_csr(h->stream, p, P.max_ni, h->rowptr, h->col, lc, ls, gs);
    HIP_TRY(hipGetLastError());
  }
  {  // multiplicities and the inverse map, from the regions on the device
    const int n = h->n, ne = P.sd_ptr.back();
    int *mult = nullptr, *iptr = nullptr, *isd = nullptr, *iloc = nullptr;
    ALLOC(mult, int, std::max(n, 1));
    ALLOC(iptr, int, n + 1);
    ALLOC(isd, int, std::max(ne, 1));
    ALLOC(iloc, int, std::max(ne, 1));
    ALLOC(h->inv_work, int, (size_t)n + (n + 4 * WG - 1) / (4 * WG) + 1);
    ALLOC(h->max_mult_dev, int, 1);
    launch_inverse_map(h->stream, p, n, mult, iptr, isd, iloc, h->inv_work, h->max_mult_dev);
    HIP_TRY(hipGetLastError());
    p.mult = mult;
    h->inv_ptr = iptr;
    h->inv_sd = isd;
    h->inv_loc = iloc;
  }
  p.mi = upload(h, P.mi, ok);
  p.coff = upload(h, P.coff, ok);
  CoarsePlan &c = h->cplan;
  c.N = h->N;
  c.nev = h->nev;
  if (!ok) {
    h->err = "device allocation or upload failed (plan)";
    return AMSP_ERR_OOM;
  }
  h->ntilerows = P.trow_ptr.back();
  const int sum_ni = P.sd_ptr.back();
  const int sum_npad = P.vp_ptr.back();
  HIP_TRY(hipStreamSynchronize(h->stream));
  stage_release(h);
  double t1 = now_ms();
  h->sinfo.phase_ms[1] = tb - ta;                   // input matrix transfer only
  h->sinfo.phase_ms[0] += (ta - t0) + (t1 - tb);  // planning includes its index uploads
  h->sinfo.plan_host_ms = host_plan_ms;
  h->sinfo.plan_upload_ms = (ta - t0) + (t1 - tb);

  int *status;
  ALLOC(status, int, h->N);
  HIP_TRY(hipMemsetAsync(status, 0, h->N * sizeof(int), h->stream));
  ALLOC(h->sdiag, double, sum_ni);
  const size_t fac_elems = factor_elems(P);
  ALLOC(h->fac64, double, fac_elems);
  if (h->nev > 0) {
    launch_neumann_diag(h->stream, p, h->val, h->sdiag, status);
    int bad;
    amsp_status s = sync_status(h, status, h->N, 1, bad);
    if (s != AMSP_OK) return s;
    if (bad >= 0) {
      h->err = "weighting matrix S_i not positive in subdomain " + std::to_string(bad);
      return AMSP_ERR_NEUMANN_DIAG;
    }
  }
  // --- local Dirichlet matrices and their factors
  launch_extract_tiles(h->stream, p, h->ntilerows, h->val, h->sdiag, h->fac64, 0, 0.0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->stream));
  stage_release(h);
  double t2 = now_ms();
  h->sinfo.phase_ms[2] = t2 - t1;
  launch_profile_cholesky(h->stream, p, h->fac64, status, 2);
  HIP_TRY(hipGetLastError());
  {
    int bad;
    amsp_status s = sync_status(h, status, h->N, 2, bad);
    if (s != AMSP_OK) return s;
    if (bad >= 0) {
      h->err = "local matrix not SPD in subdomain " + std::to_string(bad);
      return AMSP_ERR_LOCAL_NOT_SPD;
    }
  }
  double t3 = now_ms();
  h->sinfo.phase_ms[3] = t3 - t2;

  // --- local eigenproblems
  ALLOC(h->lam, double, (size_t)h->N * (h->nev + 1));
  launch_fill(h->stream, (size_t)h->N * (h->nev + 1), h->lam, std::nan(""));
  if (h->nev > 0) {
    double *facB, *X, *Yb, *BY, *bval, *GK, *CC;
    int *conv;
    ALLOC(facB, double, fac_elems);
    ALLOC(X, double, (size_t)sum_npad * EIGP);
    ALLOC(Yb, double, (size_t)sum_npad * EIGP);
    ALLOC(BY, double, (size_t)sum_npad * EIGP);
    ALLOC(bval, double, std::max<long long>(P.nloc, 1));
    ALLOC(GK, double, (size_t)h->N * 2 * EIGP * EIGP);
    ALLOC(CC, double, (size_t)h->N * (EIGP * EIGP + EIGP));
    ALLOC(conv, int, h->N);
    HIP_TRY(hipMemsetAsync(conv, 0, h->N * sizeof(int), h->stream));
    launch_extract_tiles(h->stream, p, h->ntilerows, h->val, h->sdiag, facB, 1, h->opt.eig_shift);
    launch_profile_cholesky(h->stream, p, facB, status, 4);
    // the sweeps' factor: packed inverse diagonal tiles + envelope, in the
    // sweep precision (f32 in the mixed forms)
    const size_t ndiag = (size_t)h->ntilerows * DE, nenv = (size_t)P.nenv;
    const double *dsrcB = facB + (size_t)P.noff * TE;
    float *dgB32 = nullptr, *erB32 = nullptr, *ecB32 = nullptr;
    double *dgB64 = nullptr, *erB64 = nullptr, *ecB64 = nullptr;
    if (mixed) {
      ALLOC(dgB32, float, ndiag);
      ALLOC(erB32, float, nenv);
      ALLOC(ecB32, float, nenv);
      launch_tiles_to_f32(h->stream, dsrcB, dgB32, ndiag);
      launch_env_from_tiles<float>(h->stream, p, h->ntilerows, facB, erB32, ecB32);
    } else {
      ALLOC(dgB64, double, ndiag);
      ALLOC(erB64, double, nenv);
      ALLOC(ecB64, double, nenv);
      HIP_TRY(hipMemcpyAsync(dgB64, dsrcB, ndiag * sizeof(double), hipMemcpyDeviceToDevice,
                             h->stream));
      launch_env_from_tiles<double>(h->stream, p, h->ntilerows, facB, erB64, ecB64);
    }
    {
      int bad;
      amsp_status s = sync_status(h, status, h->N, 4, bad);
      if (s != AMSP_OK) return s;
      if (bad >= 0) {
        h->err = "shifted eigen-operator not SPD in subdomain " + std::to_string(bad);
        return AMSP_ERR_LOCAL_NOT_SPD;
      }
    }
    h->mem.free_one(facB);
    facB = nullptr;
    launch_eig_init(h->stream, p, h->sdiag, X);
    launch_eig_bval(h->stream, p, h->val, h->sdiag, bval);
    const double tol = h->opt.eig_tol > 0 ? h->opt.eig_tol : (mixed ? 1e-4 : 1e-12);
    std::vector<int> hconv(h->N);
    int sweeps = 0, unconv = h->N;
    // Convergence is checked every second sweep from the fourth.  Each
    // check's flags are copied to pinned memory behind its sweep and read
    // two sweeps later, so the device does not wait for the host; every
    // kernel of a sweep skips converged regions, so the sweeps run past the
    // point where all have converged change nothing.
    int *conv_host = nullptr;
    hipEvent_t conv_ev = nullptr;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&conv_host), h->N * sizeof(int),
                          hipHostMallocDefault));
    struct PinnedFlags {
      int *p;
      hipEvent_t e;
      ~PinnedFlags() {
        if (e) (void)hipEventDestroy(e);
        if (p) (void)hipHostFree(p);
      }
    } conv_guard{conv_host, nullptr};
    HIP_TRY(hipEventCreateWithFlags(&conv_ev, hipEventDisableTiming));
    conv_guard.e = conv_ev;
    int pending = 0;  // sweep whose flags are in flight to conv_host (0: none)
    for (int it = 1; it <= h->opt.eig_maxit; ++it) {
      if (mixed)
        launch_env_solve_block<float>(h->stream, p, dgB32, erB32, ecB32, X, Yb, conv);
      else
        launch_env_solve_block<double>(h->stream, p, dgB64, erB64, ecB64, X, Yb, conv);
      launch_eig_rr(h->stream, p, P.max_ni, h->val, h->sdiag, bval, Yb, BY, X, GK, CC, tol, conv,
                    h->lam, !mixed);
      sweeps = it;
      if (it >= 4 && (it % 2 == 0 || it == h->opt.eig_maxit)) {
        HIP_TRY(hipGetLastError());
        if (pending > 0) {
          HIP_TRY(hipEventSynchronize(conv_ev));
          unconv = 0;
          for (int i = 0; i < h->N; ++i) unconv += (conv_host[i] == 0);
          if (unconv == 0) {
            sweeps = pending;
            break;
          }
        }
        HIP_TRY(hipMemcpyAsync(conv_host, conv, h->N * sizeof(int), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipEventRecord(conv_ev, h->stream));
        pending = it;
      }
    }
    HIP_TRY(hipMemcpyAsync(hconv.data(), conv, h->N * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    unconv = 0;
    for (int v : hconv) unconv += (v == 0);
    h->sinfo.eig_sweeps = sweeps;
    h->sinfo.eig_unconverged = unconv;
    {
      const amsp_status js = join_coupling();
      if (js != AMSP_OK) return js;
    }
    ALLOC(h->phi64, double, (size_t)sum_ni * h->nev);
    launch_build_basis(h->stream, p, h->sdiag, X, h->phi64, h->opt.pou);
    // mixed forms: A0 is formed from the basis as stored (rounded), so the
    // coarse term stays the Galerkin projection of the basis it applies
    if (mixed && h->opt.coarse_basis == 0)
      launch_basis_round(h->stream, h->phi64, (size_t)sum_ni * h->nev,
                         h->opt.precision == AMSP_MIXED_BF16 ? 1 : 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (void *b : {(void *)dgB32, (void *)erB32, (void *)ecB32, (void *)dgB64, (void *)erB64,
                    (void *)ecB64})
      if (b) h->mem.free_one(b);
    h->mem.free_one(X);
    h->mem.free_one(Yb);
    h->mem.free_one(BY);
    h->mem.free_one(bval);
    h->mem.free_one(GK);
    h->mem.free_one(CC);
    h->mem.free_one(conv);
    // gap flags and mu_c
    std::vector<double> lam((size_t)h->N * (h->nev + 1));
    HIP_TRY(hipMemcpy(lam.data(), h->lam, lam.size() * sizeof(double), hipMemcpyDeviceToHost));
    double mu = INFINITY;
    int flags = 0;
    for (int i = 0; i < h->N; ++i) {
      const int m = P.mi[i];
      const int ni = P.sd_ptr[i + 1] - P.sd_ptr[i];
      if (m < ni) {
        const double lm = lam[(size_t)i * (h->nev + 1) + m - 1], lm1 = lam[(size_t)i * (h->nev + 1) + m];
        mu = std::min(mu, lm1);
        if (lm1 - lm < 1e-8 * std::max(lm1, 1e-12)) ++flags;
      }
    }
    h->sinfo.mu_c = mu;
    h->sinfo.n_gap_flags = flags;
  }
  if (h->nev == 0) {
    const amsp_status js = join_coupling();
    if (js != AMSP_OK) return js;
  }
  double t4 = now_ms();
  h->sinfo.phase_ms[4] = t4 - t3;

  // --- coarse matrix A0 = R0 A R0^T and its inverse factor
  const int T0 = h->T0;
  if (h->nc > 0 && h->tree) {
    const amsp_status ts = tree_coarse_setup(h, P);
    if (ts != AMSP_OK) return ts;
  } else if (h->nc > 0) {
    double *W, *A0t, *dinv;
    int *cstat;
    ALLOC(W, double, (size_t)P.ext_ptr.back() * h->nev);
    ALLOC(A0t, double, (size_t)T0 * T0 * TE);
    ALLOC(dinv, double, (size_t)T0 * TE);
    ALLOC(cstat, int, 1);
    HIP_TRY(hipMemsetAsync(cstat, 0, sizeof(int), h->stream));
    HIP_TRY(hipMemsetAsync(A0t, 0, (size_t)T0 * T0 * TE * sizeof(double), h->stream));
    launch_apply_A_to_basis(h->stream, p, c, h->val, h->phi64, W);
    launch_pair_products(h->stream, p, c, h->phi64, W, A0t, T0);
    launch_symmetrize_tiles(h->stream, A0t, T0, h->nc);
    HIP_TRY(hipGetLastError());
    if (h->opt.keep_a0) {
      ALLOC(h->a0keep, double, (size_t)T0 * T0 * TE);
      HIP_TRY(hipMemcpyAsync(h->a0keep, A0t, (size_t)T0 * T0 * TE * sizeof(double),
                             hipMemcpyDeviceToDevice, h->stream));
    }
    if (h->opt.singular) {  // pseudo-inverse on the consistent residuals
      double *u1, *alpha;
      ALLOC(u1, double, h->nc);
      ALLOC(alpha, double, 1);
      launch_singular_regularize(h->stream, p, h->phi64, A0t, T0, h->nc, u1, alpha);
      HIP_TRY(hipGetLastError());
      h->mem.free_one(u1);  // waits for the stream
      h->mem.free_one(alpha);
    }
    double t5 = now_ms();
    // Tiled right-looking Cholesky with lookahead.  Main stream: diagonal
    // factor, panel, then the update of the next tile column only, so the
    // next diagonal step can start while a second stream applies the rest of
    // the trailing update.  A third stream forms the inverse factor
    // W0 = inv(L0) by a right-looking solve of L0 X = I; its step k needs
    // only column k of L0, final once the panel of step k is done.
    //   main:  trsm(k) [panel] ... wait [rest of k-1] next(k)+potrf(k+1)
    //   bulk:  wait [panel] rest(k) [rest]
    //   inv:   wait [panel] inv_row(k) inv_update(k)
    ALLOC(h->W0, double, (size_t)T0 * T0 * TE);
    SideStream bulk, inv;
    HIP_TRY(bulk.create());
    HIP_TRY(inv.create());
    hipEvent_t ev_panel = bulk.e0, ev_rest = bulk.e1, ev_inv = inv.e1;
    HIP_TRY(hipEventRecord(ev_panel, h->stream));  // A0 formed, W0 and dinv allocated
    HIP_TRY(hipStreamWaitEvent(inv.s, ev_panel, 0));
    HIP_TRY(hipStreamWaitEvent(bulk.s, ev_panel, 0));
    HIP_TRY(hipEventRecord(ev_rest, bulk.s));
    launch_tiles_identity(inv.s, h->W0, T0);
    // the diagonal factor of step k + 1 runs in the same launch as step k's
    // update of column k + 1 (launch_dense_next_potrf)
    launch_dense_potrf_diag(h->stream, A0t, T0, 0, dinv, cstat);
    for (int k = 0; k < T0; ++k) {
      launch_dense_trsm_panel(h->stream, A0t, T0, k, dinv);
      HIP_TRY(hipEventRecord(ev_panel, h->stream));
      HIP_TRY(hipStreamWaitEvent(inv.s, ev_panel, 0));
      launch_dense_inv_row(inv.s, h->W0, T0, k, dinv);
      launch_dense_inv_update(inv.s, A0t, h->W0, T0, k);
      HIP_TRY(hipStreamWaitEvent(h->stream, ev_rest, 0));  // rest of step k-1
      launch_dense_next_potrf(h->stream, A0t, T0, k, dinv, cstat);
      HIP_TRY(hipStreamWaitEvent(bulk.s, ev_panel, 0));
      launch_dense_syrk_rest(bulk.s, A0t, T0, k);
      HIP_TRY(hipEventRecord(ev_rest, bulk.s));
    }
    HIP_TRY(hipEventRecord(ev_inv, inv.s));
    HIP_TRY(hipStreamWaitEvent(h->stream, ev_inv, 0));
    HIP_TRY(hipStreamWaitEvent(h->stream, ev_rest, 0));
    HIP_TRY(hipGetLastError());
    int cs = 0;
    HIP_TRY(hipMemcpyAsync(&cs, cstat, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (cs) {
      h->err = "coarse matrix A0 not SPD";
      return AMSP_ERR_COARSE_NOT_SPD;
    }
    h->mem.free_one(W);
    h->mem.free_one(A0t);
    h->mem.free_one(dinv);
    if (mixed) {
      ALLOC(h->W0f, float, (size_t)T0 * T0 * TE);
      launch_dense_tiles_to_f32(h->stream, h->W0, h->W0f, T0);
      deferred.push_back(h->W0);
      h->W0 = nullptr;
    }
    h->sinfo.phase_ms[6] = now_ms() - t5;
    h->sinfo.coarse_factor_mb = (double)T0 * (T0 + 1) / 2 * TE * (mixed ? 4 : 8) * 1e-6;
  }
  double t6 = now_ms();
  h->sinfo.phase_ms[5] = (t6 - t4) - h->sinfo.phase_ms[6];

  // --- the apply's local factors: packed diagonal tiles + envelope
  {
    const size_t ndiag = (size_t)h->ntilerows * DE, nenv = (size_t)P.nenv;
    const double *dsrc = h->fac64 + (size_t)P.noff * TE;
    if (mixed) {
      ALLOC(h->fst32, float, (size_t)h->nst_f + STREAM_TAIL);
      ALLOC(h->bst32, float, (size_t)h->nst_b + STREAM_TAIL);
      launch_stream_from_tiles(h->stream, p, h->ntilerows, h->fac64, h->fst32, h->bst32);
    } else {
      ALLOC(h->dg64, double, ndiag);
      ALLOC(h->erow64, double, nenv);
      ALLOC(h->ecol64, double, nenv);
      HIP_TRY(hipMemcpyAsync(h->dg64, dsrc, ndiag * sizeof(double), hipMemcpyDeviceToDevice,
                             h->stream));
      launch_env_from_tiles<double>(h->stream, p, h->ntilerows, h->fac64, h->erow64, h->ecol64);
    }
    HIP_TRY(hipGetLastError());
    deferred.push_back(h->fac64);
    h->fac64 = nullptr;
  }
  if (mixed) {
    if (h->nev > 0) {
      const bool bf = h->opt.precision == AMSP_MIXED_BF16;
      if (bf) {
        __hip_bfloat16 *pl;
        ALLOC(pl, __hip_bfloat16, (size_t)sum_ni * h->nev);
        h->phi_lo = pl;
      } else {
        float *pl;
        ALLOC(pl, float, (size_t)sum_ni * h->nev);
        h->phi_lo = pl;
      }
      launch_basis_convert(h->stream, h->phi64, h->phi_lo, (size_t)sum_ni * h->nev, bf ? 1 : 0);
    }
  }
  // each region's dofs in ascending order (rows of the ascending-index
  // layout) and their local indices
  {
    int *asc = nullptr, *lop = nullptr;
    ALLOC(asc, int, std::max<long long>(sum_ni, 1));
    ALLOC(lop, int, std::max<long long>(sum_ni, 1));
    launch_ascending_dofs(h->stream, p, asc, lop);
    p.asc = asc;
    p.lop = lop;
    HIP_TRY(hipGetLastError());
  }
  // direct operand indices of the inverse map for the scatter
  {
    const int ne = sum_ni;
    ALLOC(h->inv_x, int, ne);
    launch_inverse_direct(h->stream, ne, h->inv_sd, h->inv_loc, p, h->inv_x);
    HIP_TRY(hipGetLastError());
  }
  // the single-vector apply's copy of the basis: ascending-global-index
  // layout, one column after the other in each region
  if (h->nev > 0) {
    const size_t cnt = (size_t)sum_ni * h->nev;
    if (!mixed) {
      double *pn;
      ALLOC(pn, double, cnt);
      launch_basis_to_natural<double>(h->stream, p, h->phi64, pn);
      h->phi_nat = pn;
    } else if (h->opt.precision == AMSP_MIXED_BF16) {
      __hip_bfloat16 *pn;
      ALLOC(pn, __hip_bfloat16, cnt);
      launch_basis_to_natural<__hip_bfloat16>(h->stream, p, (const __hip_bfloat16 *)h->phi_lo, pn);
      h->phi_nat = pn;
    } else {
      float *pn;
      ALLOC(pn, float, cnt);
      launch_basis_to_natural<float>(h->stream, p, (const float *)h->phi_lo, pn);
      h->phi_nat = pn;
    }
  }
  // --- apply / PCG scratch
  ALLOC(h->xloc, double, sum_npad);
  const int ncp = std::max(1, T0 * TS);
  ALLOC(h->cvec, double, ncp);
  ALLOC(h->t1, double, ncp);
  ALLOC(h->tvec, double, ncp);
  HIP_TRY(hipMemsetAsync(h->cvec, 0, ncp * sizeof(double), h->stream));
  HIP_TRY(hipMemsetAsync(h->t1, 0, ncp * sizeof(double), h->stream));
  HIP_TRY(hipMemsetAsync(h->tvec, 0, ncp * sizeof(double), h->stream));
  ALLOC(h->trmv_part, double, h->tree ? 1 : (size_t)std::max(1, T0 * T0) * TS);
  ALLOC(h->r, double, h->n);
  if (h->opt.cycle == 1) {
    ALLOC(h->mq, double, h->n);
    ALLOC(h->mt, double, h->n);
    ALLOC(h->mc, double, h->n);
    HIP_TRY(hipMemcpyAsync(&h->max_mult, h->max_mult_dev, sizeof(int), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->max_mult = std::max(h->max_mult, 1);
    h->omega = h->opt.smoother_weight > 0.0 ? h->opt.smoother_weight : 1.0 / h->max_mult;
  }
  ALLOC(h->z, double, h->n);
  ALLOC(h->p0, double, h->n);
  ALLOC(h->p1, double, h->n);
  ALLOC(h->q, double, h->n);
  ALLOC(h->part_a, double, MAX_PARTIALS);
  ALLOC(h->part_b, double, MAX_PARTIALS);
  ALLOC(h->part_c, double, MAX_PARTIALS);
  ALLOC(h->part_d, double, MAX_PARTIALS);
  ALLOC(h->scal, double, 8);
  ALLOC(h->st, PcgState, 1);
  HIP_TRY(hipStreamSynchronize(h->stream));
  stage_release(h);
  h->mem.free_one(status);
  for (void *b : deferred) h->mem.free_one(b);
  h->sinfo.phase_ms[7] = now_ms() - t0 + host_plan_ms;
  if (h->sinfo.eig_unconverged > 0) {
    h->err = std::to_string(h->sinfo.eig_unconverged) + " subdomain eigensolves did not converge";
  }
  return AMSP_OK;
}

static bool upload_coupling(amsp_handle *h, hipStream_t stream, CouplingDev &d) {
  const HostPlan &P = h->hp;
  bool ok = true;
  if (h->nc > 0) {
    d.ext_ptr = upload_on(h, stream, P.ext_ptr, ok);
    d.ext_rowptr = upload_on(h, stream, P.ext_rowptr, ok);
    d.ext_src = upload_on(h, stream, P.ext_src, ok);
    d.ext_loc = upload_on(h, stream, P.ext_loc, ok);
    d.npairs = (int)P.pair_i.size();
    d.pair_i = upload_on(h, stream, P.pair_i, ok);
    d.pair_j = upload_on(h, stream, P.pair_j, ok);
    d.pair_ptr = upload_on(h, stream, P.pair_ptr, ok);
    d.pair_l = upload_on(h, stream, P.pair_l, ok);
    d.pair_e = upload_on(h, stream, P.pair_e, ok);
  }
  return ok;
}

// ----------------------------------------- allocation-free block apply ----
// Workspace of amsp_apply_noalloc: one array per device, held until the
// process ends and shared by every handle on that device.  Host code never
// uses the array's name as an address: the device address of each device's
// copy is taken once (hipGetSymbolAddress, with that device current) by the
// first amsp_setup on the device, and only that address reaches kernels.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

// Takes the device address of this device's scratch array (once per device);
// the current device is `device`.
static amsp_status scratch_init(int device, std::string &msg) {
  if (device < 0 || device >= kMaxDevices) {
    msg = "device index beyond the library's limit of " + std::to_string(kMaxDevices);
    return AMSP_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return AMSP_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    msg = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return AMSP_ERR_HIP;
  }
  g_scratch_dev[device] = ptr;
  return AMSP_OK;
}

extern "C" amsp_status amsp_setup(const amsp_csr *A, const int32_t *partition, int32_t nparts,
                                  int32_t nev, const amsp_options *opt, amsp_handle **out) {
  if (!out) return AMSP_ERR_ARG;
  *out = nullptr;
  amsp_options o;
  amsp_default_options(&o);
  if (opt) o = *opt;
  if (o.eig_maxit < 1) o.eig_maxit = 1;
  if (o.chunk < 1) o.chunk = 1;
  if (o.timing_stride < 1) o.timing_stride = 1;
  if (!(o.eig_shift > 0.0)) {
    g_setup_error = "eig_shift must be positive";
    return AMSP_ERR_ARG;
  }
  if (o.coarse_solver < 0 || o.coarse_solver > 2) {
    g_setup_error = "coarse_solver must be 0, 1 or 2";
    return AMSP_ERR_ARG;
  }
  if (o.coarse_basis < 0 || o.coarse_basis > 1) {
    g_setup_error = "coarse_basis must be 0 or 1";
    return AMSP_ERR_ARG;
  }
  if (o.cycle < 0 || o.cycle > 1 || !(o.smoother_weight >= 0.0) || !std::isfinite(o.smoother_weight)) {
    g_setup_error = "cycle must be 0 or 1 and smoother_weight finite and >= 0";
    return AMSP_ERR_ARG;
  }
  std::string msg;
  int64_t offdiag_zeros = -1;
  int s = validate_inputs(A, partition, nparts, nev, o.overlap, msg, &offdiag_zeros);
  if (s != AMSP_OK) {
    g_setup_error = msg;
    return (amsp_status)s;
  }
  amsp_handle *h = new (std::nothrow) amsp_handle();
  if (!h) return AMSP_ERR_OOM;
  h->hp.offdiag_zeros = offdiag_zeros != 0;
  h->opt = o;
  if (h->opt.flexible < 0) h->opt.flexible = (o.precision != AMSP_FP64) ? 1 : 0;
  h->stream = (hipStream_t)o.stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    g_setup_error = "hipGetDevice failed";
    delete h;
    return AMSP_ERR_HIP;
  }
  h->n = (int)A->n;
  h->nnz = A->nnz;
  h->N = nparts;
  h->nev = nev;
  double t0 = now_ms();
  try {
    s = build_plan_local(A, partition, nparts, nev, o, h->hp, msg);
  } catch (const std::bad_alloc &) {
    s = AMSP_ERR_OOM;
    msg = "host allocation failed during planning";
  }
  if (s != AMSP_OK) {
    g_setup_error = msg;
    delete h;
    return (amsp_status)s;
  }
  // the local apply keeps a region's vector and envelope segment starts in
  // LDS (160 KB per workgroup, less the kernel's 512 B of static LDS)
  if ((o.precision == AMSP_FP64 ? local_apply_lds_bytes(h->hp.max_npad, 8)
                                 : local_apply_stream_lds_bytes(h->hp.max_npad)) >
      160 * 1024 - 512) {
    g_setup_error = "largest region (" + std::to_string(h->hp.max_npad) +
                    " padded rows) exceeds the local apply's LDS capacity";
    delete h;
    return AMSP_ERR_ARG;
  }
  h->nc = h->hp.nc;
  h->T0 = (h->nc + TS - 1) / TS;
  h->tree = !o.singular && (o.coarse_solver == 2 || (o.coarse_solver == 0 && h->nc > 8192));
  h->sinfo.coarse_solver = h->tree ? 2 : 1;
  h->sinfo.phase_ms[0] = now_ms() - t0;
  h->sinfo.nsub = h->N;
  h->sinfo.nc = h->nc;
  h->sinfo.sum_ni = h->hp.sd_ptr.back();
  h->sinfo.max_ni = h->hp.max_ni;
  h->sinfo.factor_tiles = h->hp.ntiles;
  amsp_status ds = scratch_init(h->device, h->err);
  if (ds != AMSP_OK) {
    g_setup_error = h->err;
    delete h;
    return ds;
  }
  try {
    ds = device_setup(h, A);
  } catch (const std::bad_alloc &) {
    ds = AMSP_ERR_OOM;
    h->err = "host allocation failed during setup";
  }
  if (ds != AMSP_OK) {
    g_setup_error = h->err;
    delete h;
    return ds;
  }
  *out = h;
  return AMSP_OK;
}

// ------------------------------------------------------------- apply ------
static amsp_status apply_one(amsp_handle *h, const double *r, double *z, int parts,
                             double *partial_rz, const int *done) {
  const Plan &p = h->plan;
  const int do_local = (parts & 1) ? 1 : 0;
  const int do_coarse = ((parts & 2) && h->nc > 0) ? 1 : 0;
  const bool mixed = h->opt.precision != AMSP_FP64;
  const bool bf = h->opt.precision == AMSP_MIXED_BF16;
  if (!do_local && !do_coarse) {  // coarse part asked for, but no coarse space
    launch_fill(h->stream, h->n, z, 0.0);
    if (partial_rz) launch_fill(h->stream, reduce_blocks(h->n), partial_rz, 0.0);
    HIP_TRY(hipGetLastError());
    return AMSP_OK;
  }
  // Coarse part first (restriction, then the coarse solve), so that the
  // local apply adds the prolongation Phi_i t_i to each region's output as
  // it stores it; without the local part the prolongation runs before the
  // scatter instead.
  int tk;
  if (do_coarse) {
    tk = tstart(h, 2);
    if (!mixed)
      launch_restrict<double>(h->stream, p, r, (const double *)h->phi_nat, h->cvec, done);
    else if (!bf)
      launch_restrict<float>(h->stream, p, r, (const float *)h->phi_nat, h->cvec, done);
    else
      launch_restrict<__hip_bfloat16>(h->stream, p, r, (const __hip_bfloat16 *)h->phi_nat,
                                      h->cvec, done);
    // with the local part, the second dense product leaves its per-tile
    // products, which the local apply sums for its own coarse values
    double *t2 = do_local ? nullptr : h->tvec;
    if (h->tree) {
      coarse_solve_tree(h, h->stream, h->cvec, h->tvec, done);
    } else if (!mixed) {
      launch_trmv<double>(h->stream, h->W0, h->T0, h->cvec, h->trmv_part, h->t1, 0, done);
      launch_trmv<double>(h->stream, h->W0, h->T0, h->t1, h->trmv_part, t2, 1, done);
    } else {
      launch_trmv<float>(h->stream, h->W0f, h->T0, h->cvec, h->trmv_part, h->t1, 0, done);
      launch_trmv<float>(h->stream, h->W0f, h->T0, h->t1, h->trmv_part, t2, 1, done);
    }
    tstop(h, 2, tk);
  }
  if (do_local) {
    const bool parts = do_coarse && !h->tree;
    const double *t = do_coarse && h->tree ? h->tvec : nullptr;
    const double *tpart = parts ? h->trmv_part : nullptr;
    hipEvent_t e0, e1;
    tk = tpair(h, 1, &e0, &e1);
    if (!mixed)
      launch_local_apply_t<double, double, double>(h->stream, p, h->hp.max_npad, r, h->dg64,
                                                   h->erow64, h->ecol64,
                                                   (const double *)h->phi_nat, t, tpart, h->T0,
                                                   h->xloc, done, e0, e1);
    else if (!bf)
      launch_local_apply_stream<float>(h->stream, p, h->hp.max_npad, r, h->fst32, h->bst32,
                                       (const float *)h->phi_nat, t, tpart, h->T0, h->xloc, done,
                                       e0, e1);
    else
      launch_local_apply_stream<__hip_bfloat16>(h->stream, p, h->hp.max_npad, r, h->fst32,
                                                h->bst32, (const __hip_bfloat16 *)h->phi_nat, t,
                                                tpart, h->T0, h->xloc, done, e0, e1);
    tpair_done(h, 1, tk);
  }
  tk = tstart(h, 3);
  const int mni = h->hp.max_ni;
  const int prolong = do_coarse && !do_local;
  if (!mixed || h->nev == 0)
    launch_scatter_sum_t<double>(h->stream, p, mni, h->n, h->inv_ptr, h->inv_x, h->xloc,
                                 (const double *)h->phi_nat, h->tvec, z,
                                 partial_rz ? r : nullptr, partial_rz, do_local, prolong, done);
  else if (!bf)
    launch_scatter_sum_t<float>(h->stream, p, mni, h->n, h->inv_ptr, h->inv_x, h->xloc,
                                (const float *)h->phi_nat, h->tvec, z, partial_rz ? r : nullptr,
                                partial_rz, do_local, prolong, done);
  else
    launch_scatter_sum_t<__hip_bfloat16>(h->stream, p, mni, h->n, h->inv_ptr, h->inv_x, h->xloc,
                                         (const __hip_bfloat16 *)h->phi_nat, h->tvec, z,
                                         partial_rz ? r : nullptr, partial_rz, do_local, prolong,
                                         done);
  tstop(h, 3, tk);
  HIP_TRY(hipGetLastError());
  return AMSP_OK;
}

// z_k = M^{-1} r_k (parts as in apply_one) for nr <= EIGP columns, n apart,
// with one pass over the local factor: the block solve with the Dirichlet
// factor (f32-stored in the mixed forms, f64 arithmetic), the restriction of
// all columns, one coarse solve per column, the prolongation and the scatter.
// Workspace of the block apply: gathered, solved and output blocks (rows x
// EIGP each), the coarse vectors (ncp x EIGP each) and the coarse products'
// partial sums (T0^2 x TS x EIGP).
struct BlockWs {
  double *X, *Y, *XN, *C, *T, *C2, *Part;
  bool clear_c;  // the coarse input's padding must be zeroed by this call
};

static size_t block_ws_doubles(const amsp_handle *h) {
  const size_t rows = (size_t)h->hp.vp_ptr.back();
  const size_t ncp = (size_t)std::max(1, h->T0 * TS);
  return 3 * rows * EIGP + 3 * ncp * EIGP +
         (h->tree ? 1 : std::max<size_t>((size_t)h->T0 * h->T0, 1) * TS * EIGP);
}

// Carves the workspace out of one buffer of block_ws_doubles(h) doubles.
static BlockWs block_ws_from(const amsp_handle *h, double *base) {
  const size_t rows = (size_t)h->hp.vp_ptr.back();
  const size_t ncp = (size_t)std::max(1, h->T0 * TS);
  BlockWs w;
  w.X = base;
  w.Y = w.X + rows * EIGP;
  w.XN = w.Y + rows * EIGP;
  w.C = w.XN + rows * EIGP;
  w.T = w.C + ncp * EIGP;
  w.C2 = w.T + ncp * EIGP;
  w.Part = w.C2 + ncp * EIGP;
  w.clear_c = true;
  return w;
}

static amsp_status apply_block_ws(amsp_handle *h, const double *r, double *z, int nr, int parts,
                                  const BlockWs &ws);

static amsp_status apply_block(amsp_handle *h, const double *r, double *z, int nr, int parts) {
  const size_t rows = (size_t)h->hp.vp_ptr.back();
  const size_t ncp = (size_t)std::max(1, h->T0 * TS);
  if (!h->bX) {
    ALLOC(h->bX, double, rows * EIGP);
    ALLOC(h->bY, double, rows * EIGP);
    ALLOC(h->bXN, double, rows * EIGP);
    ALLOC(h->bC, double, ncp * EIGP);
    ALLOC(h->bT, double, ncp * EIGP);
    ALLOC(h->bC2, double, ncp * EIGP);
    ALLOC(h->bPart, double,
          h->tree ? 1 : std::max<size_t>((size_t)h->T0 * h->T0, 1) * TS * EIGP);
    launch_fill(h->stream, ncp * EIGP, h->bC, 0.0);  // coarse padding stays zero
  }
  const BlockWs ws{h->bX, h->bY, h->bXN, h->bC, h->bT, h->bC2, h->bPart, false};
  return apply_block_ws(h, r, z, nr, parts, ws);
}

static amsp_status apply_block_ws(amsp_handle *h, const double *r, double *z, int nr, int parts,
                                  const BlockWs &ws) {
  const Plan &p = h->plan;
  const int n = h->n;
  hipStream_t s = h->stream;
  const bool mixed = h->opt.precision != AMSP_FP64;
  const bool bf = h->opt.precision == AMSP_MIXED_BF16;
  const int do_local = (parts & 1) ? 1 : 0;
  const int do_coarse = ((parts & 2) && h->nc > 0) ? 1 : 0;
  const size_t ncp = (size_t)std::max(1, h->T0 * TS);
  double *const bX = ws.X, *const bY = ws.Y, *const bXN = ws.XN, *const bC = ws.C,
               *const bT = ws.T, *const bC2 = ws.C2, *const bPart = ws.Part;
  if (do_coarse && ws.clear_c) launch_fill(s, ncp * nr, bC, 0.0);  // padding rows read as zero
  if (mixed && do_local && !h->dg32) {
    const size_t nenv = (size_t)h->hp.nenv;
    ALLOC(h->dg32, float, (size_t)h->ntilerows * DE);
    ALLOC(h->er32, float, std::max<size_t>(nenv, 1));
    ALLOC(h->ec32, float, std::max<size_t>(nenv, 1));
    launch_streams_to_env(s, p, h->ntilerows, h->fst32, h->bst32, h->dg32, h->er32, h->ec32);
  }
  launch_gather_multi(s, p, n, nr, r, bX);
  if (do_local) {
    if (mixed)
      launch_env_solve_block<float>(s, p, h->dg32, h->er32, h->ec32, bX, bY, nullptr);
    else
      launch_env_solve_block<double>(s, p, h->dg64, h->erow64, h->ecol64, bX, bY, nullptr);
  }
  const void *phi = mixed ? h->phi_lo : (const void *)h->phi64;
  if (do_coarse) {
    if (!mixed)
      launch_restrict_multi<double>(s, p, nr, ncp, (const double *)phi, bX, bC);
    else if (!bf)
      launch_restrict_multi<float>(s, p, nr, ncp, (const float *)phi, bX, bC);
    else
      launch_restrict_multi<__hip_bfloat16>(s, p, nr, ncp, (const __hip_bfloat16 *)phi, bX, bC);
    // t_k = W0^T (W0 c_k) for all columns, W0's tiles read once per product
    if (h->tree) {
      for (int k = 0; k < nr; ++k) coarse_solve_tree(h, s, bC + k * ncp, bT + k * ncp, nullptr);
    } else if (!mixed) {
      launch_trmm<double>(s, h->W0, h->T0, bC, ncp, nr, bPart, bC2, 0);
      launch_trmm<double>(s, h->W0, h->T0, bC2, ncp, nr, bPart, bT, 1);
    } else {
      launch_trmm<float>(s, h->W0f, h->T0, bC, ncp, nr, bPart, bC2, 0);
      launch_trmm<float>(s, h->W0f, h->T0, bC2, ncp, nr, bPart, bT, 1);
    }
  }
  const double *tcoarse = do_coarse ? bT : nullptr;
  const double *ylocal = do_local ? bY : nullptr;
  if (!mixed)
    launch_prolong_multi<double>(s, p, nr, ncp, (const double *)phi, tcoarse, ylocal, bXN);
  else if (!bf)
    launch_prolong_multi<float>(s, p, nr, ncp, (const float *)phi, tcoarse, ylocal, bXN);
  else
    launch_prolong_multi<__hip_bfloat16>(s, p, nr, ncp, (const __hip_bfloat16 *)phi, tcoarse,
                                         ylocal, bXN);
  launch_scatter_multi(s, n, nr, h->inv_ptr, h->inv_x, bXN, z);
  HIP_TRY(hipGetLastError());
  return AMSP_OK;
}

// z = M^{-1} r with the handle's cycle: the additive operator, or one
// symmetric two-grid cycle x1 = w S r, x2 = x1 + C (r - A x1),
// z = x2 + w S (r - A x2) from the same local-solve and coarse kernels.
static amsp_status apply_prec(amsp_handle *h, const double *r, double *z, double *partial_rz,
                              const int *done) {
  if (h->opt.cycle != 1) return apply_one(h, r, z, 3, partial_rz, done);
  const int n = h->n;
  hipStream_t s = h->stream;
  amsp_status st = apply_one(h, r, z, 1, nullptr, done);
  if (st != AMSP_OK) return st;
  launch_scale_done(s, n, h->omega, z, done);
  launch_spmv_sell(s, n, h->sptr, h->scol, h->sval, z, h->mq, done);
  launch_sub_done(s, n, r, h->mq, h->mt, done);
  if ((st = apply_one(h, h->mt, h->mc, 2, nullptr, done)) != AMSP_OK) return st;
  launch_axpy_dot(s, n, 1.0, h->mc, z, nullptr, nullptr, done);
  launch_spmv_sell(s, n, h->sptr, h->scol, h->sval, z, h->mq, done);
  launch_sub_done(s, n, r, h->mq, h->mt, done);
  if ((st = apply_one(h, h->mt, h->mc, 1, nullptr, done)) != AMSP_OK) return st;
  launch_axpy_dot(s, n, h->omega, h->mc, z, partial_rz ? r : nullptr, partial_rz, done);
  HIP_TRY(hipGetLastError());
  return AMSP_OK;
}

extern "C" amsp_status amsp_apply_parts(amsp_handle *h, const double *r_dev, double *z_dev,
                                        int32_t nrhs, int32_t parts) {
  if (!h || !r_dev || !z_dev || nrhs < 1 || parts < 1 || parts > 3) return AMSP_ERR_ARG;
  for (int k = 0; k < nrhs; ++k) {
    const double *rk = r_dev + (size_t)k * h->n;
    double *zk = z_dev + (size_t)k * h->n;
    // two or more columns: EIGP at a time through the block solve (the
    // multiplicative cycle keeps the column-by-column path)
    if (nrhs - k >= 2 && !(h->opt.cycle == 1 && parts == 3)) {
      const int nr = std::min(EIGP, nrhs - k);
      amsp_status s = apply_block(h, rk, zk, nr, parts);
      if (s != AMSP_OK) return s;
      k += nr - 1;
      continue;
    }
    amsp_status s = parts == 3 ? apply_prec(h, rk, zk, nullptr, nullptr)
                               : apply_one(h, rk, zk, parts, nullptr, nullptr);
    if (s != AMSP_OK) return s;
  }
  return AMSP_OK;
}

extern "C" amsp_status amsp_apply_noalloc(amsp_handle *h, const double *r_dev, double *z_dev,
                                         int32_t nrhs, int32_t parts) {
  if (!h || !r_dev || !z_dev || nrhs < 1 || parts < 1 || parts > 3) return AMSP_ERR_ARG;
  if (h->opt.cycle == 1 && parts == 3) {
    h->err = "amsp_apply_noalloc: the multiplicative cycle is not available here";
    return AMSP_ERR_ARG;
  }
  if (h->opt.precision != AMSP_FP64 && (parts & 1) && !h->dg32) {
    h->err = "amsp_apply_noalloc: the mixed forms' block solve reads a float32 copy of the local "
             "factor that the first amsp_apply with nrhs >= 2 builds; call that once first";
    return AMSP_ERR_ARG;
  }
  const size_t need = block_ws_doubles(h) * sizeof(double);
  if (need > kNoallocScratchBytes) {
    h->err = "amsp_apply_noalloc: workspace of " + std::to_string(need) + " bytes exceeds the " +
             std::to_string(kNoallocScratchBytes) + "-byte scratch array";
    return AMSP_ERR_ARG;
  }
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = (h->device >= 0 && h->device < kMaxDevices) ? g_scratch_dev[h->device] : nullptr;
  }
  if (!base) {
    h->err = "amsp_apply_noalloc: no scratch address for the handle's device";
    return AMSP_ERR_HIP;
  }
  const BlockWs ws = block_ws_from(h, static_cast<double *>(base));
  for (int k = 0; k < nrhs; k += EIGP) {
    const int nr = std::min(EIGP, nrhs - k);
    amsp_status st = apply_block_ws(h, r_dev + (size_t)k * h->n, z_dev + (size_t)k * h->n, nr,
                                    parts, ws);
    if (st != AMSP_OK) return st;
  }
  return AMSP_OK;
}

extern "C" amsp_status amsp_apply(amsp_handle *h, const double *r_dev, double *z_dev, int32_t nrhs) {
  return amsp_apply_parts(h, r_dev, z_dev, nrhs, 3);
}

extern "C" amsp_status amsp_spmv(amsp_handle *h, const double *x_dev, double *y_dev) {
  if (!h || !x_dev || !y_dev) return AMSP_ERR_ARG;
  launch_spmv_sell(h->stream, h->n, h->sptr, h->scol, h->sval, x_dev, y_dev);
  HIP_TRY(hipGetLastError());
  return AMSP_OK;
}

extern "C" amsp_status amsp_grad_values(amsp_handle *h, const double *lambda_dev,
                                        const double *u_dev, double *grad_dev) {
  if (!h || !lambda_dev || !u_dev || !grad_dev) return AMSP_ERR_ARG;
  launch_grad_values(h->stream, h->n, h->rowptr, h->col, lambda_dev, u_dev, grad_dev);
  HIP_TRY(hipGetLastError());
  return AMSP_OK;
}

// Entries of the apply's local factors: one packed diagonal tile per tile
// row and the envelope (each sweep reads the diagonal tiles and one form).
static int64_t apply_factor_elems(const HostPlan &P) {
  return (int64_t)P.trow_ptr.back() * DE + P.nenv;
}

// Algorithmic bytes of one local-apply launch: gather of r and the region
// index, envelope segment starts, both factor sweeps, basis and coarse
// solution (or the partials it is summed from) read for the prolongation,
// local output.
static int64_t local_apply_bytes(const amsp_handle *h) {
  const HostPlan &P = h->hp;
  const bool mixed = h->opt.precision != AMSP_FP64;
  const int64_t sni = P.sd_ptr.back(), snp = P.vp_ptr.back();
  const int64_t fb = mixed ? 4 : 8;
  const int64_t pb = mixed ? (h->opt.precision == AMSP_MIXED_BF16 ? 2 : 4) : 8;
  // the mixed forms stream the factor (diagonal tiles, envelope and block
  // padding) once per sweep; the FP64 form reads diagonal tiles and envelope
  const int64_t fac = mixed ? (int64_t)(h->nst_f + h->nst_b) * fb : 2 * apply_factor_elems(P) * fb;
  int64_t b = sni * (8 + 4) + sni * 8 + 2 * (snp + h->N) * 4 + fac;
  if (h->nc > 0) {
    b += sni * h->nev * pb;  // basis rows for the prolongation
    if (h->tree) {
      b += (int64_t)h->nc * 8;  // the coarse solution
    } else {  // the second coarse product's per-tile partials, summed here
      for (int64_t g = 0; g < h->nc; ++g) b += (int64_t)(h->T0 - g / TS) * 8;
    }
  }
  return b;
}

static int64_t bytes_per_iter(const amsp_handle *h) {
  const HostPlan &P = h->hp;
  const bool mixed = h->opt.precision != AMSP_FP64;
  const int64_t n = h->n, nnz = h->nnz, sni = P.sd_ptr.back(), snp = P.vp_ptr.back();
  const int64_t fb = mixed ? 4 : 8;
  const int64_t pb = mixed ? (h->opt.precision == AMSP_MIXED_BF16 ? 2 : 4) : 8;
  int64_t b = 0;
  b += nnz * 12 + (n + 1) * 4 + n * 8 * 4;          // spmv with the fused p update
  b += n * 8 * 6;                                   // x, r update
  b += sni * (8 + 4) + sni * 8 + 2 * (snp + h->N) * 4;  // local gather, write, segments
  b += mixed ? (int64_t)(h->nst_f + h->nst_b) * fb      // forward + backward factor sweep
             : 2 * apply_factor_elems(P) * fb;
  if (h->nc > 0) {
    b += sni * h->nev * pb * 2;                     // restrict + prolong basis reads
    b += h->tree ? 2 * (int64_t)h->tp.xtiles * TE * (mixed ? 4 : 8)        // fronts' X twice
                 : 2 * (int64_t)h->T0 * (h->T0 + 1) / 2 * TE * (mixed ? 4 : 8);  // W0 twice
  }
  b += sni * (8 + 8) + n * 8 * 3;                   // scatter: inverse map, locals, z, r
  if (h->opt.flexible) b += n * 8;
  return b;
}

// PCG on nr <= EIGP columns at once: one CG recurrence per column (the same
// steps and stopping rule as amsp_pcg), all sharing each SpMV (entries read
// once) and each preconditioner application (the block path of amsp_apply).
// Scalars go through the host twice per step.  Converged columns keep
// alpha = beta = 0.  Adds to the totals in *inf; the history of the last
// column is kept for amsp_get_pcg_history.
static amsp_status pcg_columns(amsp_handle *h, const double *F, double *U, int nr, double rtol,
                               int maxit, amsp_info &inf) {
  const int n = h->n;
  const size_t ld = (size_t)n, tot = ld * nr;
  hipStream_t s = h->stream;
  double *R = nullptr, *Z = nullptr, *Pd = nullptr, *Q = nullptr, *part = nullptr, *sc = nullptr;
  ALLOC(R, double, tot);
  ALLOC(Z, double, tot);
  ALLOC(Pd, double, tot);
  ALLOC(Q, double, tot);
  ALLOC(part, double, (size_t)256 * EIGP);
  ALLOC(sc, double, 4 * EIGP);  // [0,16) alpha/beta, [16,32) dots, [32,48) rr
  auto release = [&]() {
    for (double *b : {R, Z, Pd, Q, part, sc}) h->mem.free_one(b);
  };
  auto to_host = [&](const double *src, double *dst) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dst, src, nr * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  };
  std::vector<double> f2(nr), rr(nr);
  std::vector<int> active(nr), its(nr, 0);
  std::vector<double> hist;
  launch_fill(s, tot, U, 0.0);
  HIP_TRY(hipMemcpyAsync(R, F, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_col_dots(s, n, ld, nr, F, F, part, sc + 16);
  HIP_TRY(to_host(sc + 16, f2.data()));
  for (int k = 0; k < nr; ++k) {
    if (!std::isfinite(f2[k])) {
      release();
      h->err = "right-hand side not finite";
      return AMSP_ERR_BREAKDOWN;
    }
    rr[k] = f2[k];
    active[k] = f2[k] > 0.0;
  }
  hist.push_back(f2[nr - 1]);
  int broken = 0;  // bit k: column k broke down
  int it = 0;
  auto any_active = [&]() {
    for (int v : active)
      if (v) return true;
    return false;
  };
  std::vector<double> rt(nr, 0.0), fl(nr, 0.0), rec(nr, 0.0);
  const int nb = reduce_blocks(n);
  amsp_status st = AMSP_OK;
  // as in amsp_pcg: stop on the recursive residuals, recompute f - A u, and
  // restart the columns whose true residual is above max(rtol, floor) from
  // it (at most 3 times)
  // The per-column scalars stay on the device (ColCgState).  Behind every
  // step the state is copied to a pinned slot, and the host reads step t's
  // copy while step t + 1 runs; once no column is active the step already
  // enqueued changes nothing (all its coefficients are zero).
  ColCgState *cs = nullptr, *cs_host = nullptr;
  ALLOC(cs, ColCgState, 1);
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&cs_host), 2 * sizeof(ColCgState),
                        hipHostMallocDefault));
  hipEvent_t cev[2] = {nullptr, nullptr};
  struct Guard {
    ColCgState *p;
    hipEvent_t *e;
    ~Guard() {
      for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
      if (p) (void)hipHostFree(p);
    }
  } guard{cs_host, cev};
  for (hipEvent_t &e : cev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  {
    ColCgState init{};
    for (int k = 0; k < nr; ++k) {
      init.f2[k] = f2[k];
      init.rr[k] = rr[k];
    }
    HIP_TRY(hipMemcpyAsync(cs, &init, sizeof(ColCgState), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  const double rtol2 = rtol * rtol;
  for (int restarts = 0;; ++restarts) {
    if ((st = apply_block(h, R, Z, nr, 3)) != AMSP_OK) return st;
    launch_col_dots(s, n, ld, nr, R, Z, part, sc + 16);
    HIP_TRY(hipMemcpyAsync(cs->rz, sc + 16, nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    {
      int act[EIGP] = {0};
      for (int k = 0; k < nr; ++k) act[k] = active[k];
      HIP_TRY(hipMemcpyAsync(cs->active, act, sizeof(act), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(Pd, Z, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
    int pend = -1;  // slot of the state copy in flight
    bool live = any_active();
    while (live && it < maxit) {
      launch_spmm_sell(s, n, h->sptr, h->scol, h->sval, ld, nr, Pd, Q);
      launch_col_dots(s, n, ld, nr, Pd, Q, part, sc + 16);
      launch_col_alpha(s, nr, cs, sc + 16, sc);
      launch_col_update(s, n, ld, nr, sc, Pd, Q, U, R, part, sc + 32);
      if ((st = apply_block(h, R, Z, nr, 3)) != AMSP_OK) return st;
      launch_col_dots(s, n, ld, nr, R, Z, part, sc + 16);
      launch_col_beta(s, nr, cs, sc + 32, sc + 16, rtol2, sc);
      launch_col_direction(s, n, ld, nr, sc, Z, Pd);
      const int slot = pend == 0 ? 1 : 0;
      HIP_TRY(hipMemcpyAsync(cs_host + slot, cs, sizeof(ColCgState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(cev[slot], s));
      HIP_TRY(hipGetLastError());
      ++it;
      if (pend >= 0) {  // the previous step's state, read while this step runs
        HIP_TRY(hipEventSynchronize(cev[pend]));
        hist.push_back(cs_host[pend].rr[nr - 1]);
        if (cs_host[pend].nact == 0) {
          --it;  // this step found no active column
          pend = -1;
          break;
        }
      }
      pend = slot;
    }
    if (pend >= 0) {  // the last step's state
      HIP_TRY(hipEventSynchronize(cev[pend]));
      hist.push_back(cs_host[pend].rr[nr - 1]);
    }
    HIP_TRY(hipStreamSynchronize(s));
    {
      ColCgState fin{};
      HIP_TRY(hipMemcpy(&fin, cs, sizeof(ColCgState), hipMemcpyDeviceToHost));
      for (int k = 0; k < nr; ++k) {
        rr[k] = fin.rr[k];
        its[k] = fin.its[k];
        active[k] = fin.active[k];
      }
      broken |= fin.breakdown;
    }
    for (int k = 0; k < nr; ++k) rec[k] = f2[k] > 0.0 ? std::sqrt(rr[k] / f2[k]) : 0.0;
    // true residuals (left in R) and, where needed, the attainable floors
    launch_spmm_sell(s, n, h->sptr, h->scol, h->sval, ld, nr, U, Q);
    bool again = false;
    for (int k = 0; k < nr; ++k) {
      const double fk = std::sqrt(f2[k]);
      rt[k] = 0.0;
      if (!(fk > 0.0)) continue;
      launch_residual(s, n, F + k * ld, Q + k * ld, R + k * ld, part);
      launch_sum_partials(s, part, nb, sc + 47);
      double r2 = 0.0;
      HIP_TRY(hipMemcpyAsync(&r2, sc + 47, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      rt[k] = std::sqrt(r2) / fk;
      if (rt[k] > rtol && fl[k] == 0.0) {
        launch_abs_spmv_sq(s, n, h->rowptr, h->col, h->val, U + k * ld, part);
        launch_sum_partials(s, part, nb, sc + 47);
        double a2 = 0.0;
        HIP_TRY(hipMemcpyAsync(&a2, sc + 47, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        fl[k] = DBL_EPSILON * std::sqrt(a2) / fk;
      }
      rr[k] = r2;
      const bool ok = rt[k] <= std::max(rtol, fl[k]);
      // a column that broke down stops; the others restart as usual
      active[k] = !ok && std::isfinite(rt[k]) && restarts < 3 && it < maxit && !(broken >> k & 1);
      again = again || active[k];
    }
    if (!again) break;
  }
  for (int k = 0; k < nr; ++k) {
    const bool conv = rt[k] <= std::max(rtol, fl[k]) && std::isfinite(rt[k]);
    if (!conv) inf.converged = 0;
    inf.iterations += its[k];
    inf.first_segment += its[k];  // the block path does not split its segments
    inf.relres_true = std::max(inf.relres_true, rt[k]);
    inf.relres_recursive = std::max(inf.relres_recursive, rec[k]);
    inf.relres_floor = std::max(inf.relres_floor, fl[k]);
  }
  h->hist_len = std::min((int)hist.size(), h->hist_cap);
  h->hist_f2 = f2[nr - 1];
  HIP_TRY(hipMemcpyAsync(h->hist, hist.data(), h->hist_len * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  release();
  h->mem.free_one(cs);
  if (broken) {
    h->err = "CG breakdown in a column (p.Ap <= 0 or a non-finite value)";
    return AMSP_ERR_BREAKDOWN;
  }
  return AMSP_OK;
}

extern "C" amsp_status amsp_pcg(amsp_handle *h, const double *f_dev, double *u_dev, int32_t nrhs,
                                double rtol, int32_t maxit, amsp_info *info) {
  if (!h || !f_dev || !u_dev || nrhs < 1 || maxit < 0 || !(rtol >= 0.0)) return AMSP_ERR_ARG;
  const int n = h->n;
  const int nb = reduce_blocks(n);
  amsp_info inf{};
  inf.bytes_per_iter = bytes_per_iter(h);
  inf.local_apply_bytes = local_apply_bytes(h);
  if (nrhs >= 2 && h->opt.cycle == 0) {  // columns share operator applications
    if (h->hist_cap < maxit + 2) {
      if (h->hist) h->mem.free_one(h->hist);
      h->hist_cap = std::max(maxit + 2, 1024);
      ALLOC(h->hist, double, h->hist_cap);
    }
    const double t0 = now_ms();
    inf.converged = 1;
    bool broke = false;  // a breakdown stops its column only: the others still run
    for (int k0 = 0; k0 < nrhs; k0 += EIGP) {
      const int nr = std::min(EIGP, nrhs - k0);
      amsp_status st = nr >= 2 ? pcg_columns(h, f_dev + (size_t)k0 * n, u_dev + (size_t)k0 * n, nr,
                                             rtol, maxit, inf)
                               : AMSP_OK;
      if (nr == 1) {  // a last single column: the one-column path
        amsp_info one{};
        st = amsp_pcg(h, f_dev + (size_t)k0 * n, u_dev + (size_t)k0 * n, 1, rtol, maxit, &one);
        if (st != AMSP_OK && st != AMSP_ERR_PCG_NOCONV && st != AMSP_ERR_BREAKDOWN) return st;
        inf.iterations += one.iterations;
        inf.first_segment += one.first_segment;
        inf.relres_true = std::max(inf.relres_true, one.relres_true);
        inf.relres_recursive = std::max(inf.relres_recursive, one.relres_recursive);
        inf.relres_floor = std::max(inf.relres_floor, one.relres_floor);
        if (!one.converged) inf.converged = 0;
        if (st != AMSP_ERR_BREAKDOWN) st = AMSP_OK;
      }
      if (st == AMSP_ERR_BREAKDOWN) {
        broke = true;
        inf.converged = 0;
        st = AMSP_OK;
      }
      if (st != AMSP_OK) return st;
    }
    inf.solve_ms = now_ms() - t0;
    if (info) *info = inf;
    if (broke) {
      h->err = "CG breakdown in a column (p.Ap <= 0 or a non-finite value)";
      return AMSP_ERR_BREAKDOWN;
    }
    return inf.converged ? AMSP_OK : AMSP_ERR_PCG_NOCONV;
  }
  h->timing_active = h->opt.timing != 0;
  h->ev_used = 0;
  h->ev_rec.clear();
  h->cur_seg = 0;
  h->cur_t = -1;
  h->seg_cut.clear();
  for (int &c : h->ev_count) c = 0;
  if (h->hist_cap < maxit + 2) {
    if (h->hist) h->mem.free_one(h->hist);
    h->hist_cap = std::max(maxit + 2, 1024);
    ALLOC(h->hist, double, h->hist_cap);
  }
  {
    PcgState init{};
    init.hist = h->hist;
    init.hist_cap = h->hist_cap;
    HIP_TRY(hipMemcpyAsync(h->st, &init, sizeof(PcgState), hipMemcpyHostToDevice, h->stream));
  }
  if (!h->st_host) {
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h->st_host), 2 * sizeof(PcgState),
                          hipHostMallocDefault));
    for (hipEvent_t &e : h->st_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  double t0 = now_ms();
  amsp_status final_status = AMSP_OK;
  int tot_it = 0, tot_first = 0;
  double worst_true = 0.0, worst_rec = 0.0, worst_floor = 0.0;
  int all_conv = 1, tot_restarts = 0;
  PcgState hs{};
  for (int k = 0; k < nrhs; ++k) {
    const double *f = f_dev + (size_t)k * n;
    double *x = u_dev + (size_t)k * n;
    launch_fill(h->stream, n, x, 0.0);
    launch_copy_scale(h->stream, n, f, h->r, 1.0);
    int restarts = 0;
    bool fresh = true;
    double relres_true = 0.0, floor_rel = 0.0;
    for (;;) {
      // z = M^{-1} r with r.z partials; r.r partials; p_old = 0
      h->cur_t = -1;
      launch_dot(h->stream, n, h->r, h->r, h->part_d, nullptr);
      amsp_status s = apply_prec(h, h->r, h->z, h->part_b, nullptr);
      if (s != AMSP_OK) return s;
      launch_fill(h->stream, n, h->p0, 0.0);
      launch_pcg_init(h->stream, h->st, h->part_d, nb, h->part_b, nb, fresh ? rtol : -1.0, maxit);
      HIP_TRY(hipGetLastError());
      const int *done = &h->st->done;
      double *pold = h->p0, *pnew = h->p1;
      int prev_it = 0;
      double prev_rr = -1.0;
      // step index of the next launch (iterations completed before it) and
      // whether it is the first step after this (re)start
      int t = fresh ? 0 : hs.it;
      bool first = true;
      HIP_TRY(hipMemcpyAsync(&hs, h->st, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      // Chunks of steps run back to back.  Behind each chunk the state is
      // copied to a pinned slot; the host reads a chunk's copy while the
      // next chunk runs, so the device does not wait for the host between
      // chunks.  Chunk sizes follow the observed residual decay (minus the
      // steps still in flight), so that few steps are enqueued after
      // convergence; those return at once.
      int pend = -1, pend_steps = 0;  // slot of the copy in flight, steps of its chunk
      while (!hs.done) {
        int next = h->opt.chunk;
        if (prev_rr > 0.0 && hs.it > prev_it && hs.rr < prev_rr && hs.rr > 0.0) {
          const double rate = std::log(hs.rr / prev_rr) / (double)(hs.it - prev_it);
          const double need = std::log(hs.tol2 / hs.rr) / rate;
          // + 1: convergence is seen by the following step
          next = (int)std::ceil(need) + 1 - pend_steps;
          next = std::max(pend >= 0 ? 0 : 1, std::min(next, h->opt.chunk));
        }
        for (int c = 0; c < next; ++c) {
          h->cur_t = t;
          int tk = tstart(h, 0);
          launch_cg_dir(h->stream, n, h->sptr, h->scol, h->sval, h->z, pold, pnew, h->q, h->part_a,
                        h->st, h->part_d, h->part_b, h->part_c, t, first ? 1 : 0,
                        h->opt.flexible);
          tstop(h, 0, tk);
          tk = tstart(h, 4);
          launch_cg_update(h->stream, n, x, h->r, pnew, h->q, h->st, h->part_a, t, h->part_d,
                           h->opt.flexible ? h->z : nullptr, h->part_c);
          tstop(h, 4, tk);
          s = apply_prec(h, h->r, h->z, h->part_b, done);
          if (s != AMSP_OK) return s;
          std::swap(pold, pnew);
          ++t;
          first = false;
        }
        HIP_TRY(hipGetLastError());
        int slot = -1;
        if (next > 0) {
          slot = pend == 0 ? 1 : 0;
          HIP_TRY(hipMemcpyAsync(&h->st_host[slot], h->st, sizeof(PcgState),
                                 hipMemcpyDeviceToHost, h->stream));
          HIP_TRY(hipEventRecord(h->st_ev[slot], h->stream));
        }
        if (pend >= 0) {  // the previous chunk's state, read while this chunk runs
          HIP_TRY(hipEventSynchronize(h->st_ev[pend]));
          prev_rr = hs.rr;
          prev_it = hs.it;
          hs = h->st_host[pend];
        }
        pend = slot;
        pend_steps = slot >= 0 ? next : 0;
      }
      // steps enqueued after convergence were no-ops: hs is the final state
      HIP_TRY(hipStreamSynchronize(h->stream));
      h->seg_cut.push_back(hs.it);  // steps >= hs.it of this segment were no-ops
      ++h->cur_seg;
      h->cur_t = -1;
      // true residual
      launch_spmv(h->stream, n, h->rowptr, h->col, h->val, x, h->q, nullptr, nullptr);
      launch_residual(h->stream, n, f, h->q, h->r, h->part_a);
      launch_sum_partials(h->stream, h->part_a, nb, h->scal);
      launch_abs_spmv_sq(h->stream, n, h->rowptr, h->col, h->val, x, h->part_c);
      launch_sum_partials(h->stream, h->part_c, nb, h->scal + 1);
      double rrt[2] = {0.0, 0.0};
      HIP_TRY(hipMemcpyAsync(rrt, h->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      relres_true = hs.f2 > 0 ? std::sqrt(rrt[0] / hs.f2) : 0.0;
      floor_rel = hs.f2 > 0 ? DBL_EPSILON * std::sqrt(rrt[1] / hs.f2) : 0.0;
      if (hs.breakdown) {
        final_status = AMSP_ERR_BREAKDOWN;
        break;
      }
      if (!(relres_true <= std::max(rtol, floor_rel)) && hs.it < maxit && restarts < 3) {
        // false convergence of the recursive residual: restart from r = f - A x
        ++restarts;
        fresh = false;
        continue;
      }
      break;
    }
    const double rel_rec = hs.f2 > 0 ? std::sqrt(hs.rr / hs.f2) : 0.0;
    tot_first += h->seg_cut.empty() ? hs.it : h->seg_cut.front();
    h->hist_len = std::min(hs.it + 1, h->hist_cap);
    h->hist_f2 = hs.f2;
    tot_it += hs.it;
    tot_restarts += restarts;
    worst_true = std::max(worst_true, relres_true);
    worst_rec = std::max(worst_rec, rel_rec);
    worst_floor = std::max(worst_floor, floor_rel);
    const bool conv = (relres_true <= std::max(rtol, floor_rel)) && !hs.breakdown;
    if (!conv) all_conv = 0;
    if (!conv && final_status == AMSP_OK) final_status = AMSP_ERR_PCG_NOCONV;
  }
  inf.iterations = tot_it;
  inf.first_segment = tot_first;
  inf.converged = all_conv;
  inf.relres_recursive = worst_rec;
  inf.relres_true = worst_true;
  inf.restarts = tot_restarts;
  inf.relres_floor = worst_floor;
  inf.solve_ms = now_ms() - t0;
  if (h->timing_active) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (auto &rc : h->ev_rec) {
      const bool worked = rc.t < 0 || rc.seg >= (int)h->seg_cut.size() || rc.t < h->seg_cut[rc.seg];
      float ms = 0.f;
      if (worked && hipEventElapsedTime(&ms, h->evs[rc.idx], h->evs[rc.idx + 1]) == hipSuccess) {
        inf.kernel_ms[rc.cls] += ms;
        inf.kernel_launches[rc.cls] += 1;
      }
    }
    h->ev_rec.clear();
    h->ev_used = 0;
    h->timing_active = false;
  }
  if (info) *info = inf;
  return final_status;
}

// ------------------------------------------ independent problems at once --
// One CG recurrence per (problem, column) on a block-diagonal matrix whose
// blocks are the problems (rows [prob_ptr[s], prob_ptr[s+1])).  Every matrix
// product and preconditioner application acts on all problems and columns
// at once (the preconditioner of a block-diagonal matrix is block-diagonal:
// its regions, local factors and coarse blocks never couple two problems);
// the scalars of each recurrence come from its own problem's rows only.  The
// stopping rule of amsp_pcg applies per recurrence, restarts included.
extern "C" amsp_status amsp_pcg_batched(amsp_handle *h, int32_t nprob, const int64_t *prob_ptr,
                                        const double *f_dev, double *u_dev, int32_t nrhs,
                                        double rtol, int32_t maxit, amsp_info *info,
                                        int32_t *iterations, double *relres) {
  if (!h || !prob_ptr || !f_dev || !u_dev || nprob < 1 || nrhs < 1 || nrhs > EIGP ||
      !(rtol > 0.0) || maxit < 0)
    return AMSP_ERR_ARG;
  if (h->opt.cycle == 1) {
    h->err = "amsp_pcg_batched: the multiplicative cycle is not available here";
    return AMSP_ERR_ARG;
  }
  if (prob_ptr[0] != 0 || prob_ptr[nprob] != h->n) {
    h->err = "amsp_pcg_batched: prob_ptr must run from 0 to n";
    return AMSP_ERR_ARG;
  }
  for (int q = 0; q < nprob; ++q)
    if (prob_ptr[q + 1] <= prob_ptr[q]) {
      h->err = "amsp_pcg_batched: prob_ptr must be increasing";
      return AMSP_ERR_ARG;
    }
  const double t0 = now_ms();
  const int n = h->n, nseg = nprob, nr = nrhs, nrec = nseg * nr;
  const size_t ld = (size_t)n, tot = ld * nr;
  hipStream_t s = h->stream;
  // row blocks of at most CH rows inside each problem
  constexpr long long CH = 2048;
  std::vector<long long> brow{0};
  std::vector<int> bseg, sblk{0};
  for (int q = 0; q < nseg; ++q) {
    for (long long r = prob_ptr[q]; r < prob_ptr[q + 1]; r += CH) {
      bseg.push_back(q);
      brow.push_back(std::min<long long>(r + CH, prob_ptr[q + 1]));
    }
    sblk.push_back((int)bseg.size());
  }
  const int nblk = (int)bseg.size();
  bool ok = true;
  const long long *d_brow = upload(h, brow, ok);
  const int *d_bseg = upload(h, bseg, ok);
  const int *d_sblk = upload(h, sblk, ok);
  std::vector<long long> sp(prob_ptr, prob_ptr + nprob + 1);
  const long long *d_sptr = upload(h, sp, ok);
  double *R = h->mem.alloc<double>(tot), *Z = h->mem.alloc<double>(tot),
         *Pd = h->mem.alloc<double>(tot), *Q = h->mem.alloc<double>(tot);
  double *part = h->mem.alloc<double>((size_t)nblk * nr);
  double *sc = h->mem.alloc<double>((size_t)5 * nrec);  // alpha/beta, dots, rr, r2, a2
  double *st_rz = h->mem.alloc<double>(nrec), *st_f2 = h->mem.alloc<double>(nrec),
         *st_rr = h->mem.alloc<double>(nrec);
  int *st_act = h->mem.alloc<int>(nrec), *st_its = h->mem.alloc<int>((size_t)2 * nrec),
      *flags = h->mem.alloc<int>(2);
  auto release = [&]() {
    for (const void *b : {(const void *)d_brow, (const void *)d_bseg, (const void *)d_sblk,
                          (const void *)d_sptr, (const void *)R, (const void *)Z,
                          (const void *)Pd, (const void *)Q, (const void *)part, (const void *)sc,
                          (const void *)st_rz, (const void *)st_f2, (const void *)st_rr,
                          (const void *)st_act, (const void *)st_its, (const void *)flags})
      if (b) h->mem.free_one(const_cast<void *>(b));
  };
  if (!ok || !R || !Z || !Pd || !Q || !part || !sc || !st_rz || !st_f2 || !st_rr || !st_act ||
      !st_its || !flags) {
    release();
    h->err = "amsp_pcg_batched: device allocation failed";
    return AMSP_ERR_OOM;
  }
  double *alpha = sc, *dots = sc + nrec, *rrn = sc + 2 * nrec, *r2d = sc + 3 * nrec,
         *a2d = sc + 4 * nrec;
  // the problems must not be coupled
  {
    HIP_TRY(hipMemsetAsync(flags, 0, 2 * sizeof(int), s));
    launch_check_blocks(s, n, h->rowptr, h->col, nseg, d_sptr, flags);
    int fl = 0;
    HIP_TRY(hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (fl) {
      release();
      h->err = "amsp_pcg_batched: a stored entry couples two problems";
      return AMSP_ERR_ARG;
    }
  }
  auto rec_to_host = [&](const double *src, std::vector<double> &dst) -> hipError_t {
    dst.resize(nrec);
    hipError_t e = hipMemcpyAsync(dst.data(), src, nrec * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  };
  std::vector<double> f2, rr(nrec), rt(nrec, 0.0), fl(nrec, 0.0), rec(nrec, 0.0);
  std::vector<int> active(nrec), its(nrec, 0), broken(nrec, 0);
  launch_fill(s, tot, u_dev, 0.0);
  HIP_TRY(hipMemcpyAsync(R, f_dev, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_seg_dots(s, nblk, nseg, d_brow, d_sblk, ld, nr, f_dev, f_dev, part, dots);
  HIP_TRY(rec_to_host(dots, f2));
  for (int r = 0; r < nrec; ++r) {
    if (!std::isfinite(f2[r])) {
      release();
      h->err = "right-hand side not finite";
      return AMSP_ERR_BREAKDOWN;
    }
    rr[r] = f2[r];
    active[r] = f2[r] > 0.0;
  }
  HIP_TRY(hipMemcpyAsync(st_f2, f2.data(), nrec * sizeof(double), hipMemcpyHostToDevice, s));
  int *st_brk = st_its + nrec;  // per recurrence: broke down
  HIP_TRY(hipMemsetAsync(st_its, 0, 2 * nrec * sizeof(int), s));
  HIP_TRY(hipMemsetAsync(flags, 0, 2 * sizeof(int), s));
  int *fl_host = nullptr;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&fl_host), 4 * sizeof(int), hipHostMallocDefault));
  hipEvent_t fev[2] = {nullptr, nullptr};
  struct Guard {
    int *p;
    hipEvent_t *e;
    ~Guard() {
      for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
      if (p) (void)hipHostFree(p);
    }
  } guard{fl_host, fev};
  for (hipEvent_t &e : fev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const double rtol2 = rtol * rtol;
  int it = 0;
  bool breakdown = false;
  amsp_status st = AMSP_OK;
  for (int restarts = 0;; ++restarts) {
    HIP_TRY(hipMemcpyAsync(st_act, active.data(), nrec * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(st_rr, rr.data(), nrec * sizeof(double), hipMemcpyHostToDevice, s));
    if ((st = apply_block(h, R, Z, nr, 3)) != AMSP_OK) {
      release();
      return st;
    }
    launch_seg_dots(s, nblk, nseg, d_brow, d_sblk, ld, nr, R, Z, part, st_rz);
    HIP_TRY(hipMemcpyAsync(Pd, Z, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
    bool live = false;
    for (int v : active) live = live || v;
    int pend = -1;
    while (live && it < maxit) {
      launch_spmm_sell(s, n, h->sptr, h->scol, h->sval, ld, nr, Pd, Q);
      launch_seg_dots(s, nblk, nseg, d_brow, d_sblk, ld, nr, Pd, Q, part, dots);
      launch_seg_alpha(s, nrec, st_rz, st_f2, st_rr, st_act, st_its, st_brk, flags, dots, alpha);
      launch_seg_update(s, nblk, nseg, d_brow, d_bseg, d_sblk, ld, nr, alpha, Pd, Q, u_dev, R,
                        part, rrn);
      if ((st = apply_block(h, R, Z, nr, 3)) != AMSP_OK) {
        release();
        return st;
      }
      launch_seg_dots(s, nblk, nseg, d_brow, d_sblk, ld, nr, R, Z, part, dots);
      launch_seg_beta(s, nrec, st_rz, st_f2, st_rr, st_act, st_its, st_brk, flags, rrn, dots, rtol2,
                      alpha);
      launch_seg_direction(s, nblk, nseg, d_brow, d_bseg, ld, nr, alpha, Z, Pd);
      const int slot = pend == 0 ? 1 : 0;
      HIP_TRY(hipMemcpyAsync(fl_host + 2 * slot, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(fev[slot], s));
      HIP_TRY(hipGetLastError());
      ++it;
      if (pend >= 0) {  // the previous step's flags, read while this step runs
        HIP_TRY(hipEventSynchronize(fev[pend]));
        if (fl_host[2 * pend + 1] == 0) {
          --it;  // this step found no active recurrence (its coefficients are zero)
          pend = -1;
          break;
        }
      }
      pend = slot;
    }
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<double> rrv;
    HIP_TRY(rec_to_host(st_rr, rrv));
    HIP_TRY(hipMemcpy(its.data(), st_its, nrec * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(broken.data(), st_brk, nrec * sizeof(int), hipMemcpyDeviceToHost));
    for (int v : broken) breakdown = breakdown || v != 0;
    for (int r = 0; r < nrec; ++r) rec[r] = f2[r] > 0.0 ? std::sqrt(rrv[r] / f2[r]) : 0.0;
    // true residuals R = F - A U and their attainable floors, per recurrence
    launch_spmm_sell(s, n, h->sptr, h->scol, h->sval, ld, nr, u_dev, Q);
    launch_sub_columns(s, tot, f_dev, Q, R);
    launch_seg_dots(s, nblk, nseg, d_brow, d_sblk, ld, nr, R, R, part, r2d);
    for (int k = 0; k < nr; ++k)
      launch_abs_spmv_rows(s, n, h->rowptr, h->col, h->val, u_dev + k * ld, Q + k * ld);
    launch_seg_dots(s, nblk, nseg, d_brow, d_sblk, ld, nr, Q, Q, part, a2d);
    std::vector<double> r2, a2;
    HIP_TRY(rec_to_host(r2d, r2));
    HIP_TRY(rec_to_host(a2d, a2));
    bool again = false;
    for (int r = 0; r < nrec; ++r) {
      const double fk = std::sqrt(f2[r]);
      rt[r] = fk > 0.0 ? std::sqrt(r2[r]) / fk : 0.0;
      fl[r] = fk > 0.0 ? DBL_EPSILON * std::sqrt(a2[r]) / fk : 0.0;
      rr[r] = r2[r];
      const bool okr = !(fk > 0.0) || rt[r] <= std::max(rtol, fl[r]);
      // a broken recurrence stops; the others restart as usual
      active[r] = !okr && std::isfinite(rt[r]) && restarts < 3 && it < maxit && !broken[r];
      again = again || active[r];
    }
    if (!again) break;
  }
  amsp_info inf{};
  inf.converged = 1;
  for (int r = 0; r < nrec; ++r) {
    const bool conv = (rt[r] <= std::max(rtol, fl[r]) || f2[r] == 0.0) && std::isfinite(rt[r]);
    if (!conv) inf.converged = 0;
    inf.iterations += its[r];
    inf.first_segment += its[r];
    inf.relres_true = std::max(inf.relres_true, rt[r]);
    inf.relres_recursive = std::max(inf.relres_recursive, rec[r]);
    inf.relres_floor = std::max(inf.relres_floor, fl[r]);
    if (iterations) iterations[(size_t)(r % nseg) * nr + r / nseg] = its[r];
    if (relres) relres[(size_t)(r % nseg) * nr + r / nseg] = rt[r];
  }
  inf.restarts = 0;
  inf.solve_ms = now_ms() - t0;
  inf.bytes_per_iter = 0;
  if (info) *info = inf;
  release();
  if (breakdown) {
    h->err = "CG breakdown in a recurrence (p.Ap <= 0 or a non-finite value)";
    return AMSP_ERR_BREAKDOWN;
  }
  return inf.converged ? AMSP_OK : AMSP_ERR_PCG_NOCONV;
}

// ---------------------------------------------------------------- GMRES ----
// Restarted GMRES with flexible right preconditioning (Saad, Iterative
// Methods for Sparse Linear Systems, Section 9.4.1): Arnoldi on A M^{-1}
// with the preconditioned vectors kept, Gram-Schmidt twice per step on the
// device, Givens rotations and the triangular solve on the host.
extern "C" amsp_status amsp_gmres(amsp_handle *h, const double *f_dev, double *u_dev, int32_t nrhs,
                                  int32_t restart, double rtol, int32_t maxit, amsp_info *info) {
  if (!h || !f_dev || !u_dev || nrhs < 1 || restart < 1 || restart > AMSP_GMRES_MAX_RESTART ||
      maxit < 0 || !(rtol >= 0.0))
    return AMSP_ERR_ARG;
  const int n = h->n, m = restart, nb = reduce_blocks(n);
  const size_t ld = (size_t)n;
  hipStream_t s = h->stream;
  amsp_info inf{};
  inf.bytes_per_iter = bytes_per_iter(h);
  inf.local_apply_bytes = local_apply_bytes(h);
  h->timing_active = false;
  const double t0 = now_ms();
  if (h->hist_cap < maxit + 2) {
    if (h->hist) h->mem.free_one(h->hist);
    h->hist_cap = std::max(maxit + 2, 1024);
    ALLOC(h->hist, double, h->hist_cap);
  }
  // scalars on the device: [0, 64) first Gram-Schmidt coefficients, [64, 128)
  // second ones, [128] squared norm, [192, 256) the cycle's y
  double *V = nullptr, *Z = nullptr, *part = nullptr, *sc = nullptr;
  ALLOC(V, double, ld * (m + 1));
  ALLOC(Z, double, ld * m);
  ALLOC(part, double, (size_t)nb * (m + 2));
  ALLOC(sc, double, 256);
  double *w = h->q, *pn = part + (size_t)nb * (m + 1);
  auto release = [&]() {
    h->mem.free_one(V);
    h->mem.free_one(Z);
    h->mem.free_one(part);
    h->mem.free_one(sc);
  };
  auto sq_to_host = [&](double &out) -> hipError_t {  // sc[128] -> host
    hipError_t e = hipMemcpyAsync(&out, sc + 128, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  };
  amsp_status final_status = AMSP_OK;
  int tot_it = 0, tot_restarts = 0, all_conv = 1;
  double worst_true = 0.0, worst_est = 0.0, worst_floor = 0.0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  std::vector<double> g2;
  if (!h->gm_host) {
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&h->gm_host), 2 * 129 * sizeof(double),
                          hipHostMallocDefault));
    for (hipEvent_t &e : h->gm_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // One Arnoldi step on the device: z_j = M^-1 v_j, w = A z_j, two rounds of
  // classical Gram-Schmidt against v_0..v_j, v_{j+1} = w / |w|; its 129
  // coefficients are copied behind it to pinned slot j % 2.
  auto arnoldi_step = [&](int j) -> amsp_status {
    double *vj = V + (size_t)j * ld, *zj = Z + (size_t)j * ld;
    amsp_status st = apply_prec(h, vj, zj, nullptr, nullptr);
    if (st != AMSP_OK) return st;
    launch_spmv_sell(s, n, h->sptr, h->scol, h->sval, zj, w);
    launch_gs_dots(s, n, V, ld, j + 1, w, part, sc);
    launch_gs_update(s, n, V, ld, j + 1, sc, w, nullptr);
    launch_gs_dots(s, n, V, ld, j + 1, w, part, sc + 64);
    launch_gs_update(s, n, V, ld, j + 1, sc + 64, w, pn);
    launch_sum_partials(s, pn, nb, sc + 128);
    launch_gs_normalize(s, n, w, sc + 128, V + (size_t)(j + 1) * ld);
    HIP_TRY(hipMemcpyAsync(h->gm_host + (j & 1) * 129, sc, 129 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(h->gm_ev[j & 1], s));
    HIP_TRY(hipGetLastError());
    return AMSP_OK;
  };
  for (int rhs = 0; rhs < nrhs; ++rhs) {
    const double *f = f_dev + (size_t)rhs * n;
    double *x = u_dev + (size_t)rhs * n;
    launch_fill(s, n, x, 0.0);
    launch_copy_scale(s, n, f, h->r, 1.0);
    launch_dot(s, n, f, f, pn, nullptr);
    launch_sum_partials(s, pn, nb, sc + 128);
    double f2 = 0.0;
    HIP_TRY(sq_to_host(f2));
    const double nf = std::sqrt(f2);
    if (!std::isfinite(nf)) {
      release();
      h->err = "right-hand side not finite";
      return AMSP_ERR_BREAKDOWN;
    }
    g2.assign(1, f2);
    double beta = nf, est = nf > 0.0 ? 1.0 : 0.0, relres_true = est, floor_rel = 0.0;
    int it = 0, cycles = 0;
    bool conv = nf == 0.0;
    while (!conv && it < maxit) {
      launch_gs_normalize(s, n, h->r, sc + 128, V);  // v_0 = r / beta
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int k = 0;
      // Step j + 1 is enqueued before the host reads step j's coefficients,
      // so the device runs on while the host applies the rotations, unless
      // the estimate's recent decay says that step j converges (a step
      // enqueued after the last one is harmless: its results are not used).
      double est_prev = -1.0;
      bool queued = false;  // step j already enqueued
      for (int j = 0; j < m; ++j) {
        if (!queued) {
          const amsp_status st = arnoldi_step(j);
          if (st != AMSP_OK) {
            release();
            return st;
          }
        }
        double pred = est;  // estimate expected after step j
        if (est_prev > 0.0 && est < est_prev) pred = est * (est / est_prev);
        queued = j + 1 < m && it + 1 < maxit && pred > rtol;
        if (queued) {
          const amsp_status st = arnoldi_step(j + 1);
          if (st != AMSP_OK) {
            release();
            return st;
          }
        }
        HIP_TRY(hipEventSynchronize(h->gm_ev[j & 1]));
        const double *coef = h->gm_host + (j & 1) * 129;
        double *hj = H.data() + (size_t)j * (m + 1);  // column j of H
        for (int i = 0; i <= j; ++i) hj[i] = coef[i] + coef[64 + i];
        const double hnext = std::sqrt(coef[128]);
        hj[j + 1] = hnext;
        for (int i = 0; i < j; ++i) {  // earlier rotations
          const double a = hj[i], b = hj[i + 1];
          hj[i] = cs[i] * a + sn[i] * b;
          hj[i + 1] = -sn[i] * a + cs[i] * b;
        }
        const double a = hj[j], b = hj[j + 1], rho = std::hypot(a, b);
        cs[j] = rho > 0.0 ? a / rho : 1.0;
        sn[j] = rho > 0.0 ? b / rho : 0.0;
        hj[j] = rho;
        hj[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++it;
        k = j + 1;
        g2.push_back(g[j + 1] * g[j + 1]);
        est_prev = est;
        est = nf > 0.0 ? std::fabs(g[j + 1]) / nf : 0.0;
        if (std::fabs(g[j + 1]) <= rtol * nf || it >= maxit || !(hnext > 0.0) || !(rho > 0.0)) break;
      }
      // y = R^{-1} g (R: the rotated upper triangle of H), x += Z y
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < k; ++c) t -= H[(size_t)c * (m + 1) + i] * y[c];
        const double d = H[(size_t)i * (m + 1) + i];
        y[i] = d != 0.0 ? t / d : 0.0;
      }
      HIP_TRY(hipMemcpyAsync(sc + 192, y.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
      launch_basis_combine(s, n, Z, ld, k, sc + 192, x);
      // true residual; it seeds the next cycle
      launch_spmv_sell(s, n, h->sptr, h->scol, h->sval, x, w);
      launch_residual(s, n, f, w, h->r, pn);
      launch_sum_partials(s, pn, nb, sc + 128);
      double r2 = 0.0;
      HIP_TRY(sq_to_host(r2));
      beta = std::sqrt(r2);
      relres_true = beta / nf;
      ++cycles;
      if (!std::isfinite(beta)) {
        release();
        h->err = "GMRES breakdown: residual not finite";
        return AMSP_ERR_BREAKDOWN;
      }
      if (relres_true <= rtol) {
        conv = true;
      } else if (est <= rtol) {
        // the estimate met rtol but the recomputed residual did not: accept
        // if it is at the rounding floor, otherwise the next cycle continues
        launch_abs_spmv_sq(s, n, h->rowptr, h->col, h->val, x, pn);
        launch_sum_partials(s, pn, nb, sc + 128);
        double a2 = 0.0;
        HIP_TRY(sq_to_host(a2));
        floor_rel = DBL_EPSILON * std::sqrt(a2) / nf;
        conv = relres_true <= floor_rel;
      }
      if (!(beta > 0.0)) conv = true;  // exact solution
    }
    h->hist_len = std::min((int)g2.size(), h->hist_cap);
    h->hist_f2 = f2;
    HIP_TRY(hipMemcpyAsync(h->hist, g2.data(), h->hist_len * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    tot_it += it;
    tot_restarts += std::max(cycles - 1, 0);
    worst_true = std::max(worst_true, relres_true);
    worst_est = std::max(worst_est, est);
    worst_floor = std::max(worst_floor, floor_rel);
    if (!conv) {
      all_conv = 0;
      if (final_status == AMSP_OK) final_status = AMSP_ERR_PCG_NOCONV;
    }
  }
  release();
  inf.iterations = tot_it;
  inf.first_segment = tot_it;  // GMRES: every step counts (no CG segments)
  inf.converged = all_conv;
  inf.relres_recursive = worst_est;
  inf.relres_true = worst_true;
  inf.restarts = tot_restarts;
  inf.relres_floor = worst_floor;
  inf.solve_ms = now_ms() - t0;
  if (info) *info = inf;
  return final_status;
}

// ------------------------------------------------------- introspection ----
extern "C" amsp_status amsp_get_setup_info(const amsp_handle *h, amsp_setup_info *info) {
  if (!h || !info) return AMSP_ERR_ARG;
  *info = h->sinfo;
  return AMSP_OK;
}

extern "C" amsp_status amsp_get_pcg_history(const amsp_handle *hc, double *relres_host,
                                            int32_t cap, int32_t *count) {
  amsp_handle *h = const_cast<amsp_handle *>(hc);
  if (!h || !count) return AMSP_ERR_ARG;
  *count = h->hist_len;
  if (!relres_host || h->hist_len == 0) return AMSP_OK;
  const int k = std::min(cap, h->hist_len);
  std::vector<double> tmp(k);
  HIP_TRY(hipMemcpyAsync(tmp.data(), h->hist, k * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int j = 0; j < k; ++j) relres_host[j] = h->hist_f2 > 0 ? std::sqrt(tmp[j] / h->hist_f2) : 0.0;
  return AMSP_OK;
}

extern "C" amsp_status amsp_get_eigenvalues(const amsp_handle *hc, double *lambda_host) {
  amsp_handle *h = const_cast<amsp_handle *>(hc);
  if (!h || !lambda_host) return AMSP_ERR_ARG;
  HIP_TRY(hipMemcpyAsync(lambda_host, h->lam, (size_t)h->N * (h->nev + 1) * sizeof(double),
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return AMSP_OK;
}

extern "C" amsp_status amsp_get_coarse_matrix(const amsp_handle *hc, double *a0_host) {
  amsp_handle *h = const_cast<amsp_handle *>(hc);
  if (!h || !a0_host) return AMSP_ERR_ARG;
  if (h->nc == 0) return AMSP_OK;
  if (!h->a0keep) {
    h->err = "A0 not kept: set amsp_options.keep_a0 = 1 before amsp_setup";
    return AMSP_ERR_ARG;
  }
  const int T0 = h->T0, nc = h->nc;
  std::vector<double> t((size_t)T0 * T0 * TE);
  HIP_TRY(hipMemcpyAsync(t.data(), h->a0keep, t.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int R = 0; R < nc; ++R)
    for (int C = 0; C < nc; ++C)
      a0_host[(size_t)R * nc + C] =
          t[((size_t)(R / TS) * T0 + C / TS) * TE + (size_t)(R % TS) * TS + (C % TS)];
  return AMSP_OK;
}

extern "C" amsp_status amsp_get_region(const amsp_handle *hc, int32_t i, int32_t *ni, int32_t *dofs,
                                       double *phi) {
  amsp_handle *h = const_cast<amsp_handle *>(hc);
  if (!h || !ni || i < 0 || i >= h->N) return AMSP_ERR_ARG;
  const int r0 = h->hp.sd_ptr[i], cnt = h->hp.sd_ptr[i + 1] - r0;
  *ni = cnt;
  if (dofs) std::memcpy(dofs, h->hp.sd_dofs.data() + r0, cnt * sizeof(int));
  if (phi && h->nev > 0) {
    if (!h->phi64) return AMSP_ERR_ARG;
    HIP_TRY(hipMemcpyAsync(phi, h->phi64 + (size_t)r0 * h->nev, (size_t)cnt * h->nev * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return AMSP_OK;
}

extern "C" amsp_status amsp_plan_regions(const amsp_csr *A, const int32_t *partition,
                                         int32_t nparts, int32_t nev, const amsp_options *opt,
                                         int32_t *region_ptr, int32_t *region_dofs, int64_t cap,
                                         int64_t *ntiles, int64_t *npairs) {
  if (!region_ptr) return AMSP_ERR_ARG;
  amsp_options o;
  amsp_default_options(&o);
  if (opt) o = *opt;
  std::string msg;
  int64_t offdiag_zeros = -1;
  int s = validate_inputs(A, partition, nparts, nev, o.overlap, msg, &offdiag_zeros);
  if (s != AMSP_OK) {
    g_setup_error = msg;
    return (amsp_status)s;
  }
  HostPlan P;
  P.offdiag_zeros = offdiag_zeros != 0;
  try {
    s = build_plan(A, partition, nparts, nev, o, P, msg);
  } catch (const std::bad_alloc &) {
    g_setup_error = "host allocation failed during planning";
    return AMSP_ERR_OOM;
  }
  if (s != AMSP_OK) {
    g_setup_error = msg;
    return (amsp_status)s;
  }
  for (int i = 0; i <= nparts; ++i) region_ptr[i] = P.sd_ptr[i];
  if (region_dofs) {
    if (cap < (int64_t)P.sd_dofs.size()) return AMSP_ERR_ARG;
    std::memcpy(region_dofs, P.sd_dofs.data(), P.sd_dofs.size() * sizeof(int32_t));
  }
  if (ntiles) *ntiles = P.ntiles;
  if (npairs) *npairs = (int64_t)P.pair_i.size();
  return AMSP_OK;
}

extern "C" amsp_status amsp_selftest_mfma(const double *a_host, const double *b_host, double *d_host) {
  if (!a_host || !b_host || !d_host) return AMSP_ERR_ARG;
  double *d = nullptr;
  if (hipMalloc(&d, (64 + 64 + 256) * sizeof(double)) != hipSuccess) return AMSP_ERR_HIP;
  amsp_status st = AMSP_OK;
  if (hipMemcpy(d, a_host, 64 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d + 64, b_host, 64 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    st = AMSP_ERR_HIP;
  } else {
    launch_selftest_mfma(nullptr, d, d + 64, d + 128);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpy(d_host, d + 128, 256 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      st = AMSP_ERR_HIP;
  }
  hipFree(d);
  return st;
}

extern "C" void amsp_release_caches(void) {
  release_dev_cache();
  plan_release_caches();
}

extern "C" void amsp_destroy(amsp_handle *h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream); else hipDeviceSynchronize();
  delete h;
}

extern "C" const char *amsp_status_string(amsp_status s) {
  switch (s) {
    case AMSP_OK: return "AMSP_OK";
    case AMSP_ERR_ARG: return "AMSP_ERR_ARG";
    case AMSP_ERR_CSR: return "AMSP_ERR_CSR";
    case AMSP_ERR_NONSYM: return "AMSP_ERR_NONSYM";
    case AMSP_ERR_PARTITION: return "AMSP_ERR_PARTITION";
    case AMSP_ERR_NEUMANN_DIAG: return "AMSP_ERR_NEUMANN_DIAG";
    case AMSP_ERR_LOCAL_NOT_SPD: return "AMSP_ERR_LOCAL_NOT_SPD";
    case AMSP_ERR_EIG_NOCONV: return "AMSP_ERR_EIG_NOCONV";
    case AMSP_ERR_COARSE_NOT_SPD: return "AMSP_ERR_COARSE_NOT_SPD";
    case AMSP_ERR_PCG_NOCONV: return "AMSP_ERR_PCG_NOCONV";
    case AMSP_ERR_BREAKDOWN: return "AMSP_ERR_BREAKDOWN";
    case AMSP_ERR_HIP: return "AMSP_ERR_HIP";
    case AMSP_ERR_OOM: return "AMSP_ERR_OOM";
  }
  return "AMSP_UNKNOWN";
}

extern "C" const char *amsp_last_error(const amsp_handle *h) { return h ? h->err.c_str() : ""; }
extern "C" const char *amsp_setup_error(void) { return g_setup_error.c_str(); }
