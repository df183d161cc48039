// Host-side input validation and index planning (integer work only).
//
// Planning turns (CSR pattern, partition, overlap) into the per-subdomain
// index sets the device kernels consume:
//   * cores Omega_i from the partition and regions Omega_i^delta by delta
//     rounds of graph growth (Section 3.1: non-overlapping graph subdomains
//     and an overlapping support region around each);
//   * a local order per region (reverse Cuthill-McKee by default) and the
//     region's local CSR in that order;
//   * the 64x64 tile profile of each local lower triangle;
//   * dof multiplicities and the inverse map dof -> (subdomain, local index);
//   * extended regions (one more layer) and the subdomain pairs whose
//     supports couple through A, used to form A0 = R0 A R0^T.
#include "amsp_plan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <condition_variable>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include <unistd.h>
#include <unordered_map>

namespace amsp {

namespace {
constexpr size_t kCacheMin = size_t(1) << 20;
constexpr size_t kCacheCap = size_t(4) << 30;
// Blocks of the cache are page-locked when a device is present, so that the
// plan's uploads are direct transfers; without a device (host-only
// planning) they are ordinary memory.
struct Block {
  size_t size;
  bool pinned;
};
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, std::pair<void *, bool>> free_blocks;  // size -> (block, pinned)
  std::unordered_map<void *, Block> live;
  size_t held = 0;
};
void register_exit_release();
BlockCache &block_cache() {
  // never destroyed: blocks may be returned after static destructors ran; the
  // free blocks are released by plan_release_caches (exit handler)
  static BlockCache *c = new BlockCache();
  return *c;
}
void *block_new(size_t bytes, bool &pinned) {
  void *p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocPortable) == hipSuccess && p) {
    pinned = true;
    return p;
  }
  (void)hipGetLastError();  // clear the failed call's error
  pinned = false;
  return ::operator new(bytes);
}
void block_delete(void *p, bool pinned) {
  if (pinned)
    (void)hipHostFree(p);
  else
    ::operator delete(p);
}
}  // namespace

void *plan_alloc(size_t bytes) {
  if (bytes < kCacheMin) return ::operator new(bytes);
  register_exit_release();
  BlockCache &c = block_cache();
  const size_t want = (bytes + kCacheMin - 1) & ~(kCacheMin - 1);
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free_blocks.lower_bound(want);
    if (it != c.free_blocks.end() && it->first <= 2 * want) {
      void *p = it->second.first;
      c.live[p] = Block{it->first, it->second.second};
      c.held -= it->first;
      c.free_blocks.erase(it);
      return p;
    }
  }
  bool pinned;
  void *p = block_new(want, pinned);
  std::lock_guard<std::mutex> lk(c.mu);
  c.live[p] = Block{want, pinned};
  return p;
}

void plan_free(void *p, size_t bytes) {
  if (!p) return;
  if (bytes < kCacheMin) {
    ::operator delete(p);
    return;
  }
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  const Block blk = it->second;
  c.live.erase(it);
  if (c.held + blk.size <= kCacheCap) {
    c.free_blocks.emplace(blk.size, std::make_pair(p, blk.pinned));
    c.held += blk.size;
  } else {
    block_delete(p, blk.pinned);
  }
}

namespace {
// Persistent workers for the planner's parallel loops: starting and joining
// fresh threads costs ~0.5 ms per loop, and planning runs a few dozen loops.
// One loop runs on the pool at a time; a caller that finds it busy (the
// coupling thread and the main thread may plan concurrently) starts its own
// threads.  After a fork the child builds a new pool (the parent's workers
// do not exist there).
std::mutex g_pool_mu;
class PlanPool;
PlanPool *g_pool = nullptr;

class PlanPool {
 public:
  static PlanPool *get(int nworkers) {
    register_exit_release();
    std::lock_guard<std::mutex> lk(g_pool_mu);
    // a forked child cannot use (or join) its parent's workers: it leaves
    // that pool alone and builds its own
    if (!g_pool || g_pool->pid_ != getpid()) g_pool = new PlanPool(nworkers);
    return g_pool;
  }
  // Stops and joins the workers (no loop may be running) and frees the pool.
  static void shutdown() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    PlanPool *pool = g_pool;
    if (!pool || pool->pid_ != getpid()) return;
    g_pool = nullptr;
    {
      std::lock_guard<std::mutex> l2(pool->mu_);
      pool->stop_ = true;
    }
    pool->cv_.notify_all();
    for (std::thread &t : pool->threads_) t.join();
    delete pool;
  }
  // fn(i) for i in [0, n) on the caller and up to nth - 1 workers; false
  // when another loop occupies the pool
  template <typename F>
  bool run(int n, int nth, F &fn) {
    std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    const int want = std::min(nth - 1, nworkers_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      call_ = [](void *c, int i) { (*static_cast<F *>(c))(i); };
      ctx_ = &fn;
      count_ = n;
      want_ = want;
      finished_ = 0;
      next_.store(0);
      ++gen_;
    }
    cv_.notify_all();
    for (;;) {
      const int i = next_.fetch_add(1);
      if (i >= n) break;
      fn(i);
    }
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return finished_ == want_; });
    return true;
  }

 private:
  explicit PlanPool(int nworkers) : nworkers_(nworkers), pid_(getpid()) {
    for (int w = 0; w < nworkers; ++w) threads_.emplace_back([this, w] { loop(w); });
  }
  void loop(int w) {
    unsigned long long seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return gen_ != seen || stop_; });
      if (stop_) return;
      seen = gen_;
      if (w >= want_) continue;  // not asked to join this loop
      void (*call)(void *, int) = call_;
      void *ctx = ctx_;
      const int n = count_;
      lk.unlock();
      for (;;) {
        const int i = next_.fetch_add(1);
        if (i >= n) break;
        call(ctx, i);
      }
      lk.lock();
      if (++finished_ == want_) cv_done_.notify_one();
    }
  }
  const int nworkers_;
  const pid_t pid_;
  std::mutex busy_, mu_;
  std::condition_variable cv_, cv_done_;
  unsigned long long gen_ = 0;
  void (*call_)(void *, int) = nullptr;
  void *ctx_ = nullptr;
  int count_ = 0, want_ = 0, finished_ = 0;
  bool stop_ = false;
  std::atomic<int> next_{0};
  std::vector<std::thread> threads_;
};

// At process exit the planner's workers are joined and its cached host
// blocks released before the HIP runtime tears itself down: the handler is
// registered after a first runtime call, and exit handlers run in reverse
// order of registration.
void register_exit_release() {
  static std::once_flag once;
  std::call_once(once, [] {
    int ndev = 0;
    (void)hipGetDeviceCount(&ndev);  // the runtime's own exit work is registered by now
    (void)hipGetLastError();
    std::atexit([] { plan_release_caches(); });
  });
}
}  // namespace

void scratch_release();

void plan_release_caches() {
  PlanPool::shutdown();
  scratch_release();
  BlockCache &c = block_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (auto &kv : c.free_blocks) block_delete(kv.second.first, kv.second.second);
  c.free_blocks.clear();
  c.held = 0;
}

// Run fn(i) for i in [0, count) on up to 16 threads (dynamic schedule).
template <typename F>
static void parallel_for(int count, F fn) {
  unsigned hw = std::thread::hardware_concurrency();
#ifdef AMSP_PLAN_SERIAL
  hw = 1;
#endif
  const int maxth = (int)std::min<unsigned>(hw ? hw : 1, 16);
  const int nth = std::max(1, std::min(maxth, count));
  if (nth > 1 && PlanPool::get(maxth - 1)->run(count, nth, fn)) return;
  std::atomic<int> next(0);
  auto work = [&]() {
    for (;;) {
      int i = next.fetch_add(1);
      if (i >= count) break;
      fn(i);
    }
  };
  std::vector<std::thread> ts;
  for (int t = 1; t < nth; ++t) ts.emplace_back(work);
  work();
  for (auto &t : ts) t.join();
}

void plan_parallel_for(int count, const std::function<void(int)> &fn) {
  parallel_for(count, [&](int c) { fn(c); });
}

// ptr[0] = 0, ptr[j + 1] = ptr[j] + cnt[j] for j < n (chunked, in parallel).
template <typename V1, typename V2>
static void exclusive_scan(const V1 &cnt, V2 &ptr, int n) {
  const int nch = 16;
  std::vector<long long> part(nch + 1, 0);
  auto rng = [&](int c, int &a, int &b) {
    a = (int)((long long)n * c / nch);
    b = (int)((long long)n * (c + 1) / nch);
  };
  parallel_for(nch, [&](int c) {
    int a, b;
    rng(c, a, b);
    long long t = 0;
    for (int j = a; j < b; ++j) t += cnt[j];
    part[c + 1] = t;
  });
  for (int c = 0; c < nch; ++c) part[c + 1] += part[c];
  ptr[0] = 0;
  parallel_for(nch, [&](int c) {
    int a, b;
    rng(c, a, b);
    long long t = part[c];
    for (int j = a; j < b; ++j) {
      t += cnt[j];
      ptr[j + 1] = (int)t;
    }
  });
}

int validate_inputs(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
                    int32_t overlap, std::string &msg, int64_t *offdiag_zeros) {
  if (offdiag_zeros) *offdiag_zeros = -1;
  if (!A || !part || !A->row_ptr || !A->col_idx || !A->val) {
    msg = "null pointer argument";
    return AMSP_ERR_ARG;
  }
  if (nev < 0 || nev > MAXNEV) {
    msg = "nev must be in [0, " + std::to_string(MAXNEV) + "]";
    return AMSP_ERR_ARG;
  }
  if (overlap < 0 || overlap > 64) {
    msg = "overlap must be in [0, 64]";
    return AMSP_ERR_ARG;
  }
  const int64_t n = A->n;
  if (n < 1 || n > (int64_t)1 << 30) {
    msg = "n out of range";
    return n < 1 ? AMSP_ERR_ARG : AMSP_ERR_OOM;
  }
  if (nparts < 1 || nparts > n) {
    msg = "nparts must be in [1, n]";
    return AMSP_ERR_PARTITION;
  }
  const int64_t *rp = A->row_ptr;
  if (rp[0] != 0 || rp[n] != A->nnz || A->nnz >= ((int64_t)1 << 31)) {
    msg = "row_ptr[0] must be 0, row_ptr[n] == nnz < 2^31";
    return AMSP_ERR_CSR;
  }
  // One pass over row chunks: row structure, column range and order, finite
  // values, diagonal present, max |a|, counts of strictly upper / lower
  // entries, and for every strictly upper entry (i, c) the largest
  // |a_ci - a_ic| over its mirror (a missing mirror counts as infinite).
  // Each chunk records its first failing row (the lowest failing row overall
  // is reported).  A structure error is reported before any asymmetry: the
  // mirror lookups read rows not yet checked (guarded so that they stay in
  // bounds) and mean something only once every row is well formed.
  const int nchunk = 64;
  std::vector<int> cerr(nchunk, 0);
  std::vector<int64_t> crow(nchunk, -1), cup(nchunk, 0), clo(nchunk, 0), czero(nchunk, 0);
  std::vector<double> cmax(nchunk, 0.0), cdiff(nchunk, 0.0);
  auto chunk_rows = [&](int c, int64_t &r0, int64_t &r1) {
    r0 = n * c / nchunk;
    r1 = n * (c + 1) / nchunk;
  };
  const int64_t nnz = A->nnz;
  parallel_for(nchunk, [&](int c) {
    int64_t r0, r1;
    chunk_rows(c, r0, r1);
    double amax = 0.0, dmax = 0.0;
    int64_t up = 0, lo = 0, zero = 0;
    for (int64_t i = r0; i < r1; ++i) {
      if (rp[i] < 0 || rp[i + 1] < rp[i] || rp[i + 1] > nnz) {
        cerr[c] = 4;
        crow[c] = i;
        return;
      }
      bool diag = false;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t cc = A->col_idx[e];
        if (cc < 0 || cc >= n || (e > rp[i] && cc <= A->col_idx[e - 1]) || !std::isfinite(A->val[e])) {
          cerr[c] = 1;
          crow[c] = i;
          return;
        }
        if (cc == i) diag = true;
        up += (cc > i);
        lo += (cc < i);
        zero += (cc != i && A->val[e] == 0.0);
        amax = std::max(amax, std::fabs(A->val[e]));
        if (cc > i) {
          const int64_t b0 = rp[cc], b1 = rp[cc + 1];
          double d = INFINITY;
          if (b0 >= 0 && b0 <= b1 && b1 <= nnz) {
            const int32_t *b = A->col_idx + b0, *en = A->col_idx + b1;
            const int32_t *f = std::lower_bound(b, en, (int32_t)i);
            if (f != en && *f == i) d = std::fabs(A->val[b0 + (f - b)] - A->val[e]);
          }
          dmax = std::max(dmax, d);
        }
      }
      if (!diag) {
        cerr[c] = 2;
        crow[c] = i;
        return;
      }
    }
    cmax[c] = amax;
    cdiff[c] = dmax;
    cup[c] = up;
    clo[c] = lo;
    czero[c] = zero;
  });
  for (int c = 0; c < nchunk; ++c) {
    if (cerr[c] == 4) {
      msg = "row_ptr not monotone at row " + std::to_string(crow[c]);
      return AMSP_ERR_CSR;
    }
    if (cerr[c] == 1) {
      msg = "column index out of range, unsorted, or non-finite value in row " + std::to_string(crow[c]);
      return AMSP_ERR_CSR;
    }
    if (cerr[c] == 2) {
      msg = "missing diagonal entry in row " + std::to_string(crow[c]);
      return AMSP_ERR_CSR;
    }
  }
  double amax = 0.0, dmax = 0.0;
  int64_t nup = 0, nlo = 0, nzero = 0;
  for (int c = 0; c < nchunk; ++c) {
    amax = std::max(amax, cmax[c]);
    dmax = std::max(dmax, cdiff[c]);
    nup += cup[c];
    nlo += clo[c];
    nzero += czero[c];
  }
  // Every strictly upper entry (i, c) has its mirror (c, i) with the same
  // value up to 1e-14 max|a|; with as many lower as upper entries this pairs
  // them all, so the pattern and the values are symmetric.  Only when that
  // fails is the first failing row looked for, in a second pass.
  const double tol = 1e-14 * amax;
  if (!(dmax <= tol)) {
    parallel_for(nchunk, [&](int c) {
      int64_t r0, r1;
      chunk_rows(c, r0, r1);
      for (int64_t i = r0; i < r1; ++i) {
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
          const int32_t cc = A->col_idx[e];
          if (cc <= i) continue;
          const int32_t *b = A->col_idx + rp[cc], *en = A->col_idx + rp[cc + 1];
          const int32_t *f = std::lower_bound(b, en, (int32_t)i);
          if (f == en || *f != i || std::fabs(A->val[rp[cc] + (f - b)] - A->val[e]) > tol) {
            cerr[c] = 3;
            crow[c] = i;
            return;
          }
        }
      }
    });
    for (int c = 0; c < nchunk; ++c)
      if (cerr[c] == 3) {
        msg = "matrix not symmetric in row " + std::to_string(crow[c]);
        return AMSP_ERR_NONSYM;
      }
  }
  if (nup != nlo) {
    msg = "matrix pattern not symmetric (upper and lower entry counts differ)";
    return AMSP_ERR_NONSYM;
  }
  // partition values in range and every part non-empty (chunk counts, or
  // one serial count when there are very many parts)
  const int pchunks = nparts <= 4096 ? nchunk : 1;
  auto prow = [&](int c, int64_t &r0, int64_t &r1) {
    r0 = n * c / pchunks;
    r1 = n * (c + 1) / pchunks;
  };
  std::vector<std::vector<int64_t>> pc(pchunks);
  parallel_for(pchunks, [&](int c) {
    int64_t r0, r1;
    prow(c, r0, r1);
    pc[c].assign(nparts, 0);
    for (int64_t j = r0; j < r1; ++j) {
      if (part[j] < 0 || part[j] >= nparts) {
        cerr[c] = 5;
        crow[c] = j;
        return;
      }
      pc[c][part[j]]++;
    }
  });
  for (int c = 0; c < pchunks; ++c)
    if (cerr[c] == 5) {
      msg = "partition value out of range at dof " + std::to_string(crow[c]);
      return AMSP_ERR_PARTITION;
    }
  for (int32_t k = 0; k < nparts; ++k) {
    int64_t cnt = 0;
    for (int c = 0; c < pchunks; ++c) cnt += pc[c][k];
    if (cnt == 0) {
      msg = "empty subdomain " + std::to_string(k);
      return AMSP_ERR_PARTITION;
    }
  }
  if (offdiag_zeros) *offdiag_zeros = nzero;
  return AMSP_OK;
}

// Work arrays of rcm_order, reused across calls by one worker.
struct RcmWork {
  std::vector<int> deg, level, q, touched, nb;
  std::vector<char> vis;
};

// Reverse Cuthill-McKee order of a small graph given as adjacency lists
// (local indices).  Each component starts from a pseudo-peripheral node
// (George-Liu search, at most four BFS passes); neighbours are visited by
// increasing degree, ties by index.
static void rcm_order(const std::vector<int> &adj_ptr, const std::vector<int> &adj,
                      std::vector<int> &order, RcmWork &W) {
  const int n = (int)adj_ptr.size() - 1;
  W.deg.resize(n);
  W.level.assign(n, -1);
  W.vis.assign(n, 0);
  for (int v = 0; v < n; ++v) W.deg[v] = adj_ptr[v + 1] - adj_ptr[v];
  const int *deg = W.deg.data();
  int *level = W.level.data();
  char *vis = W.vis.data();
  order.clear();
  order.reserve(n);
  W.q.resize(n);
  // BFS within the component (unvisited nodes); returns the min-degree node
  // of the last level and its eccentricity
  auto bfs_last_min = [&](int s, int &ecc) {
    int *q = W.q.data();
    int head = 0, tail = 0;
    q[tail++] = s;
    level[s] = 0;
    int last = 0;
    while (head < tail) {
      const int v = q[head++];
      last = level[v];
      for (int e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e) {
        const int w = adj[e];
        if (!vis[w] && level[w] < 0) {
          level[w] = level[v] + 1;
          q[tail++] = w;
        }
      }
    }
    int best = -1;
    for (int k = tail - 1; k >= 0 && level[q[k]] == last; --k) {
      const int v = q[k];
      if (best < 0 || deg[v] < deg[best] || (deg[v] == deg[best] && v < best)) best = v;
    }
    for (int k = 0; k < tail; ++k) level[q[k]] = -1;
    ecc = last;
    return best;
  };
  std::vector<int> &nb = W.nb;
  // Cuthill-McKee from s (appended to order): a BFS whose levels are
  // contiguous in the order, so it also yields s's eccentricity and the
  // min-degree node of its last level, as bfs_last_min would
  auto cm_from = [&](int s, int &ecc) {
    const size_t h0 = order.size();
    size_t h = h0;
    order.push_back(s);
    vis[s] = 1;
    level[s] = 0;
    while (h < order.size()) {
      const int v = order[h++];
      nb.clear();
      for (int e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e)
        if (!vis[adj[e]]) nb.push_back(adj[e]);
      for (size_t x = 1; x < nb.size(); ++x) {  // short lists: insertion sort by (degree, index)
        const int w = nb[x];
        size_t y = x;
        while (y > 0 && (deg[nb[y - 1]] > deg[w] || (deg[nb[y - 1]] == deg[w] && nb[y - 1] > w))) {
          nb[y] = nb[y - 1];
          --y;
        }
        nb[y] = w;
      }
      for (int w : nb)
        if (!vis[w]) {
          vis[w] = 1;
          level[w] = level[v] + 1;
          order.push_back(w);
        }
    }
    const int last = level[order.back()];
    int best = -1;
    for (size_t k = order.size(); k-- > h0 && level[order[k]] == last;) {
      const int v = order[k];
      if (best < 0 || deg[v] < deg[best] || (deg[v] == deg[best] && v < best)) best = v;
    }
    for (size_t k = h0; k < order.size(); ++k) level[order[k]] = -1;
    ecc = last;
    return best;
  };
  for (int s0 = 0; s0 < n; ++s0) {
    if (vis[s0]) continue;
    // George-Liu: up to four BFS passes, each from the min-degree node of the
    // previous pass's last level, while the eccentricity grows; the order
    // starts from the last start that did not increase it.  A pass from a
    // candidate start is the Cuthill-McKee traversal itself, kept when the
    // search stops there.
    int ecc;
    int s = bfs_last_min(s0, ecc);
    for (int it = 1;; ++it) {
      const size_t h0 = order.size();
      int e2;
      const int cand = cm_from(s, e2);
      if (e2 <= ecc || it == 4) break;  // the fourth pass's start is taken unchecked
      for (size_t k = h0; k < order.size(); ++k) vis[order[k]] = 0;  // undo
      order.resize(h0);
      ecc = e2;
      s = cand;
    }
  }
  std::reverse(order.begin(), order.end());
}

// Ascending order of distinct indices: a bitmap scan over their range when
// it is compact (typical for mesh numberings), otherwise a comparison sort.
static void sort_distinct(std::vector<int> &v, std::vector<unsigned long long> &bits) {
  if (v.empty()) return;
  int lo = v[0], hi = v[0];
  for (int g : v) {
    lo = std::min(lo, g);
    hi = std::max(hi, g);
  }
  const long long range = (long long)hi - lo + 1;
  if (range > 64LL * (long long)v.size()) {
    std::sort(v.begin(), v.end());
    return;
  }
  const size_t nw = (size_t)((range + 63) / 64);
  bits.assign(nw, 0ULL);
  for (int g : v) bits[(g - lo) >> 6] |= 1ULL << ((g - lo) & 63);
  size_t k = 0;
  for (size_t wi = 0; wi < nw; ++wi) {
    unsigned long long b = bits[wi];
    while (b) {
      v[k++] = lo + (int)(wi * 64) + __builtin_ctzll(b);
      b &= b - 1;
    }
  }
}

// Per-subdomain planning result (built independently, concatenated in order).
struct SubPlan {
  std::vector<int> dofs;                 // local order -> global dof
  std::vector<int> nat;                  // local order -> rank by global index
  std::vector<int> rowlen;               // local CSR row lengths (entries: on the device)
  size_t nloc = 0;                       // local CSR entries
  std::vector<int> tfirst;               // tile profile
  std::vector<int> eptr, uptr;           // envelope segment starts (npad + 1 each)
  bool env_overflow = false;             // envelope beyond 32-bit segment offsets
  std::vector<int> ext;                  // extended region (ascending global)
  std::vector<int> ext_rowlen, ext_src, ext_loc;
  std::vector<int> pair_j, pair_len, pair_l, pair_e;
};

namespace {
struct Scratch {
  // stamp: visit marks (a fresh value per use); loc: -1 between uses.  Kept
  // between planning calls (see scratch_get), indexable up to n_cap.
  std::vector<int> stamp, loc;
  int n_cap = 0;
  int gen = 0;
  RcmWork rcm;
  std::vector<unsigned long long> bits;  // bitmap for ordering a region's dofs
  std::vector<int> tptr, tcol, pos;  // local CSR columns in ascending order, relabelling
  std::vector<int> frontier, next, adj_ptr, adj, order, mincol, fenv;
  std::vector<std::pair<int, int>> row;
  explicit Scratch(int n) : n_cap(n) {
    stamp.assign(n, -1);
    loc.assign(n, -1);
  }
  int next_mark() {  // a stamp value no entry holds yet
    if (gen == INT_MAX) {
      std::fill(stamp.begin(), stamp.end(), -1);
      gen = 0;
    }
    return ++gen;
  }
};

// Workers' scratch, kept between planning calls: a fresh Scratch costs two
// n-sized fills (~1 ms per worker at n = 1M), which would otherwise delay
// every worker's first region.  At most kScratchCap bytes are kept.
constexpr size_t kScratchCap = size_t(1) << 30;
struct ScratchCache {
  std::mutex mu;
  std::vector<std::unique_ptr<Scratch>> free;
  size_t held = 0;
};
ScratchCache &scratch_cache() {
  static ScratchCache *c = new ScratchCache();  // never destroyed (see block_cache)
  return *c;
}
size_t scratch_bytes(const Scratch &s) { return 2 * (size_t)s.n_cap * sizeof(int); }
std::unique_ptr<Scratch> scratch_get(int n) {
  {
    ScratchCache &c = scratch_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    for (size_t k = c.free.size(); k-- > 0;)
      if (c.free[k]->n_cap >= n) {
        std::unique_ptr<Scratch> s = std::move(c.free[k]);
        c.free.erase(c.free.begin() + k);
        c.held -= scratch_bytes(*s);
        return s;
      }
  }
  return std::unique_ptr<Scratch>(new Scratch(n));
}
// Returns a Scratch whose loc entries are all -1 again.
void scratch_put(std::unique_ptr<Scratch> s) {
  ScratchCache &c = scratch_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (c.held + scratch_bytes(*s) > kScratchCap) return;  // freed here
  c.held += scratch_bytes(*s);
  c.free.push_back(std::move(s));
}
}  // namespace

void scratch_release() {
  ScratchCache &c = scratch_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.free.clear();
  c.held = 0;
}

#ifdef AMSP_PLAN_PROFILE
#include <chrono>
static double g_sec[8];
#define SEC(k) do { auto t_ = std::chrono::steady_clock::now(); g_sec[k] += std::chrono::duration<double, std::milli>(t_ - ts_).count(); ts_ = t_; } while (0)
#else
#define SEC(k) do { } while (0)
#endif

// ZV: A may store off-diagonal zeros (read each visited entry's value).
template <bool ZV>
static void plan_region(int i, const amsp_csr *A, const std::vector<int> &core_ptr,
                        const std::vector<int> &core, int nev, const amsp_options &opt,
                        Scratch &S, SubPlan &out) {
#ifdef AMSP_PLAN_PROFILE
  auto ts_ = std::chrono::steady_clock::now();
#endif
  const int64_t *rp = A->row_ptr;
  const int32_t *ci = A->col_idx;
  const double *va = A->val;
  const int delta = opt.overlap;
  std::vector<int> region(core.begin() + core_ptr[i], core.begin() + core_ptr[i + 1]);
  const int mark = S.next_mark();
  for (int g : region) S.stamp[g] = mark;
  S.frontier = region;
  const int layers = delta;
  size_t region_size = region.size();
  for (int d = 0; d < layers; ++d) {
    S.next.clear();
    const int nf = (int)S.frontier.size();
    for (int f = 0; f < nf; ++f) {
      const int g = S.frontier[f];
      // the rows ahead are mostly first touches of A: fetch them early
      if (f + 16 < nf) __builtin_prefetch(ci + rp[S.frontier[f + 16]]);
      for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
        const int c = ci[e];
        // the stamp test first: most neighbours are already in the region,
        // and it spares the read of the value
        if (c != g && S.stamp[c] != mark && (!ZV || va[e] != 0.0)) {
          S.stamp[c] = mark;
          S.next.push_back(c);
        }
      }
    }
    region.insert(region.end(), S.next.begin(), S.next.end());
    if (d == delta - 1) region_size = region.size();
    S.frontier.swap(S.next);
  }
  region.resize(region_size);
  sort_distinct(region, S.bits);
  SEC(0);
  const int ni = (int)region.size();
  std::vector<int> &loc = S.loc;
  for (int k = 0; k < ni; ++k) loc[region[k]] = k;
  // one pass over the region's rows of A (ascending order): the local CSR
  // columns in that order (tcol, diagonal included) and, when A may store
  // off-diagonal zeros, the adjacency for the ordering (off-diagonal, nonzero
  // values).  Without such zeros the ordering takes tcol itself: every row
  // lists itself once (the diagonal is present), which the searches skip as
  // already visited and which adds one to every degree, so the order is the
  // same.
  if (ZV) {
    S.adj_ptr.assign(ni + 1, 0);
    S.adj.clear();
  }
  S.tptr.assign(ni + 1, 0);
  S.tcol.clear();
  for (int k = 0; k < ni; ++k) {
    const int g = region[k];
    for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
      const int c = ci[e];
      const int lc = loc[c];
      if (lc < 0) continue;
      S.tcol.push_back(lc);
      if (ZV && c != g && va[e] != 0.0) S.adj.push_back(lc);
    }
    if (ZV) S.adj_ptr[k + 1] = (int)S.adj.size();
    S.tptr[k + 1] = (int)S.tcol.size();
  }
  SEC(1);
  if (opt.local_order == AMSP_ORDER_RCM) {
    if (ZV)
      rcm_order(S.adj_ptr, S.adj, S.order, S.rcm);
    else
      rcm_order(S.tptr, S.tcol, S.order, S.rcm);
  } else {
    S.order.resize(ni);
    for (int k = 0; k < ni; ++k) S.order[k] = k;
  }
  SEC(2);
  // relabel to the chosen order: pos[ascending index] = local index
  S.pos.resize(ni);
  out.dofs.resize(ni);
  out.nat.resize(ni);
  for (int k = 0; k < ni; ++k) {
    out.dofs[k] = region[S.order[k]];
    out.nat[k] = S.order[k];  // region is ascending, so its index is the rank
    S.pos[S.order[k]] = k;
  }
  // row lengths and each row's first local column in the chosen order (the
  // entries themselves, sorted by local column, are built on the device
  // from the same rule: the row's matrix entries whose column is in the region)
  S.mincol.assign(ni, 0);
  out.rowlen.resize(ni);
  for (int k = 0; k < ni; ++k) {
    const int j = S.order[k];
    int mc = k;
    for (int e = S.tptr[j]; e < S.tptr[j + 1]; ++e) mc = std::min(mc, S.pos[S.tcol[e]]);
    S.mincol[k] = mc;
    out.rowlen[k] = S.tptr[j + 1] - S.tptr[j];
  }
  out.nloc = S.tcol.size();
  SEC(3);
  const int nt = (ni + TS - 1) / TS;
  out.tfirst.resize(nt);
  for (int I = 0; I < nt; ++I) {
    int f = I;
    if (opt.dense_tiles) {
      f = 0;
    } else {
      for (int k = I * TS; k < std::min(ni, (I + 1) * TS); ++k) f = std::min(f, S.mincol[k] / TS);
    }
    out.tfirst[I] = f;
  }
  // Envelope of the factor below the diagonal tiles.  Cholesky fill stays
  // right of each row's first entry; fenv[r] = min over rows s >= r of that
  // first column (padding rows: s itself) is nondecreasing, so that
  //   row form:    row r of block I keeps columns fenv[r] .. 64I - 1,
  //   column form: column c of block J keeps rows 64(J+1) .. last(c), with
  //                last(c) = max{ r : fenv[r] <= c },
  // both contiguous and holding the same entries.
  const int npad = nt * TS;
  S.fenv.resize(npad);
  int m = npad;
  for (int r = npad - 1; r >= 0; --r) {
    const int f = r >= ni ? r : (opt.dense_tiles ? 0 : S.mincol[r]);
    m = std::min(m, f);
    S.fenv[r] = m;
  }
  out.eptr.resize(npad + 1);
  out.uptr.resize(npad + 1);
  out.eptr[0] = out.uptr[0] = 0;
  long long er = 0, eu = 0;
  int last = 0;  // max r with fenv[r] <= c (fenv[0] = 0 <= c always)
  for (int r = 0; r < npad; ++r) {
    er += std::max(0, (r / TS) * TS - S.fenv[r]);
    const int c = r;
    while (last + 1 < npad && S.fenv[last + 1] <= c) ++last;
    eu += std::max(0, last - (c / TS + 1) * TS + 1);
    out.eptr[r + 1] = (int)std::min<long long>(er, INT_MAX);
    out.uptr[r + 1] = (int)std::min<long long>(eu, INT_MAX);
  }
  out.env_overflow = er >= INT_MAX;
  SEC(4);
  for (int k = 0; k < ni; ++k) loc[region[k]] = -1;
}

// Extended region of subdomain i (its region grown by one more layer) and
// the entries of A coupling each extended row to the region (local indices).
template <bool ZV>
static void plan_ext(int i, const amsp_csr *A, const HostPlan &P, Scratch &S, SubPlan &out) {
  const int64_t *rp = A->row_ptr;
  const int32_t *ci = A->col_idx;
  const double *va = A->val;
  const int r0 = P.sd_ptr[i], ni = P.sd_ptr[i + 1] - r0;
  std::vector<int> &loc = S.loc;
  for (int k = 0; k < ni; ++k) loc[P.sd_dofs[r0 + k]] = k;
  out.ext.assign(P.sd_dofs.begin() + r0, P.sd_dofs.begin() + r0 + ni);
  const int mark = S.next_mark();
  for (int k = 0; k < ni; ++k) {
    const int g = P.sd_dofs[r0 + k];
    for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
      const int c = ci[e];
      if (c != g && loc[c] < 0 && S.stamp[c] != mark && (!ZV || va[e] != 0.0)) {
        S.stamp[c] = mark;
        out.ext.push_back(c);
      }
    }
  }
  sort_distinct(out.ext, S.bits);
  out.ext_rowlen.resize(out.ext.size());
  out.ext_src.clear();
  out.ext_loc.clear();
  out.ext_src.reserve(out.ext.size() * 6);
  out.ext_loc.reserve(out.ext.size() * 6);
  for (size_t q = 0; q < out.ext.size(); ++q) {
    const int g = out.ext[q];
    int cnt = 0;
    for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
      const int c = ci[e];
      if (loc[c] >= 0) {
        out.ext_src.push_back((int)e);
        out.ext_loc.push_back(loc[c]);
        ++cnt;
      }
    }
    out.ext_rowlen[q] = cnt;
  }
  for (int k = 0; k < ni; ++k) loc[P.sd_dofs[r0 + k]] = -1;
}

#ifdef AMSP_PLAN_PROFILE
#include <cstdio>
#define PTIME(label) do { auto t_ = std::chrono::steady_clock::now(); fprintf(stderr, "  %s %.1f ms\n", label, std::chrono::duration<double, std::milli>(t_ - tp_).count()); tp_ = t_; } while (0)
#define PSTART auto tp_ = std::chrono::steady_clock::now()
#else
#define PTIME(label) do { } while (0)
#define PSTART do { } while (0)
#endif


int build_plan_local(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
                     const amsp_options &opt, HostPlan &P, std::string &msg) {
  PSTART;
  const int n = (int)A->n;
  const int N = nparts;
  P.n = n;
  P.N = N;
  P.nev = nev;
  // cores: the dofs of each part in ascending order (counting sort of the
  // partition; in parallel over row chunks, each chunk's rows placed after
  // those of the chunks before it)
  std::vector<int> core_ptr(N + 1, 0), core(n);
  const int nch = N <= 16384 ? std::max(1, std::min(64, n / 16384)) : 1;
  {
    std::vector<int> cnt((size_t)nch * N, 0);
    auto rows = [&](int c, int &a, int &b) {
      a = (int)((long long)n * c / nch);
      b = (int)((long long)n * (c + 1) / nch);
    };
    parallel_for(nch, [&](int c) {
      int a, b;
      rows(c, a, b);
      int *h = cnt.data() + (size_t)c * N;
      for (int j = a; j < b; ++j) h[part[j]]++;
    });
    int run = 0;
    for (int i = 0; i < N; ++i) {
      core_ptr[i] = run;
      for (int c = 0; c < nch; ++c) {
        const int x = cnt[(size_t)c * N + i];
        cnt[(size_t)c * N + i] = run;
        run += x;
      }
    }
    core_ptr[N] = run;
    parallel_for(nch, [&](int c) {
      int a, b;
      rows(c, a, b);
      int *at = cnt.data() + (size_t)c * N;
      for (int j = a; j < b; ++j) core[at[part[j]]++] = j;
    });
  }
  std::vector<SubPlan> sub(N);
  {
    parallel_for(N, [&](int i) {
      auto sc = scratch_get(n);
      if (P.offdiag_zeros)
        plan_region<true>(i, A, core_ptr, core, nev, opt, *sc, sub[i]);
      else
        plan_region<false>(i, A, core_ptr, core, nev, opt, *sc, sub[i]);
      scratch_put(std::move(sc));
    });
  }
  PTIME("regions");
  for (int i = 0; i < N; ++i)
    if (sub[i].env_overflow) {
      msg = "region " + std::to_string(i) + " too large: its factor envelope exceeds 2^31 entries";
      return AMSP_ERR_ARG;
    }
#ifdef AMSP_PLAN_PROFILE
  fprintf(stderr, "   grow+sort %.1f adj %.1f rcm %.1f lcsr %.1f env %.1f (thread-summed ms)\n", g_sec[0], g_sec[1], g_sec[2], g_sec[3], g_sec[4]);
  for (double &x : g_sec) x = 0;
#endif
  P.sd_ptr.assign(N + 1, 0);
  P.vp_ptr.assign(N + 1, 0);
  P.trow_ptr.assign(N + 1, 0);
  P.mi.assign(N, 0);
  P.coff.assign(N + 1, 0);
  std::vector<size_t> loc_off(N + 1, 0);
  std::vector<long long> tile_off(N + 1, 0);
  for (int i = 0; i < N; ++i) {
    const int ni = (int)sub[i].dofs.size();
    const int nt = (int)sub[i].tfirst.size();
    P.sd_ptr[i + 1] = P.sd_ptr[i] + ni;
    P.vp_ptr[i + 1] = P.vp_ptr[i] + nt * TS;
    P.trow_ptr[i + 1] = P.trow_ptr[i] + nt;
    P.mi[i] = std::min(nev, ni);
    P.coff[i + 1] = P.coff[i] + P.mi[i];
    loc_off[i + 1] = loc_off[i] + sub[i].nloc;
    long long t = 0;
    for (int I = 0; I < nt; ++I) t += I - sub[i].tfirst[I] + 1;
    tile_off[i + 1] = tile_off[i] + t;
  }
  const int sum_ni = P.sd_ptr[N];
  P.sd_dofs.resize(sum_ni);
  P.nat.resize(sum_ni);
  P.loc_rowptr.resize(sum_ni + 1);
  P.loc_rowptr[0] = 0;
  P.nloc = (long long)loc_off[N];
  P.tfirst.resize(P.trow_ptr[N]);
  P.toff.resize(P.trow_ptr[N]);
  P.ebase.assign(N + 1, 0);
  for (int i = 0; i < N; ++i) P.ebase[i + 1] = P.ebase[i] + sub[i].eptr.back();
  P.eptr.resize((size_t)P.vp_ptr[N] + N);
  P.uptr.resize((size_t)P.vp_ptr[N] + N);
  parallel_for(N, [&](int i) {
    SubPlan &S = sub[i];
    const int r0 = P.sd_ptr[i], ni = (int)S.dofs.size();
    int acc = (int)loc_off[i];
    for (int k = 0; k < ni; ++k) {
      P.sd_dofs[r0 + k] = S.dofs[k];
      P.nat[r0 + k] = S.nat[k];
      acc += S.rowlen[k];
      P.loc_rowptr[r0 + k + 1] = acc;
    }
    const int g0 = P.trow_ptr[i];
    long long t = tile_off[i] - g0;  // off-diagonal tiles of the regions before i
    for (size_t I = 0; I < S.tfirst.size(); ++I) {
      P.tfirst[g0 + I] = S.tfirst[I];
      P.toff[g0 + I] = t;
      t += (long long)I - S.tfirst[I];
    }
    std::copy(S.eptr.begin(), S.eptr.end(), P.eptr.begin() + P.vp_ptr[i] + i);
    std::copy(S.uptr.begin(), S.uptr.end(), P.uptr.begin() + P.vp_ptr[i] + i);
  });
  P.max_ni = 0;
  P.max_npad = 0;
  for (int i = 0; i < N; ++i) {
    P.max_ni = std::max(P.max_ni, P.sd_ptr[i + 1] - P.sd_ptr[i]);
    P.max_npad = std::max(P.max_npad, P.vp_ptr[i + 1] - P.vp_ptr[i]);
  }
  P.ntiles = tile_off[N];
  P.noff = tile_off[N] - P.trow_ptr[N];
  P.nenv = P.ebase[N];
  P.nc = P.coff[N];
  PTIME("concat");
  (void)msg;
  return AMSP_OK;
}

int build_plan_coupling(const amsp_csr *A, const amsp_options &opt, HostPlan &P, std::string &msg) {
  PSTART;
  (void)opt;
  const int n = P.n, N = P.N, nev = P.nev;
  // The multiplicities and the inverse map dof -> (subdomain, local index)
  // are built on the device from the uploaded regions (launch_inverse_map).
  // Every dof lies in the core of its own part, so each has at least one copy.
  P.ext_ptr.assign(N + 1, 0);
  P.ext_rowptr.assign(1, 0);
  P.ext_src.clear();
  P.ext_loc.clear();
  P.pair_i.clear();
  P.pair_j.clear();
  P.pair_ptr.assign(1, 0);
  P.pair_l.clear();
  P.pair_e.clear();
  if (nev == 0 || P.nc == 0) return AMSP_OK;
  std::vector<SubPlan> sub(N);
  {
    parallel_for(N, [&](int i) {
      auto sc = scratch_get(n);
      if (P.offdiag_zeros)
        plan_ext<true>(i, A, P, *sc, sub[i]);
      else
        plan_ext<false>(i, A, P, *sc, sub[i]);
      scratch_put(std::move(sc));
    });
  }
  std::vector<size_t> exs_off(N + 1, 0);
  for (int i = 0; i < N; ++i) {
    P.ext_ptr[i + 1] = P.ext_ptr[i] + (int)sub[i].ext.size();
    exs_off[i + 1] = exs_off[i] + sub[i].ext_src.size();
  }
  P.ext_rowptr.resize(P.ext_ptr[N] + 1);
  P.ext_rowptr[0] = 0;
  P.ext_src.resize(exs_off[N]);
  P.ext_loc.resize(exs_off[N]);
  ivec ext_dofs;
  ext_dofs.resize(P.ext_ptr[N]);
  parallel_for(N, [&](int i) {
    SubPlan &S = sub[i];
    const int x0 = P.ext_ptr[i];
    int eacc = (int)exs_off[i];
    for (size_t q = 0; q < S.ext.size(); ++q) {
      ext_dofs[x0 + q] = S.ext[q];
      eacc += S.ext_rowlen[q];
      P.ext_rowptr[x0 + q + 1] = eacc;
    }
    std::copy(S.ext_src.begin(), S.ext_src.end(), P.ext_src.begin() + exs_off[i]);
    std::copy(S.ext_loc.begin(), S.ext_loc.end(), P.ext_loc.begin() + exs_off[i]);
    std::vector<int>().swap(S.ext_src);
    std::vector<int>().swap(S.ext_loc);
  });
  PTIME("ext regions");
  // coupled subdomain pairs for A0, grouped by partner subdomain (ascending)
  {
    // every dof's list of (extended region j, index in it), j ascending: the
    // dofs in 64 ranges, each range taking, region by region in ascending
    // order, the part of the region's (ascending) extended set that falls in
    // it; no atomics, and the lists come out sorted
    ivec xcnt, xptr, xj, xe;
    xcnt.resize(n);
    xptr.resize(n + 1);
    const int nrg = 64;
    auto range = [&](int c, int &g0, int &g1) {
      g0 = (int)((long long)n * c / nrg);
      g1 = (int)((long long)n * (c + 1) / nrg);
    };
    auto part_of = [&](int j, int g0, int g1, int &a, int &b) {
      const int *x0 = ext_dofs.data() + P.ext_ptr[j], *x1 = ext_dofs.data() + P.ext_ptr[j + 1];
      a = b = 0;
      if (x0 == x1 || x1[-1] < g0 || x0[0] >= g1) return;
      a = (int)(std::lower_bound(x0, x1, g0) - x0);
      b = (int)(std::lower_bound(x0 + a, x1, g1) - x0);
    };
    parallel_for(nrg, [&](int c) {
      int g0, g1;
      range(c, g0, g1);
      std::fill(xcnt.begin() + g0, xcnt.begin() + g1, 0);
      for (int j = 0; j < N; ++j) {
        int a, b;
        part_of(j, g0, g1, a, b);
        const int *x = ext_dofs.data() + P.ext_ptr[j];
        for (int e = a; e < b; ++e) xcnt[x[e]]++;
      }
    });
    exclusive_scan(xcnt, xptr, n);
    xj.resize(ext_dofs.size());
    xe.resize(ext_dofs.size());
    parallel_for(nrg, [&](int c) {
      int g0, g1;
      range(c, g0, g1);
      std::fill(xcnt.begin() + g0, xcnt.begin() + g1, 0);
      for (int j = 0; j < N; ++j) {
        int a, b;
        part_of(j, g0, g1, a, b);
        const int *x = ext_dofs.data() + P.ext_ptr[j];
        for (int e = a; e < b; ++e) {
          const int g = x[e];
          const int at = xptr[g] + xcnt[g]++;
          xj[at] = j;
          xe[at] = e;
        }
      }
    });
    std::mutex mu;
    std::vector<std::unique_ptr<std::vector<int>>> slots;
    parallel_for(N, [&](int i) {
      SubPlan &S = sub[i];
      if (P.mi[i] == 0) return;
      std::unique_ptr<std::vector<int>> sl;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (!slots.empty()) {
          sl = std::move(slots.back());
          slots.pop_back();
        }
      }
      if (!sl) sl.reset(new std::vector<int>(N, -1));
      std::vector<int> &slot = *sl;
      std::vector<int> js, counts;
      for (int k = P.sd_ptr[i]; k < P.sd_ptr[i + 1]; ++k) {
        const int g = P.sd_dofs[k];
        for (int q = xptr[g]; q < xptr[g + 1]; ++q) {
          const int j = xj[q];
          if (P.mi[j] == 0) continue;
          if (slot[j] < 0) {
            slot[j] = (int)js.size();
            js.push_back(j);
            counts.push_back(0);
          }
          counts[slot[j]]++;
        }
      }
      std::vector<int> order(js.size());
      for (size_t u = 0; u < js.size(); ++u) order[u] = (int)u;
      std::sort(order.begin(), order.end(), [&](int a, int b) { return js[a] < js[b]; });
      std::vector<int> start(js.size());
      int tot = 0;
      for (int u : order) {
        start[u] = tot;
        tot += counts[u];
        S.pair_j.push_back(js[u]);
        S.pair_len.push_back(counts[u]);
      }
      S.pair_l.resize(tot);
      S.pair_e.resize(tot);
      for (int k = P.sd_ptr[i]; k < P.sd_ptr[i + 1]; ++k) {
        const int g = P.sd_dofs[k];
        for (int q = xptr[g]; q < xptr[g + 1]; ++q) {
          const int j = xj[q];
          if (P.mi[j] == 0) continue;
          const int at = start[slot[j]]++;
          S.pair_l[at] = k - P.sd_ptr[i];
          S.pair_e[at] = xe[q];
        }
      }
      for (int j : js) slot[j] = -1;
      std::lock_guard<std::mutex> lk(mu);
      slots.push_back(std::move(sl));
    });
    std::vector<size_t> poff(N + 1, 0), eoff(N + 1, 0);
    for (int i = 0; i < N; ++i) {
      poff[i + 1] = poff[i] + sub[i].pair_j.size();
      eoff[i + 1] = eoff[i] + sub[i].pair_l.size();
    }
    P.pair_i.resize(poff[N]);
    P.pair_j.resize(poff[N]);
    P.pair_ptr.resize(poff[N] + 1);
    P.pair_ptr[0] = 0;
    P.pair_l.resize(eoff[N]);
    P.pair_e.resize(eoff[N]);
    parallel_for(N, [&](int i) {
      SubPlan &S = sub[i];
      size_t acc = eoff[i];
      for (size_t q = 0; q < S.pair_j.size(); ++q) {
        P.pair_i[poff[i] + q] = i;
        P.pair_j[poff[i] + q] = S.pair_j[q];
        acc += S.pair_len[q];
        P.pair_ptr[poff[i] + q + 1] = (int)acc;
      }
      std::copy(S.pair_l.begin(), S.pair_l.end(), P.pair_l.begin() + eoff[i]);
      std::copy(S.pair_e.begin(), S.pair_e.end(), P.pair_e.begin() + eoff[i]);
    });
  }
  PTIME("pairs");
  return AMSP_OK;
}

int build_plan(const amsp_csr *A, const int32_t *part, int32_t nparts, int32_t nev,
               const amsp_options &opt, HostPlan &P, std::string &msg) {
  int s = build_plan_local(A, part, nparts, nev, opt, P, msg);
  if (s != AMSP_OK) return s;
  return build_plan_coupling(A, opt, P, msg);
}

}  // namespace amsp
