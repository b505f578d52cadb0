// Serving loop: requests (a subscription set and an update set each) arrive
// at any time and are matched concurrently on one GPU (an addition to the
// paper; each request is the problem of Sec. III solved as in Algorithm 5).
//
// Host side only.  A pool of worker threads, each with its own HIP stream,
// takes requests from one FIFO as soon as the device-memory budget admits
// them; requests therefore start the moment a worker and memory free up and
// their kernels overlap on the device with those of the requests already
// running.  A worker that takes a small request also takes the small
// requests queued behind it (up to batch_max) and matches them together
// with the batched kernels (continuous batching: whatever has arrived by the
// time a worker frees up joins the next launch).  The footprint of a
// request is charged in two steps: inputs + trees + match scratch at
// admission (known from n, m, d), then the predicted output (the learned
// slot arena) and the exact output once the match has sized them.  A
// request that would exceed the budget waits, except the oldest request in
// flight, which always proceeds, so the loop cannot deadlock.
//
// Trees named by a nonzero key stay resident after their request (LRU), and
// a later request with the same key matches against the resident tree
// without rebuilding it.  Results are copied into a pinned host pool (or
// kept on the device) and handed to the client through a completion queue.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ddm_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// first-fit allocator over one pinned host block
struct HostPool {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  size_t used = 0;
  bool init(size_t bytes) {
    size = (bytes + 4095) & ~size_t(4095);
    if (size == 0) return true;
    if (hipHostMalloc((void**)&base, size, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      base = nullptr;
      return false;
    }
    free_[0] = size;
    return true;
  }
  char* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used += bytes;
      return base + off;
    }
    return nullptr;
  }
  void release(char* p, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    size_t off = (size_t)(p - base);
    used -= bytes;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + bytes == nx->first) {
      bytes += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        pv->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
};

struct CachedTree {
  ddm_tree* t = nullptr;
  uint64_t bytes = 0;
  int users = 0;
  std::list<uint64_t>::iterator lru;
};

}  // namespace

struct ddm_server_req {
  uint64_t ticket = 0;
  ddm_request r{};
  hipEvent_t ready = nullptr;
  int64_t t_arrival = 0, t_start = 0, t_done = 0;
  uint64_t charged = 0;  // bytes charged to the budget
  int32_t status = 1;    // 1 pending, else a ddm_status
  std::string detail;
  uint64_t K = 0, slots = 0;
  uint32_t overflowed = 0;
  char* host = nullptr;  // pinned result
  uint64_t host_bytes = 0;
  bool compact = false;
  uint64_t* dev = nullptr;
  bool tree_cached = false;
};

struct ddm_server {
  int device = 0;
  ddm_server_opts o{};
  ddm_predictor* pred = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_mem, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<ddm_server_req*> queue;                    // not yet admitted
  std::unordered_map<uint64_t, ddm_server_req*> reqs;  // every unreleased request
  std::vector<uint64_t> done;                           // completion queue
  std::map<uint64_t, int> in_flight;                    // ticket -> 1
  uint64_t used = 0, peak = 0;
  uint32_t waiting = 0;          // requests in flight blocked in charge()
  std::set<uint64_t> yieldable;  // tickets blocked in charge() that may yield
  uint64_t submitted = 0, completed = 0;
  uint64_t yields = 0;  // requests that gave their memory back and were requeued
  HostPool pool;
  std::unordered_map<uint64_t, CachedTree> trees;
  std::list<uint64_t> lru;  // front = most recent
  std::vector<std::thread> workers;
};

namespace ddm {
size_t tree_bytes_estimate(uint32_t n, uint32_t d);
size_t match_stash_bytes(uint32_t m);
}

using namespace ddm;

namespace {

uint64_t admission_bytes(const ddm_request& r, bool build) {
  // inputs (already in device memory, held until the request completes),
  // the tree unless it is resident, and the match scratch (per update: probe
  // words, order, counts, offsets, lists; plus the bucket tables; and the
  // count traversal's stash of hits)
  uint64_t b = 8ull * r.d * ((uint64_t)r.n + r.m);
  if (build) b += tree_bytes_estimate(r.n, r.d);
  b += 64ull * r.m + (1u << 20);
  if (r.d > 1) b += match_stash_bytes(r.m);
  return b;
}

// Charge `bytes` to the budget, waiting until they fit.  A request alone in
// flight goes ahead even past the budget (nothing else could free memory for
// it).  When every request in flight is waiting here, none can free memory
// for the others: the youngest of those that may yield (may_yield: it can
// still give back everything it holds and start again) returns false
// without charging anything; if none may, the oldest goes ahead past the
// budget.  So the budget is exceeded only by a request that alone needs more,
// or when no waiting request can yield.  Called with the lock held.
bool charge(ddm_server* S, std::unique_lock<std::mutex>& lk, ddm_server_req* q, uint64_t bytes,
            bool may_yield = false) {
  ++S->waiting;
  if (may_yield) S->yieldable.insert(q->ticket);
  S->cv_mem.notify_all();  // the others may be waiting for everyone to wait
  bool yield = false;
  S->cv_mem.wait(lk, [&] {
    if (S->stop || S->used + bytes <= S->o.hbm_budget || S->in_flight.size() <= 1) return true;
    if (S->waiting < S->in_flight.size()) return false;  // a request is still running
    if (!S->yieldable.empty()) {
      if (may_yield && *S->yieldable.rbegin() == q->ticket) {
        yield = true;
        return true;
      }
      return false;
    }
    return S->in_flight.begin()->first == q->ticket;
  });
  --S->waiting;
  if (may_yield) S->yieldable.erase(q->ticket);
  if (yield) {
    S->cv_mem.notify_all();
    return false;
  }
  S->used += bytes;
  q->charged += bytes;
  if (S->used > S->peak) S->peak = S->used;
  return true;
}

void uncharge(ddm_server* S, ddm_server_req* q, uint64_t bytes) {
  S->used -= bytes;
  q->charged -= bytes;
  S->cv_mem.notify_all();
}

void finish(ddm_server* S, ddm_server_req* q, int32_t st, const std::string& detail) {
  std::lock_guard<std::mutex> lk(S->mu);
  q->status = st;
  q->detail = detail;
  q->t_done = now_ns();
  S->in_flight.erase(q->ticket);
  S->done.push_back(q->ticket);
  ++S->completed;
  S->cv_mem.notify_all();
  S->cv_work.notify_all();
  S->cv_done.notify_all();
}

// compact form of K sorted keys of m updates: the subscription ids and the
// offsets of every update's pairs
__global__ void compact_ids_kernel(const uint64_t* __restrict__ keys, uint64_t K,
                                   uint32_t* __restrict__ ids) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) ids[i] = (uint32_t)keys[i];
}

__global__ void compact_offsets_kernel(const uint64_t* __restrict__ keys, uint64_t K, uint32_t m,
                                       uint64_t* __restrict__ off) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > m) return;
  const uint64_t x = (uint64_t)j << 32;
  uint64_t lo = 0, hi = K;  // first key >= x
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (keys[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  off[j] = lo;
}

uint64_t host_result_bytes(bool compact, uint64_t K, uint32_t m) {
  if (!compact) return 8 * std::max<uint64_t>(K, 1);
  return ((4 * K + 7) & ~uint64_t(7)) + 8 * ((uint64_t)m + 1);
}

// Copies the K keys at `keys` (device, ordered on s) of request q into a
// slot of the pinned pool, as keys or in compact form; waits for the copy.
ddm_status deliver_host(ddm_server* S, ddm_server_req* q, const uint64_t* keys, uint64_t K,
                        hipStream_t s, std::string* why) {
  const bool compact = S->o.compact != 0;
  const uint64_t bytes = host_result_bytes(compact, K, q->r.m);
  char* host = nullptr;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if (bytes <= S->pool.size)
      S->cv_mem.wait(lk, [&] { return S->stop || (host = S->pool.alloc(bytes)) != nullptr; });
  }
  if (!host) {
    *why = bytes > S->pool.size ? "result larger than the pinned host pool" : "server stopped";
    return bytes > S->pool.size ? DDM_E_CAPACITY : DDM_E_INVALID_ARG;
  }
  q->host = host;
  q->host_bytes = bytes;
  q->compact = compact;
  hipError_t e = hipSuccess;
  char* tmp = nullptr;
  if (!compact) {
    if (K) e = hipMemcpyAsync(host, keys, 8 * K, hipMemcpyDeviceToHost, s);
  } else {
    tmp = dev_alloc(bytes, s);
    if (!tmp) {
      *why = "device allocation of a compact result failed";
      return DDM_E_NOMEM;
    }
    const uint64_t ids_bytes = (4 * K + 7) & ~uint64_t(7);
    if (K) {
      compact_ids_kernel<<<(unsigned)((K + 255) / 256), 256, 0, s>>>(keys, K, (uint32_t*)tmp);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      compact_offsets_kernel<<<(q->r.m + 1 + 255) / 256, 256, 0, s>>>(keys, K, q->r.m,
                                                                        (uint64_t*)(tmp + ids_bytes));
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, bytes, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (tmp) dev_free(tmp, s);
  if (e != hipSuccess) return hip_fail(e, "result copy", __FILE__, __LINE__);
  return DDM_OK;
}

ddm_status process(ddm_server* S, ddm_server_req* q, hipStream_t s, std::string* why,
                   bool* yielded = nullptr) {
  const ddm_request& r = q->r;
  auto fail = [&](ddm_status st) {
    *why = ddm_last_error_detail();
    return st;
  };
  if (q->ready) DDM_HIP(hipStreamWaitEvent(s, q->ready, 0));
  ddm_tree* t = nullptr;
  bool from_cache = false;
  if (r.tree_key) {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->trees.find(r.tree_key);
    if (it != S->trees.end()) {
      t = it->second.t;
      ++it->second.users;
      S->lru.erase(it->second.lru);
      S->lru.push_front(r.tree_key);
      it->second.lru = S->lru.begin();
      from_cache = true;
    }
  }
  if (!t) {
    if (!r.sub_lo && r.tree_key) {
      *why = "request names a tree key that is not resident and gives no subscriptions";
      return DDM_E_INVALID_ARG;
    }
    ddm_status st = ddm_build(r.sub_lo, r.sub_hi, r.n, r.d, s, &t);
    if (st != DDM_OK) return fail(st);
  }
  // The tree is given back (or cached) only once the stream has finished
  // with it: a cached tree may be evicted, or used by another worker, as
  // soon as it is handed over.
  auto drop_tree = [&]() {
    (void)hipStreamSynchronize(s);
    std::lock_guard<std::mutex> lk(S->mu);
    if (from_cache) {
      auto it = S->trees.find(r.tree_key);
      --it->second.users;
      return;
    }
    if (r.tree_key && S->o.tree_cache > 0 && S->trees.find(r.tree_key) == S->trees.end()) {
      CachedTree c;
      c.t = t;
      c.bytes = tree_bytes_estimate(r.n, r.d);
      S->lru.push_front(r.tree_key);
      c.lru = S->lru.begin();
      S->trees[r.tree_key] = c;
      // the tree's bytes move from the request to the cache
      q->charged -= std::min<uint64_t>(q->charged, c.bytes);
      q->tree_cached = true;
      while (S->trees.size() > S->o.tree_cache) {
        uint64_t victim = 0;
        for (auto it = S->lru.rbegin(); it != S->lru.rend(); ++it)
          if (S->trees[*it].users == 0) {
            victim = *it;
            break;
          }
        if (!victim) break;
        CachedTree& v = S->trees[victim];
        S->lru.erase(v.lru);
        S->used -= v.bytes;
        ddm_tree_free(v.t);
        S->trees.erase(victim);
        S->cv_mem.notify_all();
      }
      return;
    }
    ddm_tree_free(t);
  };
  uint32_t tn = 0, td = 0;
  (void)ddm_tree_info(t, &tn, &td, nullptr);
  if (td != r.d) {
    drop_tree();
    *why = "the resident tree has another dimension than the request";
    return DDM_E_INVALID_ARG;
  }
  if (r.m == 0 || tn == 0) {
    // still validate the inputs that exist
    ddm_status st = ddm_tree_check(t);
    drop_tree();
    q->K = 0;
    return st == DDM_OK ? DDM_OK : fail(st);
  }
  ddm_match_opts mo{};
  mo.traversal = DDM_TRAVERSE_AUTO;
  ddm_pending* pend = nullptr;
  uint64_t K = 0;
  ddm_status st;
  const bool learned = S->pred && r.d <= 3 && r.d > 1;
  uint64_t held = 0;  // bytes charged for the slot arena and the output
  if (learned) {
    // Once the predicted number of slots P is known, and before the match
    // allocates its arena, the arena (4P bytes: a 4-byte id per slot) and an
    // estimate of the output (8P bytes of keys) are charged together
    // (waiting like any other charge), so that a request that got past this
    // point rarely waits again.
    bool refused = false;
    const ArenaGrant grant = [&](uint64_t want) -> uint64_t {
      std::unique_lock<std::mutex> lk(S->mu);
      if (!charge(S, lk, q, 12 * std::max<uint64_t>(want, 1), yielded != nullptr)) {
        refused = true;
        return kArenaRefused;
      }
      held = 12 * std::max<uint64_t>(want, 1);
      return want;
    };
    st = match_learned_begin_granted(t, r.upd_lo, r.upd_hi, r.m, S->pred, &K, s, &mo, &pend,
                                     grant);
    if (refused) {
      // give everything back and start again later (the worker requeues)
      drop_tree();
      *yielded = true;
      return DDM_OK;
    }
  } else {
    st = ddm_match_begin(t, r.upd_lo, r.upd_hi, r.m, &K, s, &mo, &pend);
  }
  if (st != DDM_OK) {
    if (held) {
      std::lock_guard<std::mutex> lk(S->mu);
      uncharge(S, q, held);
    }
    drop_tree();
    return fail(st);
  }
  uint64_t slots = 0, arena = 0;
  uint32_t ovf = 0;
  if (pend) (void)ddm_pending_info(pend, &slots, &arena, &ovf);
  q->K = K;
  q->slots = slots;
  q->overflowed = ovf;
  const uint64_t out_bytes = 8 * std::max<uint64_t>(K, 1);
  const uint64_t arena_bytes = learned ? 4 * std::max<uint64_t>(arena, 1) : 0;
  {
    // the charge becomes the arena actually allocated plus the exact output
    std::unique_lock<std::mutex> lk(S->mu);
    const uint64_t need = arena_bytes + out_bytes;
    if (need <= held) {
      uncharge(S, q, held - need);
    } else if (!charge(S, lk, q, need - held, yielded != nullptr)) {
      uncharge(S, q, held);
      lk.unlock();
      ddm_match_abort(pend);
      drop_tree();
      *yielded = true;
      return DDM_OK;
    }
    held = need;
  }
  uint64_t* out = (uint64_t*)dev_alloc(out_bytes, s);
  if (!out) {
    ddm_match_abort(pend);
    drop_tree();
    std::lock_guard<std::mutex> lk(S->mu);
    uncharge(S, q, held);
    *why = "device allocation of the result failed";
    return DDM_E_NOMEM;
  }
  st = ddm_match_finish(pend, out, K);
  if (st != DDM_OK) {
    drop_tree();
    dev_free((char*)out, s);
    std::lock_guard<std::mutex> lk(S->mu);
    uncharge(S, q, held);
    return fail(st);
  }
  if (S->o.deliver_device) {
    // the result stays in device memory (charged until released); the
    // arena is gone
    drop_tree();
    q->dev = out;
    std::lock_guard<std::mutex> lk(S->mu);
    uncharge(S, q, arena_bytes);
    return DDM_OK;
  }
  st = deliver_host(S, q, out, K, s, why);
  drop_tree();
  dev_free((char*)out, s);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    uncharge(S, q, held);
  }
  return st;
}

bool batchable(const ddm_server* S, const ddm_request& r) {
  return S->o.batch_max > 1 && r.tree_key == 0 && r.n > 0 && r.m > 0 && r.n < (1u << 20) &&
         (uint64_t)r.n + r.m <= S->o.batch_small && r.sub_lo && r.sub_hi;
}

// Small requests admitted together are matched as one batch (one tree build,
// one probe, persistent count and fill traversals over all of them); the
// pairs of each request are its own, bit for bit.  A batch that reports
// invalid coordinates is redone request by request, so that only the
// offending request fails.
void process_batch(ddm_server* S, const std::vector<ddm_server_req*>& G, hipStream_t s,
                   std::vector<ddm_status>* st, std::vector<std::string>* why) {
  const uint32_t count = (uint32_t)G.size();
  st->assign(count, DDM_OK);
  why->assign(count, std::string());
  auto alone = [&]() {
    for (uint32_t i = 0; i < count; ++i) {
      (*st)[i] = process(S, G[i], s, &(*why)[i]);
      if ((*st)[i] != DDM_OK) (void)hipStreamSynchronize(s);
    }
  };
  for (auto* q : G)
    if (q->ready && hipStreamWaitEvent(s, q->ready, 0) != hipSuccess) {
      (void)hipGetLastError();
      return alone();
    }
  std::vector<ddm_batch_instance> inst(count);
  for (uint32_t i = 0; i < count; ++i) {
    const ddm_request& r = G[i]->r;
    inst[i] = ddm_batch_instance{r.sub_lo, r.sub_hi, r.upd_lo, r.upd_hi, r.n, r.m, r.d, 0};
  }
  ddm_batch_opts bo{};
  ddm_batch* b = nullptr;
  if (ddm_batch_create(inst.data(), count, nullptr, 0, &bo, &b) != DDM_OK) return alone();
  std::vector<uint64_t> ranges(count + 1);
  uint64_t total = 0;
  ddm_status r = ddm_batch_count(b, s, &total, ranges.data());
  if (r != DDM_OK) {
    ddm_batch_free(b);
    return alone();
  }
  const uint64_t out_bytes = 8 * std::max<uint64_t>(total, 1);
  {
    std::unique_lock<std::mutex> lk(S->mu);
    charge(S, lk, G[0], out_bytes);
  }
  uint64_t* out = (uint64_t*)dev_alloc(out_bytes, s);
  if (!out) {
    ddm_batch_free(b);
    std::lock_guard<std::mutex> lk(S->mu);
    uncharge(S, G[0], out_bytes);
    for (uint32_t i = 0; i < count; ++i) {
      (*st)[i] = DDM_E_NOMEM;
      (*why)[i] = "device allocation of a batch result failed";
    }
    return;
  }
  r = ddm_batch_fill(b, out, total, s);
  if (r == DDM_OK && !S->o.deliver_device) {
    for (uint32_t i = 0; i < count; ++i) {
      ddm_server_req* q = G[i];
      q->K = ranges[i + 1] - ranges[i];
      (*st)[i] = deliver_host(S, q, out + ranges[i], q->K, s, &(*why)[i]);
    }
  } else if (r == DDM_OK) {
    // device delivery: every request gets its own copy of its range
    for (uint32_t i = 0; i < count && r == DDM_OK; ++i) {
      ddm_server_req* q = G[i];
      q->K = ranges[i + 1] - ranges[i];
      const uint64_t bytes = 8 * std::max<uint64_t>(q->K, 1);
      uint64_t* d = (uint64_t*)dev_alloc(bytes, s);
      if (!d) {
        (*st)[i] = DDM_E_NOMEM;
        (*why)[i] = "device allocation of a result failed";
        continue;
      }
      if (q->K && hipMemcpyAsync(d, out + ranges[i], 8 * q->K, hipMemcpyDeviceToDevice, s) !=
                      hipSuccess)
        r = hip_fail(hipGetLastError(), "result copy", __FILE__, __LINE__);
      q->dev = d;
      std::unique_lock<std::mutex> lk(S->mu);
      S->used += bytes;  // held until the request is released
      if (S->used > S->peak) S->peak = S->used;
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess && r == DDM_OK)
    r = hip_fail(hipGetLastError(), "batch", __FILE__, __LINE__);
  ddm_batch_free(b);
  dev_free((char*)out, s);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    uncharge(S, G[0], out_bytes);
  }
  if (r != DDM_OK)
    for (uint32_t i = 0; i < count; ++i)
      if ((*st)[i] == DDM_OK) {
        (*st)[i] = r;
        (*why)[i] = ddm_last_error_detail();
      }
}

void worker_main(ddm_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    s = nullptr;
  }
  std::vector<ddm_server_req*> G;
  std::vector<ddm_status> sts;
  std::vector<std::string> whys;
  while (true) {
    G.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        if (S->stop) return true;
        if (S->queue.empty()) return false;
        ddm_server_req* h = S->queue.front();
        const bool resident = h->r.tree_key && S->trees.count(h->r.tree_key);
        return S->in_flight.empty() ||
               S->used + admission_bytes(h->r, !resident) <= S->o.hbm_budget;
      });
      if (S->stop) break;
      // the head request, then (if it is small) the small requests behind it
      // that the budget admits, up to batch_max
      while (!S->queue.empty()) {
        ddm_server_req* h = S->queue.front();
        const bool resident = h->r.tree_key && S->trees.count(h->r.tree_key);
        const uint64_t b = admission_bytes(h->r, !resident);
        if (!G.empty() && (G.size() >= S->o.batch_max || !batchable(S, h->r) ||
                           S->used + b > S->o.hbm_budget))
          break;
        S->queue.pop_front();
        S->used += b;
        h->charged = b;
        if (S->used > S->peak) S->peak = S->used;
        S->in_flight[h->ticket] = 1;
        h->t_start = now_ns();
        G.push_back(h);
        if (!batchable(S, h->r)) break;
      }
      if (!S->queue.empty()) S->cv_work.notify_one();
    }
    if (!s) {
      sts.assign(G.size(), DDM_E_DEVICE);
      whys.assign(G.size(), "worker stream creation failed");
    } else if (G.size() == 1) {
      sts.assign(1, DDM_OK);
      whys.assign(1, std::string());
      bool yielded = false;
      sts[0] = process(S, G[0], s, &whys[0], &yielded);
      if (sts[0] != DDM_OK || yielded) (void)hipStreamSynchronize(s);
      if (yielded) {
        // back to the head of the queue, holding nothing; it is admitted
        // again when memory frees up
        ddm_server_req* q = G[0];
        std::lock_guard<std::mutex> lk(S->mu);
        uncharge(S, q, q->charged);
        S->in_flight.erase(q->ticket);
        q->t_start = 0;
        q->K = q->slots = 0;
        q->overflowed = 0;
        q->tree_cached = false;
        ++S->yields;
        S->queue.push_front(q);
        S->cv_mem.notify_all();
        S->cv_work.notify_all();
        continue;
      }
    } else {
      process_batch(S, G, s, &sts, &whys);
    }
    for (size_t i = 0; i < G.size(); ++i) {
      ddm_server_req* q = G[i];
      {
        // inputs, tree (unless cached) and scratch are no longer held; a
        // device-side result stays charged until it is released
        std::lock_guard<std::mutex> lk(S->mu);
        const uint64_t keep = (q->dev && G.size() == 1) ? 8 * std::max<uint64_t>(q->K, 1) : 0;
        uncharge(S, q, q->charged - std::min(keep, q->charged));
      }
      finish(S, q, sts[i], whys[i]);
    }
  }
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
}

}  // namespace

extern "C" ddm_status ddm_server_create(const ddm_server_opts* opts, ddm_predictor* pred,
                                        ddm_server** out) {
  set_detail("");
  if (!out) return DDM_E_INVALID_ARG;
  *out = nullptr;
  ddm_server_opts o{};
  if (opts) o = *opts;
  for (int i = 0; i < 1; ++i)
    if (o.reserved[i]) {
      set_detail("ddm_server_opts: reserved fields must be zero");
      return DDM_E_INVALID_ARG;
    }
  if (o.hbm_budget == 0) o.hbm_budget = 64ull << 30;
  if (o.host_pool == 0 && !o.deliver_device) o.host_pool = 4ull << 30;
  if (o.workers == 0) o.workers = 8;
  if (o.batch_max == 0) o.batch_max = 1;
  if (o.batch_small == 0) o.batch_small = 1u << 18;
  if (o.batch_max > DDM_BATCH_MAX_INSTANCES) {
    set_detail("ddm_server_opts: batch_max above DDM_BATCH_MAX_INSTANCES");
    return DDM_E_INVALID_ARG;
  }
  if (o.workers > 64) {
    set_detail("ddm_server_opts: at most 64 workers");
    return DDM_E_INVALID_ARG;
  }
  ddm_server* S = new (std::nothrow) ddm_server();
  if (!S) return DDM_E_NOMEM;
  S->o = o;
  S->pred = pred;
  hipError_t e = hipGetDevice(&S->device);
  if (e != hipSuccess) {
    delete S;
    return hip_fail(e, "hipGetDevice", __FILE__, __LINE__);
  }
  if (!o.deliver_device && !S->pool.init(o.host_pool)) {
    delete S;
    set_detail("pinned host pool allocation failed");
    return DDM_E_NOMEM;
  }
  for (uint32_t i = 0; i < o.workers; ++i) S->workers.emplace_back(worker_main, S);
  *out = S;
  return DDM_OK;
}

extern "C" ddm_status ddm_server_submit(ddm_server* S, const ddm_request* r, int64_t arrival_ns,
                                        void* stream, uint64_t* ticket) {
  set_detail("");
  if (!S || !r || !ticket) return DDM_E_INVALID_ARG;
  if (r->d < 1 || r->d > DDM_MAX_D || (r->m && (!r->upd_lo || !r->upd_hi)) ||
      (!r->tree_key && r->n && (!r->sub_lo || !r->sub_hi)) || r->reserved) {
    set_detail("ddm_server_submit: bad request (d, pointers or reserved field)");
    return DDM_E_INVALID_ARG;
  }
  ddm_server_req* q = new (std::nothrow) ddm_server_req();
  if (!q) return DDM_E_NOMEM;
  q->r = *r;
  q->t_arrival = arrival_ns ? arrival_ns : now_ns();
  q->ready = pooled_event();
  if (!q->ready) {
    delete q;
    set_detail("event creation failed");
    return DDM_E_DEVICE;
  }
  hipError_t e = hipEventRecord(q->ready, (hipStream_t)stream);
  if (e != hipSuccess) {
    release_event(q->ready);
    delete q;
    return hip_fail(e, "hipEventRecord", __FILE__, __LINE__);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  q->ticket = S->next_ticket++;
  S->reqs[q->ticket] = q;
  S->queue.push_back(q);
  ++S->submitted;
  *ticket = q->ticket;
  S->cv_work.notify_one();
  return DDM_OK;
}

extern "C" uint32_t ddm_server_wait_any(ddm_server* S, uint32_t timeout_ms, uint64_t* tickets,
                                        uint32_t max_tickets) {
  if (!S || !tickets || max_tickets == 0) return 0;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                      [&] { return !S->done.empty() || S->stop; });
  const uint32_t n = (uint32_t)std::min<size_t>(max_tickets, S->done.size());
  for (uint32_t i = 0; i < n; ++i) tickets[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + n);
  return n;
}

extern "C" ddm_status ddm_server_result(ddm_server* S, uint64_t ticket, ddm_result* res) {
  set_detail("");
  if (!S || !res) return DDM_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_detail("unknown or released ticket");
    return DDM_E_INVALID_ARG;
  }
  ddm_server_req* q = it->second;
  *res = ddm_result{};
  res->status = q->status;
  if (q->status == 1) return DDM_OK;
  res->count = q->K;
  res->m = q->r.m;
  if (q->compact) {
    res->sub_ids = (const uint32_t*)q->host;
    res->upd_offsets = (const uint64_t*)(q->host + ((4 * q->K + 7) & ~uint64_t(7)));
  } else {
    res->pairs = q->host ? (const uint64_t*)q->host : q->dev;
  }
  res->on_device = q->dev ? 1u : 0u;
  res->t_arrival_ns = q->t_arrival;
  res->t_start_ns = q->t_start;
  res->t_done_ns = q->t_done;
  res->slots = q->slots;
  res->overflowed = q->overflowed;
  if (q->status != DDM_OK) set_detail(q->detail);
  return DDM_OK;
}

extern "C" ddm_status ddm_server_release(ddm_server* S, uint64_t ticket) {
  set_detail("");
  if (!S) return DDM_E_INVALID_ARG;
  ddm_server_req* q = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->status == 1) {
      set_detail("unknown, released or unfinished ticket");
      return DDM_E_INVALID_ARG;
    }
    q = it->second;
    S->reqs.erase(it);
    if (q->host) S->pool.release(q->host, q->host_bytes);
    if (q->dev) {
      S->used -= std::min(S->used, 8 * std::max<uint64_t>(q->K, 1));
      dev_free((char*)q->dev, nullptr);
    }
    S->cv_mem.notify_all();
    S->cv_work.notify_all();
  }
  release_event(q->ready);
  delete q;
  return DDM_OK;
}

extern "C" ddm_status ddm_server_stats(ddm_server* S, ddm_server_counters* st) {
  if (!S || !st) return DDM_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->queued = S->queue.size();
  st->in_flight = S->in_flight.size();
  st->hbm_used = S->used;
  st->hbm_peak = S->peak;
  st->host_pool_used = S->pool.used;
  st->trees_resident = S->trees.size();
  st->requeued = S->yields;
  return DDM_OK;
}

extern "C" void ddm_server_destroy(ddm_server* S) {
  if (!S) return;
  {
    // let queued and running requests finish first
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->queue.empty() && S->in_flight.empty(); });
    // resident trees are freed on the streams they were built on, which
    // live as long as the workers
    for (auto& kv : S->trees) ddm_tree_free(kv.second.t);
    S->trees.clear();
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_mem.notify_all();
  S->cv_done.notify_all();
  for (auto& w : S->workers) w.join();
  (void)hipSetDevice(S->device);
  for (auto& kv : S->reqs) {
    ddm_server_req* q = kv.second;
    if (q->dev) dev_free((char*)q->dev, nullptr);
    release_event(q->ready);
    delete q;
  }
  if (S->pool.base) (void)hipHostFree(S->pool.base);
  delete S;
}
