// Request loop over the batched GEMM (continuous batching of per-client
// product chains).  Host code: the scheduler, the tick loop and the C ABI of
// include/bgserve.h; the generator and identity kernels live in
// serve_kernels.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <limits>
#include <map>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bgserve.h"
#include "bgemm_internal.h"

namespace bs {

// Factor memory of one device region [0, bytes): host bookkeeping of offsets
// only (the region itself is allocated once, at bs_create).  A client has at
// most one active request, so when the region holds every client's factor at
// once each client gets a fixed slot; otherwise requests take first-fit
// ranges, adjacent free ranges merged on release.
struct Pool {
  static constexpr size_t kAlign = 256;
  static constexpr size_t npos = (size_t)-1;
  std::map<size_t, size_t> free_;   // offset -> length (first-fit mode)
  std::vector<size_t> fixed;        // per-client slot (fixed mode), else empty
  size_t bytes = 0, used = 0, peak = 0;
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  void init(size_t b, const size_t* need, int nc) {
    free_.clear();
    fixed.clear();
    bytes = b;
    used = peak = 0;
    size_t all = 0;
    for (int c = 0; c < nc; ++c) all += round(need[c]);
    if (all <= b) {
      fixed.resize(nc);
      size_t off = 0;
      for (int c = 0; c < nc; ++c) {
        fixed[c] = off;
        off += round(need[c]);
      }
    } else if (b) {
      free_[0] = b;
    }
  }
  size_t alloc(int c, size_t b) {
    b = round(b);
    if (!fixed.empty()) {
      used += b;
      peak = std::max(peak, used);
      return fixed[c];
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < b) continue;
      const size_t off = it->first, rest = it->second - b;
      free_.erase(it);
      if (rest) free_[off + b] = rest;
      used += b;
      peak = std::max(peak, used);
      return off;
    }
    return npos;
  }
  void release(size_t off, size_t b) {
    b = round(b);
    used -= b;
    if (!fixed.empty()) return;
    auto it = free_.emplace(off, b).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Per-client FIFO queues and the one active request of each client.  Pure
// host logic, shared by the device loop and the virtual-clock replay.
struct Scheduler {
  struct Done {
    int r, c;
    size_t off;
  };
  int nc = 0, nreq = 0;
  const double* arrival = nullptr;
  const int* client = nullptr;
  const int* length = nullptr;
  double* start = nullptr;
  double* finish = nullptr;
  std::vector<std::deque<int>> queue;
  std::vector<int> active, remaining;
  std::vector<size_t> slot;  // offset of each active request's factor in the pool
  std::vector<int> batch;    // clients served by the current tick, ascending
  std::vector<int> cand;
  int next = 0, finished = 0;
  // policy 0 (continuous batching): requests start whenever their client is
  // idle; policy 1 (lock step): requests start only when no request is
  // active, so each round of requests runs to its longest chain before the
  // next round forms -- the lock-step batch of the paper's batched approach.
  int policy = 0;
  int max_active = 0;
  int n_active = 0;
  // Factor memory: with a pool, a request holds need[c] bytes of it from its
  // start until its last product has completed; a request that does not fit
  // waits (requests start oldest first, so none overtakes it).
  Pool* pool = nullptr;
  const size_t* need = nullptr;
  long long mem_waits = 0;   // ticks at which the oldest startable request waited for memory

  void init(int num_clients, int n, const double* arr, const int* cl, const int* len, double* st,
            double* fin) {
    nc = num_clients; nreq = n; arrival = arr; client = cl; length = len; start = st; finish = fin;
    queue.assign(nc, {});
    active.assign(nc, -1);
    remaining.assign(nc, 0);
    slot.assign(nc, 0);
    batch.clear();
    next = finished = 0;
    n_active = 0;
    mem_waits = 0;
  }
  void admit(double now) {
    while (next < nreq && arrival[next] <= now) queue[client[next]].push_back(next++);
  }
  // Starts queued requests of idle clients, oldest first, while the policy,
  // max_active (0: no limit) and the factor memory allow; then the tick
  // serves every client with an active request.  A request whose last
  // product is in this tick is listed in `last` and leaves its client idle
  // for the next tick (whose product on the same state is ordered after this
  // one on the device); it counts as finished, and its memory is released,
  // when the tick completes.
  std::vector<Done> last;
  void start_request(int c, double now) {
    const int r = queue[c].front();
    queue[c].pop_front();
    active[c] = r;
    remaining[c] = length[r];
    start[r] = now;
    ++n_active;
  }
  int begin_tick(double now) {
    batch.clear();
    last.clear();
    if (!(policy == 1 && n_active > 0)) {
      cand.clear();
      for (int c = 0; c < nc; ++c)
        if (active[c] < 0 && !queue[c].empty()) cand.push_back(c);
      std::sort(cand.begin(), cand.end(),
                [&](int a, int b) { return queue[a].front() < queue[b].front(); });
      for (int c : cand) {
        if (max_active > 0 && n_active >= max_active) break;
        size_t off = 0;
        if (pool) {
          off = pool->alloc(c, need[c]);
          if (off == Pool::npos) {
            ++mem_waits;
            break;
          }
        }
        slot[c] = off;
        start_request(c, now);
      }
    }
    for (int c = 0; c < nc; ++c) {
      if (active[c] >= 0) {
        batch.push_back(c);
        if (--remaining[c] == 0) {
          last.push_back(Done{active[c], c, slot[c]});
          active[c] = -1;
          --n_active;
        }
      }
    }
    return (int)batch.size();
  }
  void complete(const std::vector<Done>& fin, double now) {
    for (const Done& d : fin) {
      finish[d.r] = now;
      if (pool) pool->release(d.off, need[d.c]);
    }
    finished += (int)fin.size();
  }
  bool done() const { return finished == nreq; }
  double next_arrival() const {
    return next < nreq ? arrival[next] : std::numeric_limits<double>::infinity();
  }
};

static bool valid_schedule(int nc, int n, const double* arr, const int* cl, const int* len) {
  if (n < 0 || (n > 0 && (!arr || !cl || !len))) return false;
  for (int r = 0; r < n; ++r) {
    if (!(arr[r] >= 0.0) || (r > 0 && arr[r] < arr[r - 1])) return false;
    if (cl[r] < 0 || cl[r] >= nc || len[r] < 1) return false;
  }
  return true;
}

}  // namespace bs

struct bs_server {
  unsigned magic;
  bg_handle_t h;
  int device;
  int nc;
  unsigned long long seed;
  std::vector<int> sizes;
  std::vector<double> scale;
  std::vector<double*> st[2];
  // factor memory: one device region, handed out per active request
  char* pool_base;
  size_t pool_bytes;
  bs::Pool pool;
  std::vector<size_t> need;       // factor bytes of each client
  std::vector<int> cur;
  std::vector<long long> products;
  // two sets of job / pointer arrays, so one tick can be prepared while the
  // previous one runs
  bg::FillJob* d_jobs[2];
  bg::FillJob* h_jobs[2];         // pinned
  const double** d_ptrs[2];
  const double** h_ptrs[2];       // pinned
  // per-instance sizes and leading dimensions of a tick's variable-size
  // launch: m, n, k, lda, ldb, ldc, each num_clients ints
  int* d_dims[2];
  int* h_dims[2];                  // pinned
  hipEvent_t ev[2];
  hipEvent_t ev0;
  int max_active;
  int policy;
  int tick_launch;                // BS_TICK_PER_SIZE or BS_TICK_VBATCHED
  long long mem_waits;            // of the last bs_run_schedule
};

static const unsigned kServerMagic = 0x5E7BE5E7u;
static bool valid(bs_server_t s) { return s && s->magic == kServerMagic; }

static size_t state_bytes(int n) { return 2 * (size_t)n * (size_t)n * sizeof(double); }
static size_t factor_bytes(int n) { return bs::Pool::round((size_t)n * (size_t)n * sizeof(double)); }
static size_t array_bytes(int nc) {
  return 2ull * nc * (sizeof(bg::FillJob) + 3 * sizeof(double*) + 6 * sizeof(int));
}

static void free_all(bs_server* s) {
  for (int b = 0; b < 2; ++b)
    for (double* p : s->st[b]) if (p) (void)hipFree(p);
  if (s->pool_base) (void)hipFree(s->pool_base);
  for (int b = 0; b < 2; ++b) {
    if (s->d_jobs[b]) (void)hipFree(s->d_jobs[b]);
    if (s->d_ptrs[b]) (void)hipFree((void*)s->d_ptrs[b]);
    if (s->h_jobs[b]) (void)hipHostFree(s->h_jobs[b]);
    if (s->h_ptrs[b]) (void)hipHostFree((void*)s->h_ptrs[b]);
    if (s->d_dims[b]) (void)hipFree(s->d_dims[b]);
    if (s->h_dims[b]) (void)hipHostFree(s->h_dims[b]);
    if (s->ev[b]) (void)hipEventDestroy(s->ev[b]);
  }
  if (s->ev0) (void)hipEventDestroy(s->ev0);
}

static hipError_t set_identity(bs_server* s, hipStream_t stream) {
  for (int c = 0; c < s->nc; ++c) {
    const hipError_t e = bg::launch_identity(s->st[s->cur[c]][c], s->sizes[c], stream);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(stream);
}

extern "C" {

unsigned long long bs_bytes_needed(int num_clients, const int* sizes) {
  if (num_clients <= 0 || !sizes) return 0;
  unsigned long long t = 0;
  for (int c = 0; c < num_clients; ++c)
    if (sizes[c] > 0) t += state_bytes(sizes[c]) + factor_bytes(sizes[c]);
  return t + array_bytes(num_clients);
}

bg_status_t bs_create(bg_handle_t h, int num_clients, const int* sizes, unsigned long long seed,
                      unsigned long long budget, bs_server_t* out) {
  if (!out || !h || num_clients <= 0 || num_clients > 65535 || !sizes) return BG_STATUS_INVALID_VALUE;
  for (int c = 0; c < num_clients; ++c)
    if (sizes[c] < 1 || sizes[c] > 4096) return BG_STATUS_INVALID_VALUE;
  // States and arrays stay resident; the rest of the budget is the factor
  // pool, which must hold at least the largest client's factor and need not
  // hold more than every client's at once.
  size_t fixed = array_bytes(num_clients), all_factors = 0, largest = 0;
  for (int c = 0; c < num_clients; ++c) {
    fixed += state_bytes(sizes[c]);
    all_factors += factor_bytes(sizes[c]);
    largest = std::max(largest, factor_bytes(sizes[c]));
  }
  size_t pool_bytes = all_factors;
  if (budget) {
    if (fixed + largest > budget) return BG_STATUS_ALLOC_FAILED;
    pool_bytes = std::min(all_factors, (size_t)budget - fixed);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BG_STATUS_DEVICE_ERROR;
  bs_server* s = new bs_server();
  s->magic = kServerMagic;
  s->h = h;
  s->device = dev;
  s->nc = num_clients;
  s->seed = seed;
  s->sizes.assign(sizes, sizes + num_clients);
  s->scale.resize(num_clients);
  s->st[0].assign(num_clients, nullptr);
  s->st[1].assign(num_clients, nullptr);
  s->pool_base = nullptr;
  s->pool_bytes = pool_bytes;
  s->need.resize(num_clients);
  s->policy = 0;
  s->tick_launch = BS_TICK_PER_SIZE;
  s->mem_waits = 0;
  s->cur.assign(num_clients, 0);
  s->products.assign(num_clients, 0);
  bool ok = true;
  for (int c = 0; c < num_clients && ok; ++c) {
    const size_t b = (size_t)sizes[c] * sizes[c] * sizeof(double);
    s->scale[c] = std::sqrt(3.0 / (double)sizes[c]);
    s->need[c] = factor_bytes(sizes[c]);
    ok = hipMalloc(&s->st[0][c], b) == hipSuccess && hipMalloc(&s->st[1][c], b) == hipSuccess;
  }
  ok = ok && hipMalloc((void**)&s->pool_base, pool_bytes) == hipSuccess;
  for (int b = 0; b < 2 && ok; ++b)
    ok = hipMalloc(&s->d_jobs[b], num_clients * sizeof(bg::FillJob)) == hipSuccess &&
         hipMalloc((void**)&s->d_ptrs[b], 3 * num_clients * sizeof(double*)) == hipSuccess &&
         hipHostMalloc((void**)&s->h_jobs[b], num_clients * sizeof(bg::FillJob)) == hipSuccess &&
         hipHostMalloc((void**)&s->h_ptrs[b], 3 * num_clients * sizeof(double*)) == hipSuccess &&
         hipMalloc((void**)&s->d_dims[b], 6 * num_clients * sizeof(int)) == hipSuccess &&
         hipHostMalloc((void**)&s->h_dims[b], 6 * num_clients * sizeof(int)) == hipSuccess &&
         hipEventCreate(&s->ev[b]) == hipSuccess;
  ok = ok && hipEventCreate(&s->ev0) == hipSuccess;
  if (!ok) {
    free_all(s);
    s->magic = 0;
    delete s;
    return BG_STATUS_ALLOC_FAILED;
  }
  void* stream = nullptr;
  bg_get_stream(h, &stream);
  if (set_identity(s, (hipStream_t)stream) != hipSuccess) {
    free_all(s);
    s->magic = 0;
    delete s;
    return BG_STATUS_DEVICE_ERROR;
  }
  *out = s;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_destroy(bs_server_t s) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  (void)hipDeviceSynchronize();
  free_all(s);
  s->magic = 0;
  delete s;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_reset(bs_server_t s) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  void* stream = nullptr;
  bg_get_stream(s->h, &stream);
  for (int c = 0; c < s->nc; ++c) {
    s->cur[c] = 0;
    s->products[c] = 0;
  }
  return set_identity(s, (hipStream_t)stream) == hipSuccess ? BG_STATUS_SUCCESS
                                                             : BG_STATUS_DEVICE_ERROR;
}

bg_status_t bs_state(bs_server_t s, int c, double* host_out, long long* products) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (c < 0 || c >= s->nc || !host_out) return BG_STATUS_INVALID_VALUE;
  const size_t b = (size_t)s->sizes[c] * s->sizes[c] * sizeof(double);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(host_out, s->st[s->cur[c]][c], b, hipMemcpyDeviceToHost) != hipSuccess)
    return BG_STATUS_DEVICE_ERROR;
  if (products) *products = s->products[c];
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_fill_factor(unsigned long long seed, int c, long long j, int n, double* out,
                           void* stream) {
  if (n < 1 || n > 4096 || c < 0 || j < 0 || !out) return BG_STATUS_INVALID_VALUE;
  return bg::launch_fill_one(out, n, c, j, std::sqrt(3.0 / (double)n), seed, (hipStream_t)stream) ==
                 hipSuccess
             ? BG_STATUS_SUCCESS
             : BG_STATUS_DEVICE_ERROR;
}

bg_status_t bs_set_tick_launch(bs_server_t s, int mode) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (mode != BS_TICK_PER_SIZE && mode != BS_TICK_VBATCHED) return BG_STATUS_INVALID_VALUE;
  s->tick_launch = mode;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_set_max_active(bs_server_t s, int max_active) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (max_active < 0) return BG_STATUS_INVALID_VALUE;
  s->max_active = max_active;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_set_policy(bs_server_t s, int policy) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (policy != BS_POLICY_CONTINUOUS && policy != BS_POLICY_LOCKSTEP) return BG_STATUS_INVALID_VALUE;
  s->policy = policy;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_memory_stats(bs_server_t s, unsigned long long* pool_bytes,
                            unsigned long long* peak_bytes, long long* waits) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (pool_bytes) *pool_bytes = s->pool_bytes;
  if (peak_bytes) *peak_bytes = s->pool.peak;
  if (waits) *waits = s->mem_waits;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_simulate(int num_clients, const int* sizes, unsigned long long pool_bytes,
                        int policy, int n_requests, const double* arrival_s, const int* client,
                        const int* length, double tick_s, int max_active, double* out_start,
                        double* out_finish, long long* out_ticks, long long* out_mem_waits) {
  if (num_clients <= 0 || !(tick_s > 0.0) || max_active < 0 ||
      (policy != BS_POLICY_CONTINUOUS && policy != BS_POLICY_LOCKSTEP) ||
      (pool_bytes && !sizes) ||
      !bs::valid_schedule(num_clients, n_requests, arrival_s, client, length) ||
      (n_requests > 0 && (!out_start || !out_finish)))
    return BG_STATUS_INVALID_VALUE;
  std::vector<size_t> need;
  bs::Pool pool;
  if (pool_bytes) {
    need.resize(num_clients);
    for (int c = 0; c < num_clients; ++c) {
      if (sizes[c] < 1 || sizes[c] > 4096) return BG_STATUS_INVALID_VALUE;
      need[c] = factor_bytes(sizes[c]);
      if (need[c] > pool_bytes) return BG_STATUS_ALLOC_FAILED;
    }
    pool.init((size_t)pool_bytes, need.data(), num_clients);
  }
  bs::Scheduler sc;
  sc.init(num_clients, n_requests, arrival_s, client, length, out_start, out_finish);
  sc.max_active = max_active;
  sc.policy = policy;
  if (pool_bytes) {
    sc.pool = &pool;
    sc.need = need.data();
  }
  double now = 0.0;
  long long ticks = 0;
  while (!sc.done()) {
    sc.admit(now);
    if (sc.begin_tick(now) == 0) {
      now = sc.next_arrival();
      continue;
    }
    now += tick_s;
    sc.complete(sc.last, now);
    ++ticks;
  }
  if (out_ticks) *out_ticks = ticks;
  if (out_mem_waits) *out_mem_waits = sc.mem_waits;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_run_schedule(bs_server_t s, int n_requests, const double* arrival_s,
                            const int* client, const int* length, double* out_start,
                            double* out_finish, long long* out_ticks) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (!bs::valid_schedule(s->nc, n_requests, arrival_s, client, length) ||
      (n_requests > 0 && (!out_start || !out_finish)))
    return BG_STATUS_INVALID_VALUE;
  void* sv = nullptr;
  bg_get_stream(s->h, &sv);
  const hipStream_t stream = (hipStream_t)sv;
  bs::Scheduler sc;
  sc.init(s->nc, n_requests, arrival_s, client, length, out_start, out_finish);
  sc.max_active = s->max_active;
  sc.policy = s->policy;
  s->pool.init(s->pool_bytes, s->need.data(), s->nc);
  sc.pool = &s->pool;
  sc.need = s->need.data();
  using clk = std::chrono::steady_clock;
  // Up to two ticks in flight: the host prepares and launches tick t + 1
  // while tick t runs.  A tick's completion time is read from its event
  // relative to an event recorded when the call starts.
  struct InFlight {
    int set;
    std::vector<bs::Scheduler::Done> fin;
  };
  std::deque<InFlight> flight;
  if (hipStreamSynchronize(stream) != hipSuccess || hipEventRecord(s->ev0, stream) != hipSuccess)
    return BG_STATUS_DEVICE_ERROR;
  const auto t0 = clk::now();
  auto now = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
  auto retire = [&](bool wait) -> bool {
    InFlight& f = flight.front();
    const hipError_t q = wait ? hipEventSynchronize(s->ev[f.set]) : hipEventQuery(s->ev[f.set]);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) return false;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev0, s->ev[f.set]) != hipSuccess) ms = (float)(now() * 1e3);
    sc.complete(f.fin, (double)ms * 1e-3);
    flight.pop_front();
    return true;
  };
  std::vector<int> order;
  long long ticks = 0;
  int set = 0;
  while (!sc.done()) {
    while (!flight.empty() && retire(false)) {}
    if (sc.done()) break;
    if (flight.size() == 2) {
      if (!retire(true)) return BG_STATUS_DEVICE_ERROR;
      continue;
    }
    sc.admit(now());
    const int nb = sc.begin_tick(now());
    if (nb == 0) {
      if (!flight.empty()) {
        if (!retire(true)) return BG_STATUS_DEVICE_ERROR;
        continue;
      }
      const double t_next = sc.next_arrival();
      while (now() < t_next) std::this_thread::yield();
      continue;
    }
    // factor jobs, and the clients grouped by size
    order = sc.batch;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return s->sizes[a] < s->sizes[b]; });
    bg::FillJob* hj = s->h_jobs[set];
    const double** hp = s->h_ptrs[set];
    const double** dp = s->d_ptrs[set];
    for (int i = 0; i < nb; ++i) {
      const int c = order[i];
      double* f = (double*)(s->pool_base + sc.slot[c]);
      hj[i] = bg::FillJob{f, s->products[c], s->sizes[c], c, s->scale[c]};
      hp[i] = f;
      hp[nb + i] = s->st[s->cur[c]][c];
      hp[2 * nb + i] = s->st[s->cur[c] ^ 1][c];
    }
    // the tick's arrays go up, all factors are generated in one launch, then
    // one batched launch per distinct size, all on the handle's stream
    int max_n = 0;
    for (int i = 0; i < nb; ++i) max_n = std::max(max_n, s->sizes[order[i]]);
    if (hipMemcpyAsync(s->d_jobs[set], hj, nb * sizeof(bg::FillJob), hipMemcpyHostToDevice,
                       stream) != hipSuccess ||
        hipMemcpyAsync((void*)dp, (const void*)hp, 3 * nb * sizeof(double*),
                       hipMemcpyHostToDevice, stream) != hipSuccess ||
        bg::launch_fill_factors(s->d_jobs[set], nb, max_n, s->seed, stream) != hipSuccess)
      return BG_STATUS_DEVICE_ERROR;
    if (s->tick_launch == BS_TICK_VBATCHED) {
      // one variable-size launch for the whole tick, planned on the device
      int* hd = s->h_dims[set];
      int* dd = s->d_dims[set];
      for (int f = 0; f < 6; ++f)
        for (int i = 0; i < nb; ++i) hd[f * nb + i] = s->sizes[order[i]];
      if (hipMemcpyAsync(dd, hd, 6 * nb * sizeof(int), hipMemcpyHostToDevice, stream) !=
          hipSuccess)
        return BG_STATUS_DEVICE_ERROR;
      const bg_status_t st =
          bg_dgemm_vbatched(s->h, 'N', 'N', dd, dd + nb, dd + 2 * nb, 1.0, dp, dd + 3 * nb,
                            dp + nb, dd + 4 * nb, 0.0, (double* const*)(dp + 2 * nb),
                            dd + 5 * nb, nb, nullptr);
      if (st != BG_STATUS_SUCCESS) return st;
    } else {
      for (int g0 = 0; g0 < nb;) {
        int g1 = g0;
        const int n = s->sizes[order[g0]];
        while (g1 < nb && s->sizes[order[g1]] == n) ++g1;
        const bg_status_t st = bg_dgemm_batched(s->h, 'N', 'N', n, n, n, 1.0, dp + g0, n,
                                                dp + nb + g0, n, 0.0,
                                                (double* const*)(dp + 2 * nb + g0), n, g1 - g0);
        if (st != BG_STATUS_SUCCESS) return st;
        g0 = g1;
      }
    }
    if (hipEventRecord(s->ev[set], stream) != hipSuccess) return BG_STATUS_DEVICE_ERROR;
    for (int c : sc.batch) {
      s->cur[c] ^= 1;
      ++s->products[c];
    }
    flight.push_back(InFlight{set, sc.last});
    set ^= 1;
    ++ticks;
  }
  if (out_ticks) *out_ticks = ticks;
  s->mem_waits = sc.mem_waits;
  return BG_STATUS_SUCCESS;
}

bg_status_t bs_run_sweeps(bs_server_t s, int sweeps, int chain, int use_graph,
                          double* out_seconds) {
  if (!valid(s)) return BG_STATUS_INVALID_HANDLE;
  if (sweeps < 0 || chain < 1) return BG_STATUS_INVALID_VALUE;
  void* sv = nullptr;
  bg_get_stream(s->h, &sv);
  const hipStream_t stream = (hipStream_t)sv;
  const int nc = s->nc;
  // clients grouped by size; per tick t and starting parity p the pointer
  // triples (factor, state in, state out)
  std::vector<int> order(nc);
  for (int c = 0; c < nc; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return s->sizes[a] < s->sizes[b]; });
  // every client takes part in every sweep: each holds a factor of the pool
  s->pool.init(s->pool_bytes, s->need.data(), nc);
  std::vector<double*> fac(nc);
  for (int c = 0; c < nc; ++c) {
    const size_t off = s->pool.alloc(c, s->need[c]);
    if (off == bs::Pool::npos) return BG_STATUS_ALLOC_FAILED;
    fac[c] = (double*)(s->pool_base + off);
  }
  int max_n = 0;
  std::vector<bg::SweepJob> jobs(nc);
  std::vector<long long> j0(nc);
  for (int i = 0; i < nc; ++i) {
    const int c = order[i];
    jobs[i] = bg::SweepJob{fac[c], s->sizes[c], c, s->scale[c]};
    max_n = std::max(max_n, s->sizes[c]);
  }
  for (int c = 0; c < nc; ++c) j0[c] = s->products[c];
  std::vector<const double*> ptrs((size_t)2 * chain * 3 * nc);
  for (int p = 0; p < 2; ++p)
    for (int t = 0; t < chain; ++t) {
      const double** row = ptrs.data() + ((size_t)p * chain + t) * 3 * nc;
      for (int i = 0; i < nc; ++i) {
        const int c = order[i];
        const int cur = s->cur[c] ^ p ^ (t & 1);
        row[i] = fac[c];
        row[nc + i] = s->st[cur][c];
        row[2 * nc + i] = s->st[cur ^ 1][c];
      }
    }
  bg::SweepJob* d_jobs = nullptr;
  long long* d_j0 = nullptr;
  const double** d_ptrs = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bg_status_t st = BG_STATUS_SUCCESS;
  auto fail = [&](bg_status_t x) { if (st == BG_STATUS_SUCCESS) st = x; };
  if (hipMalloc(&d_jobs, nc * sizeof(bg::SweepJob)) != hipSuccess ||
      hipMalloc(&d_j0, nc * sizeof(long long)) != hipSuccess ||
      hipMalloc((void**)&d_ptrs, ptrs.size() * sizeof(double*)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    fail(BG_STATUS_ALLOC_FAILED);
  if (st == BG_STATUS_SUCCESS &&
      (hipMemcpy(d_jobs, jobs.data(), nc * sizeof(bg::SweepJob), hipMemcpyHostToDevice) !=
           hipSuccess ||
       hipMemcpy(d_j0, j0.data(), nc * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy((void*)d_ptrs, ptrs.data(), ptrs.size() * sizeof(double*),
                 hipMemcpyHostToDevice) != hipSuccess))
    fail(BG_STATUS_DEVICE_ERROR);
  // one sweep starting at parity p: per tick the factors, then one batched
  // launch per size; finally the product counters advance
  auto enqueue_sweep = [&](int p, hipStream_t q) -> bg_status_t {
    for (int t = 0; t < chain; ++t) {
      const double** row = d_ptrs + ((size_t)p * chain + t) * 3 * nc;
      if (bg::launch_fill_sweep(d_jobs, nc, max_n, d_j0, t, s->seed, q) != hipSuccess)
        return BG_STATUS_DEVICE_ERROR;
      for (int g0 = 0; g0 < nc;) {
        int g1 = g0;
        const int n = s->sizes[order[g0]];
        while (g1 < nc && s->sizes[order[g1]] == n) ++g1;
        const bg_status_t r = bg_dgemm_batched(s->h, 'N', 'N', n, n, n, 1.0, row + g0, n,
                                               row + nc + g0, n, 0.0,
                                               (double* const*)(row + 2 * nc + g0), n, g1 - g0);
        if (r != BG_STATUS_SUCCESS) return r;
        g0 = g1;
      }
    }
    return bg::launch_advance(d_j0, nc, chain, q) == hipSuccess ? BG_STATUS_SUCCESS
                                                                 : BG_STATUS_DEVICE_ERROR;
  };
  const int nparity = (chain & 1) ? 2 : 1;
  if (st == BG_STATUS_SUCCESS && use_graph) {
    // The handle's stream may be the null stream, which cannot be captured:
    // capture on a private stream (default priority) with the handle
    // pointed at it, then replay on the handle's stream.
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
      fail(BG_STATUS_DEVICE_ERROR);
    } else {
      bg_set_stream(s->h, (void*)cap);
      for (int p = 0; p < nparity && st == BG_STATUS_SUCCESS; ++p) {
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          fail(BG_STATUS_DEVICE_ERROR);
          break;
        }
        const bg_status_t r = enqueue_sweep(p, cap);
        const hipError_t ec = hipStreamEndCapture(cap, &graph[p]);
        if (r != BG_STATUS_SUCCESS) fail(r);
        else if (ec != hipSuccess ||
                 hipGraphInstantiate(&exec[p], graph[p], nullptr, nullptr, 0) != hipSuccess)
          fail(BG_STATUS_DEVICE_ERROR);
      }
      bg_set_stream(s->h, sv);
      (void)hipStreamDestroy(cap);
    }
  }
  if (st == BG_STATUS_SUCCESS) {
    if (hipStreamSynchronize(stream) != hipSuccess || hipEventRecord(e0, stream) != hipSuccess)
      fail(BG_STATUS_DEVICE_ERROR);
    for (int w = 0; w < sweeps && st == BG_STATUS_SUCCESS; ++w) {
      const int p = (chain & 1) ? (w & 1) : 0;
      if (use_graph) {
        if (hipGraphLaunch(exec[p], stream) != hipSuccess) fail(BG_STATUS_DEVICE_ERROR);
      } else {
        const bg_status_t r = enqueue_sweep(p, stream);
        if (r != BG_STATUS_SUCCESS) fail(r);
      }
    }
    if (st == BG_STATUS_SUCCESS &&
        (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      fail(BG_STATUS_DEVICE_ERROR);
    float ms = 0.f;
    if (st == BG_STATUS_SUCCESS && out_seconds && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      *out_seconds = (double)ms * 1e-3;
  }
  if (st == BG_STATUS_SUCCESS) {
    const long long done = (long long)sweeps * chain;
    for (int c = 0; c < nc; ++c) {
      s->products[c] += done;
      s->cur[c] ^= (int)(done & 1);
    }
  }
  (void)hipStreamSynchronize(stream);
  for (int p = 0; p < 2; ++p) {
    if (exec[p]) (void)hipGraphExecDestroy(exec[p]);
    if (graph[p]) (void)hipGraphDestroy(graph[p]);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d_jobs) (void)hipFree(d_jobs);
  if (d_j0) (void)hipFree(d_j0);
  if (d_ptrs) (void)hipFree((void*)d_ptrs);
  return st;
}

}  // extern "C"
