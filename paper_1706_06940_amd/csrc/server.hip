// Serving runtime: resident arrays with their block Sparse Tables, a request
// queue, continuous batching over several streams, and completion tracking.
//
// Requests (array id, q queries in host memory) are queued by rmq_server_submit.
// A dispatcher thread takes whatever is pending whenever a slot -- a stream
// with its own pinned staging buffer (and, in the copying mode, device query
// buffers) -- is free, packs the requests FIFO into it while their queries fit
// the slot's capacity (admission by footprint: the slots' buffers are sized
// from the configured byte budget), and enqueues one query launch over the
// coalesced batch (each request's queries address its own resident table).
// By default that kernel reads the queries from the pinned staging buffer and
// writes the answers there itself; with RMQ_SERVER_COPY_QUERIES they go
// through device buffers with one H2D and one D2H copy.  (The copy engines
// were measured to stall now and then for several ms at moderate load, a
// whole p99 by themselves, while reading in place did not.)  Requests
// arriving meanwhile form the next batch on the next free slot, so batches
// overlap on the device.  A completion thread polls the slots' events, copies
// each request's answers to its output buffer and stamps its completion time.
#include <math.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "index.h"
#include "kernels.h"
#include "rmq.h"

using namespace rmq;

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  static const clk::time_point t0 = clk::now();
  return std::chrono::duration<double>(clk::now() - t0).count();
}

struct Request {
  uint64_t ticket;
  int32_t table;
  int64_t q;
  const int32_t* L;
  const int32_t* R;
  int32_t* out;
  double t_submit = 0, t_launch = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 in flight, 2 done, 3 failed
  int32_t batch_size = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* h = nullptr;  // pinned staging: queries (L then R) | out | seg_prefix | seg_table
  char* d = nullptr;  // device buffers, same layout
  std::vector<Request*> reqs;
  int64_t used = 0;
  bool busy = false;
};

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

}  // namespace

struct rmq_server_s {
  rmq_server_config cfg{};
  int device = 0;
  int64_t cap = 0;       // queries per slot
  int32_t max_reqs = 0;  // requests per batch
  size_t off_out = 0, off_prefix = 0, off_table = 0, slot_bytes = 0;
  // device memory admitted against cfg.hbm_budget_bytes: the table
  // descriptors and device slot buffers (fixed at creation), the resident
  // tables, and tables whose build is under way (reserved, not yet added)
  size_t hbm_fixed = 0, hbm_tables = 0, hbm_reserved = 0;
  int32_t tables_reserved = 0;
  std::vector<rmq_index> tables;
  std::vector<ArrayDesc> h_tables;
  ArrayDesc* d_tables = nullptr;
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv;  // any state change
  std::deque<Request*> pending;
  std::deque<int> inflight;    // slot indices in launch order
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  rmq_server_stats stats{};
  std::thread dispatcher, completer;
  hipError_t error = hipSuccess;
};

namespace {

rmq_status from_hip(hipError_t e) {
  if (e == hipSuccess) return RMQ_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return RMQ_ERR_OUT_OF_MEMORY;
  return RMQ_ERR_DEVICE;
}

// Pack and enqueue the requests already assigned to slot `si`.  The staging
// area holds the batch's L values followed directly by its R values, so one
// copy moves exactly 8 bytes per query.
hipError_t launch_slot(rmq_server_s* S, int si) {
  Slot& sl = S->slots[si];
  int64_t total = 0;
  for (const Request* r : sl.reqs) total += r->q;
  int32_t* hL = reinterpret_cast<int32_t*>(sl.h);
  int32_t* hR = hL + total;
  int64_t* hp = reinterpret_cast<int64_t*>(sl.h + S->off_prefix);
  int32_t* ht = reinterpret_cast<int32_t*>(sl.h + S->off_table);
  int64_t off = 0;
  const int nseg = (int)sl.reqs.size();
  for (int i = 0; i < nseg; ++i) {
    Request* r = sl.reqs[i];
    memcpy(hL + off, r->L, sizeof(int32_t) * (size_t)r->q);
    memcpy(hR + off, r->R, sizeof(int32_t) * (size_t)r->q);
    hp[i] = off;
    ht[i] = r->table;
    off += r->q;
  }
  hp[nseg] = off;
  if (!sl.d) {
    // in place: the kernel reads the queries from the pinned staging buffer
    // and writes the answers there
    const int32_t* hq = reinterpret_cast<const int32_t*>(sl.h);
    RMQ_TRY(launch_query_segments(S->d_tables,
                                  reinterpret_cast<const int64_t*>(sl.h + S->off_prefix),
                                  reinterpret_cast<const int32_t*>(sl.h + S->off_table), nseg, hq,
                                  hq + total, reinterpret_cast<int32_t*>(sl.h + S->off_out), total,
                                  S->cfg.sub_block_size > 0, sl.stream));
    return hipEventRecord(sl.done, sl.stream);
  }
  const size_t seg_bytes = sizeof(int64_t) * (size_t)(nseg + 1);
  RMQ_TRY(hipMemcpyAsync(sl.d, sl.h, 2 * sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice,
                         sl.stream));
  RMQ_TRY(hipMemcpyAsync(sl.d + S->off_prefix, sl.h + S->off_prefix, seg_bytes,
                         hipMemcpyHostToDevice, sl.stream));
  RMQ_TRY(hipMemcpyAsync(sl.d + S->off_table, sl.h + S->off_table,
                         sizeof(int32_t) * (size_t)nseg, hipMemcpyHostToDevice, sl.stream));
  const int32_t* dL = reinterpret_cast<const int32_t*>(sl.d);
  RMQ_TRY(launch_query_segments(S->d_tables, reinterpret_cast<const int64_t*>(sl.d + S->off_prefix),
                                reinterpret_cast<const int32_t*>(sl.d + S->off_table), nseg, dL,
                                dL + total, reinterpret_cast<int32_t*>(sl.d + S->off_out), total,
                                S->cfg.sub_block_size > 0, sl.stream));
  RMQ_TRY(hipMemcpyAsync(sl.h + S->off_out, sl.d + S->off_out, sizeof(int32_t) * (size_t)total,
                         hipMemcpyDeviceToHost, sl.stream));
  return hipEventRecord(sl.done, sl.stream);
}

void dispatcher_loop(rmq_server_s* S) {
  hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    int free_slot = -1;
    S->cv.wait(lk, [&] {
      if (S->stopping && S->pending.empty()) return true;
      if (S->pending.empty()) return false;
      for (size_t i = 0; i < S->slots.size(); ++i)
        if (!S->slots[i].busy) {
          free_slot = (int)i;
          return true;
        }
      return false;
    });
    if (free_slot < 0) break;  // stopping with nothing pending
    Slot& sl = S->slots[free_slot];
    sl.reqs.clear();
    sl.used = 0;
    // admission: FIFO while the slot's device capacity holds the queries
    while (!S->pending.empty() && (int32_t)sl.reqs.size() < S->max_reqs) {
      Request* r = S->pending.front();
      if (sl.used + r->q > S->cap) break;
      S->pending.pop_front();
      sl.reqs.push_back(r);
      sl.used += r->q;
    }
    sl.busy = true;
    const double t = now_s();
    for (Request* r : sl.reqs) {
      r->state = 1;
      r->t_launch = t;
      r->batch_size = (int32_t)sl.reqs.size();
    }
    S->stats.batches += 1;
    S->stats.queries += sl.used;
    int inflight_now = 1;
    for (const Slot& o : S->slots) inflight_now += (&o != &sl && o.busy) ? 1 : 0;
    if (inflight_now > S->stats.max_inflight) S->stats.max_inflight = inflight_now;
    lk.unlock();
    const hipError_t e = launch_slot(S, free_slot);
    lk.lock();
    if (e != hipSuccess) S->error = e;
    S->inflight.push_back(free_slot);
    S->cv.notify_all();
  }
}

void completer_loop(rmq_server_s* S) {
  hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv.wait(lk, [&] { return !S->inflight.empty() || (S->stopping && S->pending.empty()); });
    if (S->inflight.empty()) {
      // stopping: wait until the dispatcher has queued its last batch
      bool any_busy = false;
      for (const Slot& sl : S->slots) any_busy |= sl.busy;
      if (!any_busy) break;
      S->cv.wait_for(lk, std::chrono::microseconds(100));
      continue;
    }
    // poll the in-flight slots; finish any that is done
    int finished = -1;
    size_t pos = 0;
    for (; pos < S->inflight.size(); ++pos) {
      const hipError_t q = hipEventQuery(S->slots[S->inflight[pos]].done);
      if (q == hipSuccess) {
        finished = S->inflight[pos];
        break;
      }
      if (q != hipErrorNotReady) {
        S->error = q;
        finished = S->inflight[pos];
        break;
      }
    }
    if (finished < 0) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
      continue;
    }
    S->inflight.erase(S->inflight.begin() + (long)pos);
    Slot& sl = S->slots[finished];
    lk.unlock();
    const int32_t* hout = reinterpret_cast<const int32_t*>(sl.h + S->off_out);
    int64_t off = 0;
    for (Request* r : sl.reqs) {
      memcpy(r->out, hout + off, sizeof(int32_t) * (size_t)r->q);
      off += r->q;
    }
    const double t = now_s();
    lk.lock();
    const int st = S->error == hipSuccess ? 2 : 3;
    for (Request* r : sl.reqs) {
      r->t_done = t;
      r->state = st;
    }
    S->stats.completed += (int64_t)sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    S->cv.notify_all();
  }
}

void free_slots(rmq_server_s* S) {
  for (Slot& sl : S->slots) {
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.h) hipHostFree(sl.h);
    if (sl.d) hipFree(sl.d);
  }
}

}  // namespace

extern "C" {

rmq_status rmq_server_create(const rmq_server_config* cfg, rmq_server* out) {
  if (!cfg || !out || cfg->num_streams < 1 || cfg->num_streams > 16 || cfg->max_tables < 1 ||
      cfg->max_requests_per_batch < 1 || cfg->budget_bytes < 4096 ||
      (cfg->flags & ~RMQ_SERVER_COPY_QUERIES) != 0)
    return RMQ_ERR_INVALID_ARG;
  const int32_t k1 = cfg->sub_block_size;
  if (k1 != 0 && (k1 < RMQ_MIN_BLOCK || k1 >= RMQ_MAX_BLOCK || (k1 & (k1 - 1)) != 0))
    return RMQ_ERR_INVALID_ARG;
  rmq_server_s* S = new (std::nothrow) rmq_server_s();
  if (!S) return RMQ_ERR_OUT_OF_MEMORY;
  S->cfg = *cfg;
  hipGetDevice(&S->device);
  S->max_reqs = cfg->max_requests_per_batch;
  // per slot: L, R, out (12 bytes a query) + segment tables, from the budget
  const size_t per_slot = cfg->budget_bytes / (size_t)cfg->num_streams;
  const size_t seg_bytes = align_up(sizeof(int64_t) * (size_t)(S->max_reqs + 1)) +
                           align_up(sizeof(int32_t) * (size_t)S->max_reqs);
  if (per_slot <= seg_bytes + 3 * kAlign) {
    delete S;
    return RMQ_ERR_INVALID_ARG;
  }
  S->cap = (int64_t)((per_slot - seg_bytes - 3 * kAlign) / (3 * sizeof(int32_t)));
  S->off_out = align_up(2 * sizeof(int32_t) * (size_t)S->cap);
  S->off_prefix = S->off_out + align_up(sizeof(int32_t) * (size_t)S->cap);
  S->off_table = S->off_prefix + align_up(sizeof(int64_t) * (size_t)(S->max_reqs + 1));
  S->slot_bytes = S->off_table + align_up(sizeof(int32_t) * (size_t)S->max_reqs);
  S->hbm_fixed = sizeof(ArrayDesc) * (size_t)cfg->max_tables +
                 ((cfg->flags & RMQ_SERVER_COPY_QUERIES) ? (size_t)cfg->num_streams * S->slot_bytes
                                                         : 0);
  if (cfg->hbm_budget_bytes && S->hbm_fixed > cfg->hbm_budget_bytes) {
    delete S;
    return RMQ_ERR_OUT_OF_MEMORY;
  }
  S->slots.resize(cfg->num_streams);
  hipError_t e = hipMalloc(&S->d_tables, sizeof(ArrayDesc) * (size_t)cfg->max_tables);
  for (Slot& sl : S->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.h), S->slot_bytes, 0);
    if (e == hipSuccess && (cfg->flags & RMQ_SERVER_COPY_QUERIES))
      e = hipMalloc(reinterpret_cast<void**>(&sl.d), S->slot_bytes);
  }
  if (e != hipSuccess) {
    free_slots(S);
    if (S->d_tables) hipFree(S->d_tables);
    delete S;
    return from_hip(e);
  }
  S->stats.slot_capacity = S->cap;
  S->stats.hbm_bytes = S->hbm_fixed;
  S->dispatcher = std::thread(dispatcher_loop, S);
  S->completer = std::thread(completer_loop, S);
  *out = S;
  return RMQ_OK;
}

rmq_status rmq_server_add_array(rmq_server S, const int32_t* A, int64_t n, int32_t block_size,
                                int32_t* table_id) {
  if (!S || !table_id) return RMQ_ERR_INVALID_ARG;
  rmq_options o{};
  o.block_size = block_size;
  o.sub_block_size = S->cfg.sub_block_size;  // every table of the server alike
  const size_t need = rmq_build_bytes(n, &o);
  if (need == 0) return RMQ_ERR_INVALID_ARG;
  {
    // admission: a table slot and, under an HBM budget, the table's bytes
    // are reserved before the build, so concurrent adds cannot overrun either
    std::lock_guard<std::mutex> lk(S->mu);
    if ((int32_t)S->tables.size() + S->tables_reserved >= S->cfg.max_tables)
      return RMQ_ERR_INVALID_ARG;
    const size_t held = S->hbm_fixed + S->hbm_tables + S->hbm_reserved;
    if (S->cfg.hbm_budget_bytes && held + need > S->cfg.hbm_budget_bytes)
      return RMQ_ERR_OUT_OF_MEMORY;
    S->tables_reserved += 1;
    S->hbm_reserved += need;
  }
  auto release = [&] {
    S->tables_reserved -= 1;
    S->hbm_reserved -= need;
  };
  rmq_index ix = nullptr;
  rmq_status st = rmq_build(A, n, &o, nullptr, &ix);
  hipError_t e = st == RMQ_OK ? hipDeviceSynchronize() : hipSuccess;
  if (st == RMQ_OK && e != hipSuccess) {
    rmq_index_free(ix);
    st = from_hip(e);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  release();
  if (st != RMQ_OK) return st;
  const ArrayDesc d{ix->A,    ix->n,   ix->kshift, ix->levels, ix->nb, ix->st,
                    nullptr,  nullptr, 0,          nullptr,    ix->lg, ix->rec,
                    ix->levels, ix->sub, ix->nb1,  ix->k1shift};
  const int32_t id = (int32_t)S->tables.size();
  e = hipMemcpy(S->d_tables + id, &d, sizeof(ArrayDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    rmq_index_free(ix);
    return from_hip(e);
  }
  S->tables.push_back(ix);
  S->h_tables.push_back(d);
  S->hbm_tables += ix->bytes;
  S->stats.index_bytes += ix->bytes;
  S->stats.hbm_bytes = S->hbm_fixed + S->hbm_tables;
  *table_id = id;
  return RMQ_OK;
}

rmq_status rmq_server_submit(rmq_server S, int32_t table_id, const int32_t* L, const int32_t* R,
                             int64_t q, int32_t* out, uint64_t* ticket) {
  if (!S || !ticket || q < 1 || !L || !R || !out) return RMQ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (table_id < 0 || table_id >= (int32_t)S->tables.size() || q > S->cap || S->stopping)
    return RMQ_ERR_INVALID_ARG;
  Request* r = new (std::nothrow) Request();
  if (!r) return RMQ_ERR_OUT_OF_MEMORY;
  r->ticket = S->next_ticket++;
  r->table = table_id;
  r->q = q;
  r->L = L;
  r->R = R;
  r->out = out;
  r->t_submit = now_s();
  S->reqs[r->ticket] = r;
  S->pending.push_back(r);
  S->stats.submitted += 1;
  S->cv.notify_all();
  *ticket = r->ticket;
  return RMQ_OK;
}

rmq_status rmq_server_submit_schedule(rmq_server S, int32_t count, const rmq_request_spec* specs,
                                      uint64_t* tickets) {
  if (!S || count < 0 || (count > 0 && (!specs || !tickets))) return RMQ_ERR_INVALID_ARG;
  for (int32_t i = 0; i < count; ++i) {
    const rmq_request_spec& sp = specs[i];
    // wait for the arrival time: sleep while far, spin the last 50 us
    for (;;) {
      const double dt = sp.t_arrival - now_s();
      if (dt <= 0) break;
      if (dt > 100e-6)
        std::this_thread::sleep_for(std::chrono::duration<double>(dt - 50e-6));
    }
    const rmq_status st =
        rmq_server_submit(S, sp.table_id, sp.L, sp.R, sp.q, sp.out, &tickets[i]);
    if (st != RMQ_OK) return st;
  }
  return RMQ_OK;
}

rmq_status rmq_server_wait(rmq_server S, uint64_t ticket, rmq_request_info* info) {
  if (!S) return RMQ_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return RMQ_ERR_INVALID_ARG;
  Request* r = it->second;
  S->cv.wait(lk, [&] { return r->state >= 2; });
  if (info) {
    info->t_submit = r->t_submit;
    info->t_launch = r->t_launch;
    info->t_done = r->t_done;
    info->batch_requests = r->batch_size;
  }
  const rmq_status st = r->state == 2 ? RMQ_OK : from_hip(S->error);
  S->reqs.erase(it);
  delete r;
  return st;
}

rmq_status rmq_server_stats_get(rmq_server S, rmq_server_stats* out) {
  if (!S || !out) return RMQ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  return RMQ_OK;
}

double rmq_server_clock(void) { return now_s(); }

rmq_status rmq_server_destroy(rmq_server S) {
  if (!S) return RMQ_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    S->cv.notify_all();
  }
  S->dispatcher.join();
  S->completer.join();
  hipDeviceSynchronize();
  for (auto& kv : S->reqs) delete kv.second;
  free_slots(S);
  for (rmq_index ix : S->tables) rmq_index_free(ix);
  hipFree(S->d_tables);
  delete S;
  return RMQ_OK;
}

}  // extern "C"
