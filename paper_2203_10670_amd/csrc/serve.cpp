// Serving loop of libfcfs: continuous batching of rescale requests on one GPU.
//
// Threads. Clients call fcfs_submit from any thread (requests go to a FIFO).
// The scheduler thread builds one batch per tick: first the next chunk of
// every admitted request that still has waves to launch, then new requests
// admitted from the head of the FIFO while request slots and the device arena
// allow. A batch is a generator launch for the newly admitted requests whose
// input it must create, the descriptor upload and one batched forward launch,
// on one of two streams in turn. A request larger than the chunk size (in
// waves) runs as chunks over several batches, so requests that arrive behind
// it start in the next tick instead of after all of it. The completion thread
// waits for each batch's event in launch order, timestamps the requests whose
// last chunk it held and frees their arena inputs and slots.
//
// Memory. The arena is one device allocation made at creation; a first-fit
// free list (offsets, 256-byte granules, neighbours merged on free) hands out
// generated inputs and server-owned outputs. A request that cannot fit even
// in an empty arena fails alone with FCFS_E_NOMEM; one that does not fit now
// waits at the head of the FIFO until completions free space.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fcfs_internal.h"

namespace fcfs {
namespace {

constexpr size_t kGranule = 256;
constexpr size_t kMaxPending = 1 << 16;
constexpr int64_t kDefaultChunkWaves = 16384;   // about five times the waves the GPU holds at once

size_t round_up(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }

class Arena {
 public:
  void init(size_t bytes) {
    size_ = bytes;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  // Returns the offset, or SIZE_MAX when no free block is large enough.
  size_t alloc(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used_ += bytes;
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  size_t size_ = 0;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
};

enum TicketState { kPending = 0, kAdmitted = 1, kDone = 2 };

struct Ticket {
  fcfs_request req;
  int state = kPending;
  fcfs_status status = FCFS_OK;
  fcfs_plan_t plan = nullptr;
  FwdGeom geom;                                // launch geometry of the batched kernel
  int variant = 0;
  int64_t waves_launched = 0;                  // waves of the forward in launched batches
  int chunks_inflight = 0;                     // launched batches holding a chunk, not yet complete
  bool failed = false;                         // a batch holding one of its chunks failed
  int gen_stream = -1;                         // stream of the batch that generated the input
  int64_t ho = 0, wo = 0;
  size_t x_bytes = 0, y_bytes = 0;
  size_t x_off = SIZE_MAX, y_off = SIZE_MAX;   // arena offsets when server-owned
  void* x = nullptr;
  void* y = nullptr;
  uint64_t alg_bytes = 0;                      // input rows read + output
  double t_arrive = 0, t_start = 0, t_done = 0;
};

// A chunk of a request in the batch being built: forward instance, ticket,
// first wave and number of waves.
struct Chunk {
  int variant;
  uint64_t id;
  int64_t begin, n;
};

struct Batch {
  std::vector<uint64_t> tickets;
  hipEvent_t done = nullptr;
  int stream = 0;
  bool failed = false;
};

// Host staging and device copy of one stream's batch descriptors.
struct StreamBufs {
  hipStream_t stream = nullptr;
  hipEvent_t last = nullptr;       // event of the last batch launched on this stream
  bool busy = false;
  BatchDesc* h_desc = nullptr;     // pinned
  int64_t* h_wave = nullptr;
  GenDesc* h_gen = nullptr;
  int64_t* h_gblk = nullptr;
  BatchDesc* d_desc = nullptr;
  int64_t* d_wave = nullptr;
  GenDesc* d_gen = nullptr;
  int64_t* d_gblk = nullptr;
};

}  // namespace
}  // namespace fcfs

struct fcfs_server_ {
  int device = 0;
  int max_slots = 0;
  char* arena_base = nullptr;
  fcfs::Arena arena;
  fcfs::StreamBufs sb[2];
  int next_stream = 0;

  std::mutex mu;
  std::condition_variable cv_sched;    // scheduler: work arrived / space freed / stop
  std::condition_variable cv_done;     // waiters: a request finished
  std::condition_variable cv_batch;    // completion thread: a batch was launched
  std::deque<uint64_t> fifo;           // pending tickets in arrival order
  std::deque<uint64_t> active;         // admitted tickets with waves still to launch, in admission order
  std::vector<fcfs::Chunk> chunk_scratch;   // the chunks of the batch being built
  int64_t chunk_waves = fcfs::kDefaultChunkWaves;   // most waves of one request per batch (0: no limit)
  std::unordered_map<uint64_t, fcfs::Ticket> tickets;
  std::deque<fcfs::Batch> inflight;
  std::map<uint64_t, fcfs_plan_t> plans;   // plan cache by (p, q, method, pad)
  int slots_used = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  int fail_allocs = 0;
  int fail_batches = 0;
  uint64_t frees = 0;                  // completions and releases: arena space may have come back
  int max_batch = 0;                   // requests per launch (0: no limit)
  bool discard_outputs = false;

  // statistics of finished requests
  std::vector<double> latencies;
  double first_arrive = -1, last_done = 0;
  double done_bytes = 0;
  int64_t done_count = 0;

  std::chrono::steady_clock::time_point t0;
  std::thread scheduler, completer;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace fcfs {
namespace {

uint64_t plan_key(const fcfs_request& r) {
  return ((uint64_t)r.p << 40) | ((uint64_t)r.q << 20) | ((uint64_t)r.method << 8) | (uint64_t)r.pad;
}

// Input rows some tap reads (height axis) times the row bytes, plus the
// output. Row r is read when r = q m + d for a tap offset d = off[j] + k and a
// cell m < cells; the offsets are few, so each row is checked against them
// (no allocation; called outside the server lock).
uint64_t algorithmic_bytes(const fcfs_plan_* pl, const Ticket& t, size_t es) {
  const AxisTable& a = pl->ah;
  const int64_t h = t.req.h, cells = t.ho / a.p;
  int d[kMaxFactor * 4];
  int nd = 0;
  for (int j = 0; j < a.p; ++j)
    for (int k = 0; k < a.T; ++k) {
      const int v = a.off[j] + k;
      bool seen = false;
      for (int i = 0; i < nd; ++i) seen = seen || d[i] == v;
      if (!seen) d[nd++] = v;
    }
  int64_t rows = 0;
  for (int64_t r = 0; r < h; ++r) {
    bool hit = false;
    for (int i = 0; i < nd && !hit; ++i) {
      const int64_t e = r - d[i];
      hit = e >= 0 && e % a.q == 0 && e / a.q < cells;
    }
    rows += hit;
  }
  return (uint64_t)(t.req.n * t.req.c) * (uint64_t)(rows * t.req.w + t.ho * t.wo) * es;
}

size_t elem_size(int dtype) { return dtype == FCFS_F32 ? 4 : 2; }

int variant_of(int dtype, int taps, int kc) {
  const int ti = taps == 1 ? 0 : (taps == 2 ? 1 : 2);
  return (dtype == FCFS_BF16 ? 6 : 0) + ti * 2 + (kc == 4 ? 0 : 1);
}

// Marks a ticket finished (lock held).
void finish(fcfs_server_* s, Ticket& t, fcfs_status st, double when) {
  t.status = st;
  t.state = kDone;
  t.t_done = when;
  if (t.x_off != SIZE_MAX) {
    s->arena.release(t.x_off, t.x_bytes);
    t.x_off = SIZE_MAX;
    t.x = nullptr;
  }
  if ((st != FCFS_OK || s->discard_outputs) && t.y_off != SIZE_MAX) {
    s->arena.release(t.y_off, t.y_bytes);
    t.y_off = SIZE_MAX;
    t.y = nullptr;
  }
  if (st == FCFS_OK) {
    s->latencies.push_back(t.t_done - t.t_arrive);
    if (s->first_arrive < 0 || t.t_arrive < s->first_arrive) s->first_arrive = t.t_arrive;
    s->last_done = std::max(s->last_done, t.t_done);
    s->done_bytes += (double)t.alg_bytes;
    ++s->done_count;
  }
}

// Arena space for one request (lock held). Returns false when it does not fit now.
bool reserve(fcfs_server_* s, Ticket& t) {
  size_t xo = SIZE_MAX, yo = SIZE_MAX;
  if (!t.req.x) {
    xo = s->arena.alloc(t.x_bytes);
    if (xo == SIZE_MAX) return false;
  }
  if (!t.req.y) {
    yo = s->arena.alloc(t.y_bytes);
    if (yo == SIZE_MAX) {
      if (xo != SIZE_MAX) s->arena.release(xo, t.x_bytes);
      return false;
    }
  }
  t.x_off = xo;
  t.y_off = yo;
  t.x = t.req.x ? const_cast<void*>(t.req.x) : s->arena_base + xo;
  t.y = t.req.y ? t.req.y : s->arena_base + yo;
  return true;
}

// Forward arguments of a request (lock held or not: reads the ticket only).
void fill_desc(const Ticket& t, BatchDesc& d) {
  std::memset(&d, 0, sizeof(d));
  FwdArgs& a = d.args;
  a.x = t.x;
  a.y = t.y;
  a.weight = nullptr;
  a.planes = t.req.n * t.req.c;
  a.C = (int)t.req.c;
  a.H = (int)t.req.h;
  a.W = (int)t.req.w;
  a.Ho = (int)t.ho;
  a.Wo = (int)t.wo;
  a.Mh = (int)(t.ho / t.plan->ah.p);
  a.pad = t.plan->pad;
  a.th = t.plan->ah;
  a.tw_tab = t.plan->aw;
  fill_emit(t.plan->ah, a.emit);
  a.tw = t.geom.tw;
  a.strips = t.geom.strips;
  a.band_cells = t.geom.band_cells;
  a.bands = t.geom.bands;
  a.waves = t.geom.waves;
  d.variant = t.variant;
}

void scheduler_loop(fcfs_server_* s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    StreamBufs& sb = s->sb[s->next_stream];
    s->cv_sched.wait(lk, [&] {
      return (s->stop && s->active.empty()) ||
             (!sb.busy && (!s->active.empty() || (!s->fifo.empty() && s->slots_used < s->max_slots)));
    });
    if (s->stop) {
      // cancel whatever was never admitted; admitted requests run to the end
      const double now = s->now_us();
      while (!s->fifo.empty()) {
        Ticket& t = s->tickets[s->fifo.front()];
        s->fifo.pop_front();
        finish(s, t, FCFS_E_CANCELLED, now);
      }
      s->cv_done.notify_all();
      if (s->active.empty()) break;
      if (sb.busy) continue;
    }
    Batch batch;
    batch.stream = s->next_stream;
    int ngen = 0;
    int64_t waves = 0, gblocks = 0;
    bool wait_other = false;   // a continued chunk reads an input generated on the other stream
    const double now = s->now_us();
    std::vector<Chunk>& chunks = s->chunk_scratch;
    chunks.clear();
    auto add_chunk = [&](uint64_t id, Ticket& t) {
      const int64_t left = t.geom.waves - t.waves_launched;
      const int64_t n = s->chunk_waves > 0 ? std::min(left, s->chunk_waves) : left;
      chunks.push_back(Chunk{t.variant, id, t.waves_launched, n});
      t.waves_launched += n;
      ++t.chunks_inflight;
      batch.tickets.push_back(id);
    };
    // continue the admitted requests that still have waves to launch
    const size_t nactive = s->active.size();
    for (size_t k = 0; k < nactive; ++k) {
      const uint64_t id = s->active.front();
      s->active.pop_front();
      Ticket& t = s->tickets[id];
      if (t.failed) continue;   // an earlier chunk failed: launch nothing more
      if (t.gen_stream >= 0 && t.gen_stream != batch.stream) wait_other = true;
      add_chunk(id, t);
      if (t.waves_launched < t.geom.waves) s->active.push_back(id);
    }
    // admit from the head of the FIFO
    while (!s->stop && !s->fifo.empty() && s->slots_used < s->max_slots &&
           (s->max_batch == 0 || (int)batch.tickets.size() < s->max_batch)) {
      const uint64_t id = s->fifo.front();
      Ticket& t = s->tickets[id];
      const size_t need = (t.req.x ? 0 : round_up(t.x_bytes)) + (t.req.y ? 0 : round_up(t.y_bytes));
      if (need > s->arena.size() || s->fail_allocs > 0) {   // can never fit (or forced): fail it alone
        if (need <= s->arena.size()) --s->fail_allocs;
        s->fifo.pop_front();
        finish(s, t, FCFS_E_NOMEM, now);
        s->cv_done.notify_all();
        continue;
      }
      if (!reserve(s, t)) break;   // wait until completions or releases free space
      s->fifo.pop_front();
      t.state = kAdmitted;
      t.t_start = now;
      ++s->slots_used;
      if (!t.req.x) {
        GenDesc& gd = sb.h_gen[ngen];
        gd.x = t.x;
        gd.count = t.req.n * t.req.c * t.req.h * t.req.w;
        gd.seed = t.req.seed;
        gd.dtype = t.req.dtype;
        sb.h_gblk[ngen] = gblocks;
        gblocks += (gd.count + kGenPerBlock - 1) / kGenPerBlock;
        ++ngen;
        t.gen_stream = batch.stream;
      }
      add_chunk(id, t);
      if (t.waves_launched < t.geom.waves) s->active.push_back(id);
    }
    if (batch.tickets.empty()) {
      // the head request waits for arena space: sleep until a completion or a
      // release returns some
      const uint64_t seen = s->frees;
      s->cv_sched.wait(lk, [&] { return s->stop || s->frees != seen || s->fifo.empty(); });
      continue;
    }
    // the descriptors of the batch's chunks (one launch covers them all: the
    // waves of different requests run side by side)
    const int nreq = (int)chunks.size();
    for (int i = 0; i < nreq; ++i) {
      const Chunk& c = chunks[(size_t)i];
      BatchDesc& d = sb.h_desc[i];
      fill_desc(s->tickets[c.id], d);
      d.wave_begin = c.begin;
      sb.h_wave[i] = waves;
      waves += c.n;
    }
    sb.h_wave[nreq] = waves;
    sb.h_gblk[ngen] = gblocks;
    bool fail = false;
    if (s->fail_batches > 0) {
      --s->fail_batches;
      fail = true;
    }
    // launch (outside the lock: the upload and launches do not touch shared state)
    hipEvent_t other_last = s->sb[batch.stream ^ 1].last;
    sb.busy = true;
    s->next_stream ^= 1;
    lk.unlock();
    hipStream_t st = sb.stream;
    bool ok = !fail;
    // inputs generated by a batch on the other stream must be complete before
    // their later chunks run here (earlier batches of this stream are ordered)
    if (ok && wait_other) ok = hipStreamWaitEvent(st, other_last, 0) == hipSuccess;
    if (ok && ngen > 0) {
      ok = hipMemcpyAsync(sb.d_gen, sb.h_gen, sizeof(GenDesc) * ngen, hipMemcpyHostToDevice, st) == hipSuccess &&
           hipMemcpyAsync(sb.d_gblk, sb.h_gblk, sizeof(int64_t) * (ngen + 1), hipMemcpyHostToDevice, st) ==
               hipSuccess;
      GenArgs ga{sb.d_gen, sb.d_gblk, ngen, gblocks};
      ok = ok && launch_generate(ga, st) == FCFS_OK;
    }
    if (ok) {
      ok = hipMemcpyAsync(sb.d_desc, sb.h_desc, sizeof(BatchDesc) * nreq, hipMemcpyHostToDevice, st) ==
               hipSuccess &&
           hipMemcpyAsync(sb.d_wave, sb.h_wave, sizeof(int64_t) * (nreq + 1), hipMemcpyHostToDevice, st) ==
               hipSuccess;
      BatchArgs ba{sb.d_desc, sb.d_wave, nreq, waves};
      ok = ok && launch_forward_batch(ba, st) == FCFS_OK;
    }
    batch.failed = !ok;
    batch.done = sb.last;
    hipEventRecord(sb.last, st);
    lk.lock();
    s->inflight.push_back(std::move(batch));
    s->cv_batch.notify_all();
  }
}

void completion_loop(fcfs_server_* s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_batch.wait(lk, [&] { return !s->inflight.empty() || (s->stop && s->inflight.empty()); });
    if (s->inflight.empty()) {
      if (s->stop) break;
      continue;
    }
    Batch& b = s->inflight.front();
    hipEvent_t ev = b.done;
    lk.unlock();
    const bool dev_ok = hipEventSynchronize(ev) == hipSuccess;
    lk.lock();
    Batch done = std::move(s->inflight.front());
    s->inflight.pop_front();
    const double when = s->now_us();
    const bool bad = done.failed || !dev_ok;
    for (uint64_t id : done.tickets) {
      Ticket& t = s->tickets[id];
      --t.chunks_inflight;
      if (bad) t.failed = true;
      // a request is done when its last chunk's batch completes
      if (t.chunks_inflight == 0 && (t.waves_launched >= t.geom.waves || t.failed)) {
        if (t.waves_launched < t.geom.waves) {   // failed early: launch none of the rest
          auto it = std::find(s->active.begin(), s->active.end(), id);
          if (it != s->active.end()) s->active.erase(it);
        }
        finish(s, t, t.failed ? FCFS_E_DEVICE : FCFS_OK, when);
        --s->slots_used;
      }
    }
    s->sb[done.stream].busy = false;
    ++s->frees;
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
  }
}

void free_stream_bufs(StreamBufs& b) {
  if (b.h_desc) hipHostFree(b.h_desc);
  if (b.h_wave) hipHostFree(b.h_wave);
  if (b.h_gen) hipHostFree(b.h_gen);
  if (b.h_gblk) hipHostFree(b.h_gblk);
  if (b.d_desc) hipFree(b.d_desc);
  if (b.d_wave) hipFree(b.d_wave);
  if (b.d_gen) hipFree(b.d_gen);
  if (b.d_gblk) hipFree(b.d_gblk);
  if (b.last) hipEventDestroy(b.last);
  if (b.stream) hipStreamDestroy(b.stream);
  b = StreamBufs();
}

fcfs_status fill_result(const Ticket& t, fcfs_result* out) {
  if (out) {
    out->status = t.status;
    out->y = t.status == FCFS_OK ? t.y : nullptr;
    out->h_out = t.ho;
    out->w_out = t.wo;
    out->t_arrive_us = t.t_arrive;
    out->t_start_us = t.t_start;
    out->t_done_us = t.t_done;
  }
  return FCFS_OK;
}

}  // namespace
}  // namespace fcfs

using namespace fcfs;

extern "C" {

fcfs_status fcfs_server_create(int device, size_t mem_budget_bytes, int max_slots, fcfs_server_t* out) {
  if (!out || max_slots < 1 || max_slots > 4096 || mem_budget_bytes < kGranule) return FCFS_E_INVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FCFS_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FCFS_E_DEVICE;
  fcfs_server_* s = new (std::nothrow) fcfs_server_();
  if (!s) return FCFS_E_NOMEM;
  s->device = device;
  s->max_slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  const size_t budget = mem_budget_bytes / kGranule * kGranule;
  if (hipMalloc(reinterpret_cast<void**>(&s->arena_base), budget) != hipSuccess) {
    delete s;
    return FCFS_E_NOMEM;
  }
  s->arena.init(budget);
  bool ok = true;
  for (auto& b : s->sb) {
    ok = ok && hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b.last, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b.h_desc), sizeof(BatchDesc) * max_slots) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b.h_wave), sizeof(int64_t) * (max_slots + 1)) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b.h_gen), sizeof(GenDesc) * max_slots) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b.h_gblk), sizeof(int64_t) * (max_slots + 1)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b.d_desc), sizeof(BatchDesc) * max_slots) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b.d_wave), sizeof(int64_t) * (max_slots + 1)) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b.d_gen), sizeof(GenDesc) * max_slots) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b.d_gblk), sizeof(int64_t) * (max_slots + 1)) == hipSuccess;
  }
  s->chunk_scratch.reserve((size_t)max_slots);
  if (!ok) {
    for (auto& b : s->sb) free_stream_bufs(b);
    hipFree(s->arena_base);
    delete s;
    return FCFS_E_NOMEM;
  }
  s->scheduler = std::thread(scheduler_loop, s);
  s->completer = std::thread(completion_loop, s);
  *out = s;
  return FCFS_OK;
}

fcfs_status fcfs_submit(fcfs_server_t s, const fcfs_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return FCFS_E_INVAL;
  if (r->method != FCFS_NEAREST && r->method != FCFS_BILINEAR && r->method != FCFS_BICUBIC) return FCFS_E_INVAL;
  if (r->dtype != FCFS_F32 && r->dtype != FCFS_BF16) return FCFS_E_INVAL;
  if (r->n < 1 || r->c < 1 || r->h < 1 || r->w < 1) return FCFS_E_INVAL;
  Ticket t;
  t.req = *r;
  {
    // the plan (cached per factor, method and padding; plans live until the
    // server is destroyed, so the pointer stays valid without the lock)
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return FCFS_E_INVAL;
    const uint64_t key = plan_key(*r);
    auto it = s->plans.find(key);
    if (it == s->plans.end()) {
      fcfs_plan_t pl = nullptr;
      fcfs_status st = fcfs_plan(r->p, r->q, r->method, r->pad, &pl);
      if (st != FCFS_OK) return st;
      it = s->plans.emplace(key, pl).first;
    }
    t.plan = it->second;
  }
  // sizes, launch geometry and byte count, outside the lock
  fcfs_output_size(t.plan, r->h, r->w, &t.ho, &t.wo);
  const size_t es = elem_size(r->dtype);
  if (r->h >= (1LL << 31) || r->w >= (1LL << 31) || t.ho >= (1LL << 31) || t.wo >= (1LL << 31))
    return FCFS_E_UNSUPPORTED;
  const int64_t in_plane = r->h * r->w, out_plane = t.ho * t.wo;
  if (in_plane >= (1LL << 31) || out_plane >= (1LL << 31)) return FCFS_E_UNSUPPORTED;
  const int64_t planes_max = INT64_MAX / 4 / std::max(in_plane, out_plane);   // bytes stay below 2^63
  if (r->n > planes_max || r->c > planes_max / r->n) return FCFS_E_UNSUPPORTED;
  t.x_bytes = (size_t)(r->n * r->c * in_plane) * es;
  t.y_bytes = (size_t)(r->n * r->c * out_plane) * es;
  fcfs_status gst = plan_forward_geom_batch(t.plan, r->dtype, r->n * r->c, (int)r->h, (int)r->w, (int)t.ho,
                                            (int)t.wo, &t.geom);
  if (gst != FCFS_OK) return gst;
  t.variant = variant_of(r->dtype, t.plan->ah.T, t.geom.kc);
  t.alg_bytes = algorithmic_bytes(t.plan, t, es);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop) return FCFS_E_INVAL;
  if (s->fifo.size() >= kMaxPending) return FCFS_E_AGAIN;
  t.t_arrive = s->now_us();
  const uint64_t id = s->next_ticket++;
  s->tickets.emplace(id, std::move(t));
  s->fifo.push_back(id);
  *ticket = id;
  s->cv_sched.notify_all();
  return FCFS_OK;
}

fcfs_status fcfs_poll(fcfs_server_t s, uint64_t ticket, fcfs_result* out) {
  if (!s) return FCFS_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return FCFS_E_INVAL;
  if (it->second.state != kDone) return FCFS_E_PENDING;
  return fill_result(it->second, out);
}

fcfs_status fcfs_wait(fcfs_server_t s, uint64_t ticket, int64_t timeout_us, fcfs_result* out) {
  if (!s) return FCFS_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    auto it = s->tickets.find(ticket);
    return it == s->tickets.end() || it->second.state == kDone;
  };
  if (timeout_us < 0) s->cv_done.wait(lk, done);
  else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return FCFS_E_INVAL;
  if (it->second.state != kDone) return FCFS_E_PENDING;
  return fill_result(it->second, out);
}

fcfs_status fcfs_release(fcfs_server_t s, uint64_t ticket) {
  if (!s) return FCFS_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return FCFS_E_INVAL;
  if (it->second.state != kDone) return FCFS_E_PENDING;
  if (it->second.y_off != SIZE_MAX) s->arena.release(it->second.y_off, it->second.y_bytes);
  s->tickets.erase(it);
  ++s->frees;
  s->cv_sched.notify_all();
  return FCFS_OK;
}

fcfs_status fcfs_server_stats(fcfs_server_t s, double* p50_us, double* p99_us, double* req_per_s, double* gbps) {
  if (!s) return FCFS_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->latencies;
  auto pct = [&](double f) -> double {
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(f * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
  };
  if (p50_us) *p50_us = pct(0.50);
  if (p99_us) *p99_us = pct(0.99);
  const double span = s->last_done - s->first_arrive;
  if (req_per_s) *req_per_s = span > 0 ? s->done_count / (span * 1e-6) : 0.0;
  if (gbps) *gbps = span > 0 ? s->done_bytes / (span * 1e-6) / 1e9 : 0.0;
  return FCFS_OK;
}

fcfs_status fcfs_server_debug(fcfs_server_t s, int hook, int64_t value) {
  if (!s || value < 0) return FCFS_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (hook == 1) s->fail_allocs = (int)value;
  else if (hook == 2) s->fail_batches = (int)value;
  else return FCFS_E_INVAL;
  return FCFS_OK;
}

fcfs_status fcfs_server_config(fcfs_server_t s, int option, int64_t value) {
  if (!s || value < 0) return FCFS_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (option == FCFS_SERVER_MAX_BATCH) s->max_batch = (int)std::min<int64_t>(value, 1 << 30);
  else if (option == FCFS_SERVER_DISCARD_OUTPUTS) s->discard_outputs = value != 0;
  else if (option == FCFS_SERVER_CHUNK_WAVES) s->chunk_waves = value;
  else return FCFS_E_INVAL;
  s->cv_sched.notify_all();
  return FCFS_OK;
}

fcfs_status fcfs_server_replay(fcfs_server_t s, const fcfs_request* reqs, const double* arrival_us, int64_t count,
                               uint64_t* tickets) {
  if (!s || count < 0 || (count > 0 && (!reqs || !arrival_us || !tickets))) return FCFS_E_INVAL;
  const auto start = std::chrono::steady_clock::now();
  for (int64_t i = 0; i < count; ++i) {
    const auto due = start + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                 std::chrono::duration<double, std::micro>(arrival_us[i]));
    // sleep while far from the due time, then spin for precision
    for (;;) {
      const auto now = std::chrono::steady_clock::now();
      if (now >= due) break;
      if (due - now > std::chrono::microseconds(200)) std::this_thread::sleep_for(due - now - std::chrono::microseconds(100));
    }
    fcfs_status st;
    while ((st = fcfs_submit(s, &reqs[i], &tickets[i])) == FCFS_E_AGAIN) std::this_thread::yield();
    if (st != FCFS_OK) return st;
  }
  return FCFS_OK;
}

fcfs_status fcfs_server_reset_stats(fcfs_server_t s) {
  if (!s) return FCFS_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->latencies.clear();
  s->first_arrive = -1;
  s->last_done = 0;
  s->done_bytes = 0;
  s->done_count = 0;
  return FCFS_OK;
}

fcfs_status fcfs_server_destroy(fcfs_server_t s) {
  if (!s) return FCFS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
    s->cv_batch.notify_all();
  }
  s->scheduler.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_batch.notify_all();
  }
  s->completer.join();
  hipSetDevice(s->device);
  for (auto& b : s->sb) free_stream_bufs(b);
  hipFree(s->arena_base);
  for (auto& kv : s->plans) fcfs_plan_destroy(kv.second);
  delete s;
  return FCFS_OK;
}

}  // extern "C"
