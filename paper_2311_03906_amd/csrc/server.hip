// Sampling server: resident models, HBM-budget admission and continuous
// batching.  A scheduler thread owns one HIP stream per tick in flight.  Each tick it
// admits queued requests (FIFO) into free slots whose outputs fit in the
// arena, gives every active request a fair share of the tick's work, and
// samples all of it with one flat batched launch per evaluation path.  Three
// ticks may be in flight on three streams, so one tick's last workgroups
// overlap the next tick's first; when a tick's event completes, the requests whose
// last words it held are done and their slots take new requests.  Every
// output equals what sp_sample would write for the request alone, because
// each draw is keyed by (seed, absolute shot, location).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "device_model.hpp"
#include "server_core.hpp"

using sp::set_error;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kSlots = 3;                  // ticks in flight, one stream each
constexpr uint64_t kDefaultTickCost = 16ull << 20;
constexpr uint32_t kDefaultMaxGroups = 1u << 16;

struct Slot {
  uint8_t* host = nullptr;      // pinned staging
  uint8_t* dev = nullptr;       // in the caller's work buffer
  hipStream_t stream = nullptr; // ticks on different slots overlap on the device
  hipEvent_t ev = nullptr;
  std::vector<sp::serve::Chunk> tick;
  std::string error;
};

struct Layout {
  size_t jobs, map, slot_bytes;
};

Layout layout(uint32_t max_active, uint32_t max_groups) {
  Layout L;
  L.jobs = 0;
  L.map = align256(sizeof(sp::BatchJob) * max_active);
  L.slot_bytes = align256(L.map + sizeof(uint32_t) * (size_t)max_groups);
  return L;
}

}  // namespace

struct sp_server {
  sp_server(const sp_server_config& c, size_t arena_bytes, uint32_t max_groups)
      : cfg(c), sched(arena_bytes, c.max_active, c.max_queued, c.tick_cost, max_groups, c.launch.words_per_group) {}
  sp_server_config cfg;
  sp::serve::Scheduler sched;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread thread;
  bool stop = false;
  int device = 0;
  uint8_t* arena = nullptr;
  uint32_t max_groups = 0;
  Layout L{};
  Slot slot[kSlots];
  std::deque<int> inflight;   // slot indices, oldest first
  uint64_t gen = 0;           // bumped by submit, release and stop
  uint64_t ticks = 0, groups_launched = 0, words_launched = 0;
  std::string thread_error;
};

namespace {

// Fills slot `si` with the jobs of `tick` and queues the copy and launches.
// Called with the mutex held (reads request data).
int stage_and_launch(sp_server* S, int si) {
  Slot& sl = S->slot[si];
  const uint32_t R = S->cfg.launch.words_per_group;
  sp::BatchJob* jobs = (sp::BatchJob*)(sl.host + S->L.jobs);
  uint32_t* map = (uint32_t*)(sl.host + S->L.map);
  uint32_t n_jobs[2] = {0, 0}, groups[2] = {0, 0}, n_meas_max[2] = {0, 0};
  std::vector<uint32_t> order[2];
  for (uint32_t i = 0; i < sl.tick.size(); ++i) {
    const sp::serve::Request* r = S->sched.find(sl.tick[i].ticket);
    order[r->path == SP_PATH_DENSE ? 1 : 0].push_back(i);
  }
  uint32_t j = 0, g = 0;
  for (int p = 0; p < 2; ++p) {
    for (uint32_t i : order[p]) {
      const sp::serve::Chunk& c = sl.tick[i];
      const sp::serve::Request* r = S->sched.find(c.ticket);
      const sp_dmodel* dm = (const sp_dmodel*)r->model;
      sp::BatchJob J{};
      J.a.m = dm->tiles[0];
      J.n_tiles = (uint32_t)dm->tiles.size();
      J.tiles = dm->d_tiles;   // row tiles: the kernel takes each group's tile from the table
      J.a.ld = r->words;
      J.a.out = (uint64_t*)(S->arena + r->off) + c.w0;
      J.a.first_shot = r->first_shot + 64 * c.w0;
      J.a.shots = std::min<uint64_t>(64 * (c.w1 - c.w0), r->shots - 64 * c.w0);
      J.a.key0 = (uint32_t)r->seed;
      J.a.key1 = (uint32_t)(r->seed >> 32);
      J.a.n_words = (uint32_t)(c.w1 - c.w0);
      J.a.n_groups = (J.a.n_words + R - 1) / R;
      J.group_base = groups[p];
      const uint32_t job_groups = J.a.n_groups * J.n_tiles;
      for (uint32_t q = 0; q < job_groups; ++q) map[g + q] = n_jobs[p];
      g += job_groups;
      groups[p] += job_groups;
      n_meas_max[p] = std::max(n_meas_max[p], dm->rows_max);
      jobs[j++] = J;
      ++n_jobs[p];
    }
  }
  // jobs[] holds the sparse jobs then the dense ones; map[] the sparse
  // groups then the dense ones, each numbering jobs within its own path.
  hipError_t e = hipMemcpyAsync(sl.dev + S->L.jobs, sl.host + S->L.jobs, sizeof(sp::BatchJob) * j,
                                hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.dev + S->L.map, sl.host + S->L.map, sizeof(uint32_t) * g, hipMemcpyHostToDevice, sl.stream);
  if (e != hipSuccess) return set_error(SP_E_DEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
  const sp::BatchJob* d_jobs = (const sp::BatchJob*)(sl.dev + S->L.jobs);
  const uint32_t* d_map = (const uint32_t*)(sl.dev + S->L.map);
  for (int p = 0; p < 2; ++p) {
    if (!groups[p]) continue;
    int rc = sp::launch_batch_flat(d_jobs + (p ? n_jobs[0] : 0), d_map + (p ? groups[0] : 0), groups[p], n_meas_max[p],
                                   p ? SP_PATH_DENSE : SP_PATH_SPARSE, S->cfg.launch, sl.stream);
    if (rc) return rc;
  }
  e = hipEventRecord(sl.ev, sl.stream);
  if (e != hipSuccess) return set_error(SP_E_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
  S->ticks++;
  S->groups_launched += groups[0] + groups[1];
  for (const auto& c : sl.tick) S->words_launched += c.w1 - c.w0;
  return SP_OK;
}

void server_loop(sp_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    if (!S->stop) S->sched.admit(now_ns());
    // Keep up to kSlots ticks in flight.
    while (!S->stop && (int)S->inflight.size() < kSlots) {
      int si = 0;
      while (std::find(S->inflight.begin(), S->inflight.end(), si) != S->inflight.end()) ++si;
      Slot& sl = S->slot[si];
      sl.tick = S->sched.next_tick();
      if (sl.tick.empty()) break;
      sl.error.clear();
      if (stage_and_launch(S, si) != SP_OK) {
        sl.error = sp_last_error();   // reported when the tick is retired
        (void)hipEventRecord(sl.ev, sl.stream);
      }
      S->inflight.push_back(si);
    }
    if (S->inflight.empty()) {
      if (S->stop) break;
      // Nothing to run: sleep until a submit, a release or a stop changes
      // what admission can do.
      const uint64_t gen = S->gen;
      S->cv_work.wait(lk, [&] { return S->stop || S->gen != gen; });
      continue;
    }
    // Retire the oldest tick.
    const int si = S->inflight.front();
    Slot& sl = S->slot[si];
    lk.unlock();
    const hipError_t e = hipEventSynchronize(sl.ev);
    const uint64_t t = now_ns();
    lk.lock();
    S->inflight.pop_front();
    const bool ok = e == hipSuccess && sl.error.empty();
    const std::string err = !sl.error.empty() ? sl.error : (e == hipSuccess ? "" : hipGetErrorString(e));
    S->sched.complete(sl.tick, t, ok, err);
    sl.tick.clear();
    S->cv_done.notify_all();
  }
  // Stopping: requests that never ran are reported failed.
  S->sched.fail_all(now_ns(), "server stopped");
  S->cv_done.notify_all();
}

}  // namespace

extern "C" {

int sp_server_work_bytes(const sp_server_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return set_error(SP_E_INVALID, "null argument");
  if (cfg->max_active < 1) return set_error(SP_E_INVALID, "max_active must be >= 1");
  *bytes = (size_t)kSlots * layout(cfg->max_active, kDefaultMaxGroups).slot_bytes;
  return SP_OK;
}

int sp_server_create(const sp_server_config* cfg_in, void* d_arena, size_t arena_bytes, void* d_work,
                     size_t work_bytes, sp_server** out) {
  if (!cfg_in || !d_arena || !d_work || !out) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (((uintptr_t)d_arena & 255u) || ((uintptr_t)d_work & 255u)) return set_error(SP_E_INVALID, "buffers must be 256-byte aligned");
  sp_server_config cfg = *cfg_in;
  if (cfg.max_active < 1) return set_error(SP_E_INVALID, "max_active must be >= 1");
  if (cfg.max_queued < 1) cfg.max_queued = 1u << 20;
  if (cfg.tick_cost == 0) cfg.tick_cost = kDefaultTickCost;
  if (cfg.launch.waves_per_group == 0) cfg.launch.waves_per_group = 8;
  if (cfg.launch.words_per_group == 0) cfg.launch.words_per_group = 1;
  if (cfg.launch.waves_per_group > 16) return set_error(SP_E_INVALID, "waves_per_group must be 1..16");
  if (cfg.launch.words_per_group != 1 && cfg.launch.words_per_group != 2 && cfg.launch.words_per_group != 4)
    return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  const Layout L = layout(cfg.max_active, kDefaultMaxGroups);
  if (work_bytes < (size_t)kSlots * L.slot_bytes)
    return set_error(SP_E_INVALID, "work buffer of " + std::to_string(work_bytes) + " bytes, need " +
                                       std::to_string((size_t)kSlots * L.slot_bytes));
  sp_server* S = new (std::nothrow) sp_server(cfg, arena_bytes, kDefaultMaxGroups);
  if (!S) return set_error(SP_E_NOMEM, "out of host memory");
  S->L = L;
  S->max_groups = kDefaultMaxGroups;
  S->arena = (uint8_t*)d_arena;
  hipError_t e = hipGetDevice(&S->device);
  for (int i = 0; i < kSlots && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&S->slot[i].stream, hipStreamNonBlocking);   // default priority
    if (e != hipSuccess) break;
    S->slot[i].dev = (uint8_t*)d_work + (size_t)i * L.slot_bytes;
    e = hipHostMalloc((void**)&S->slot[i].host, L.slot_bytes, hipHostMallocDefault);
    if (e == hipSuccess) std::memset(S->slot[i].host, 0, L.slot_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->slot[i].ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    std::string msg = std::string("server setup: ") + hipGetErrorString(e);
    for (int i = 0; i < kSlots; ++i) {
      if (S->slot[i].host) (void)hipHostFree(S->slot[i].host);
      if (S->slot[i].ev) (void)hipEventDestroy(S->slot[i].ev);
      if (S->slot[i].stream) (void)hipStreamDestroy(S->slot[i].stream);
    }
    delete S;
    return set_error(SP_E_DEVICE, msg);
  }
  try {
    S->thread = std::thread(server_loop, S);
  } catch (...) {
    for (int i = 0; i < kSlots; ++i) {
      (void)hipHostFree(S->slot[i].host);
      (void)hipEventDestroy(S->slot[i].ev);
      (void)hipStreamDestroy(S->slot[i].stream);
    }
    delete S;
    return set_error(SP_E_NOMEM, "cannot start the scheduler thread");
  }
  *out = S;
  return SP_OK;
}

int sp_server_submit(sp_server* S, const sp_dmodel* model, uint64_t seed, uint64_t first_shot, uint64_t shots,
                     uint64_t* ticket) {
  if (!S || !model || !ticket) return set_error(SP_E_INVALID, "null argument");
  if (model->device != S->device) return set_error(SP_E_INVALID, "model on another device");
  if (first_shot + shots < first_shot) return set_error(SP_E_INVALID, "shot range overflows 64 bits");
  if ((shots + 63) / 64 > 0x7FFFFFFFull) return set_error(SP_E_LIMIT, "too many shots for one request");
  if (sp::lds_bytes(model->rows_max, S->cfg.launch.words_per_group, S->cfg.launch.waves_per_group, model->path) >
      model->lds_max)
    return set_error(SP_E_LIMIT, "the model's slabs exceed the LDS of one workgroup with this launch shape");
  sp::serve::Request r;
  r.model = model;
  r.n_meas = model->n_meas;
  r.nb = model->nb;
  r.tiles = (uint32_t)model->tiles.size();
  r.path = model->path;
  r.seed = seed;
  r.first_shot = first_shot;
  r.shots = shots;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return set_error(SP_E_INVALID, "server is stopping");
  const int rc = S->sched.submit(r, now_ns(), ticket);
  if (rc == 1) return set_error(SP_E_BUDGET, "request output exceeds the server's HBM arena");
  if (rc == 2) return set_error(SP_E_BUDGET, "request queue is full");
  if (rc == 3) return set_error(SP_E_LIMIT, "the model has more row tiles than a tick has workgroups");
  S->gen++;
  S->cv_work.notify_one();
  return SP_OK;
}

static void fill_status(const sp_server* S, const sp::serve::Request& r, sp_request_status* st) {
  st->state = r.state;
  st->d_out = r.state == sp::serve::QUEUED || r.bytes == 0 ? nullptr : (uint64_t*)(S->arena + r.off);
  st->n_meas = r.n_meas;
  st->ld_words = r.words;
  st->t_submit_ns = r.t_submit;
  st->t_admit_ns = r.t_admit;
  st->t_done_ns = r.t_done;
}

int sp_server_status(sp_server* S, uint64_t ticket, sp_request_status* st) {
  if (!S || !st) return set_error(SP_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  const sp::serve::Request* r = S->sched.find(ticket);
  if (!r) return set_error(SP_E_INVALID, "unknown ticket");
  fill_status(S, *r, st);
  if (r->state == sp::serve::FAILED) return set_error(SP_E_DEVICE, r->error);
  return SP_OK;
}

int sp_server_wait(sp_server* S, uint64_t ticket, int64_t timeout_ms, sp_request_status* st) {
  if (!S) return set_error(SP_E_INVALID, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto finished = [&] {
    const sp::serve::Request* r = S->sched.find(ticket);
    return !r || r->state == sp::serve::DONE || r->state == sp::serve::FAILED;
  };
  if (timeout_ms < 0) S->cv_done.wait(lk, finished);
  else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished))
    return set_error(SP_E_TIMEOUT, "request not finished within the timeout");
  const sp::serve::Request* r = S->sched.find(ticket);
  if (!r) return set_error(SP_E_INVALID, "unknown ticket");
  if (st) fill_status(S, *r, st);
  if (r->state == sp::serve::FAILED) return set_error(SP_E_DEVICE, r->error);
  return SP_OK;
}

int sp_server_release(sp_server* S, uint64_t ticket) {
  if (!S) return set_error(SP_E_INVALID, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  const int rc = S->sched.release(ticket);
  if (rc == -1) return set_error(SP_E_INVALID, "unknown ticket");
  if (rc == -2) return set_error(SP_E_INVALID, "request not finished");
  S->gen++;
  S->cv_work.notify_one();   // arena space freed: queued requests may fit now
  return SP_OK;
}

int sp_server_stats(sp_server* S, sp_server_counters* st) {
  if (!S || !st) return set_error(SP_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  st->queued = (uint32_t)S->sched.queued();
  st->active = (uint32_t)S->sched.active();
  st->arena_in_use = S->sched.arena().in_use();
  st->arena_capacity = S->sched.arena().capacity();
  st->ticks = S->ticks;
  st->groups_launched = S->groups_launched;
  st->words_launched = S->words_launched;
  return SP_OK;
}

void sp_server_destroy(sp_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->gen++;
  }
  S->cv_work.notify_all();
  if (S->thread.joinable()) S->thread.join();
  for (int i = 0; i < kSlots; ++i) {
    (void)hipStreamSynchronize(S->slot[i].stream);
    (void)hipHostFree(S->slot[i].host);
    (void)hipEventDestroy(S->slot[i].ev);
    (void)hipStreamDestroy(S->slot[i].stream);
  }
  delete S;
}

}  // extern "C"
