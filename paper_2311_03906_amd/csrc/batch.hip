// Batched sampling of many (model, shot range) jobs in one persistent launch,
// and capture of launch sequences into HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device_model.hpp"

using sp::set_error;

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return set_error(SP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

// The jobs of one evaluation path (each path has its own kernel).
struct SubBatch {
  int path = SP_PATH_SPARSE;
  sp::BatchJob* jobs = nullptr;        // device
  sp::BatchTask* tasks = nullptr;      // device, persistent schedule
  uint32_t* group_job = nullptr;       // device, flat schedule
  sp::BatchCounters* ctr = nullptr;    // device, persistent schedule
  uint32_t n_jobs = 0, n_tasks = 0, total_groups = 0, n_meas_max = 0, grid = 0;
};

}  // namespace

struct sp_batch {
  SubBatch sub[2];
  int n_sub = 0;
  int schedule = SP_SCHED_PERSISTENT;
  sp_launch launch{};
  int device = 0;
};

struct sp_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host image of one sub-batch before upload.
struct SubPlan {
  int path = SP_PATH_SPARSE;
  std::vector<sp::BatchJob> jobs;
  std::vector<sp::BatchTask> tasks;
  std::vector<uint32_t> group_job;
  uint64_t total_groups = 0;
  uint32_t n_meas_max = 0;
  size_t off_ctr = 0, off_jobs = 0, off_tasks = 0, off_map = 0;
};

struct Plan {
  SubPlan sub[2];
  int n_sub = 0;
  sp_launch launch{};
  size_t total_bytes = 0;
};

// Groups handed out per task: enough Philox blocks per task to amortise the
// hand-out, never more than 32 groups.
uint32_t task_groups(uint32_t nb) { return std::max<uint32_t>(1, std::min<uint32_t>(32, 2048 / std::max<uint32_t>(nb, 1))); }

int make_plan(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule, Plan& P) {
  if (n && !items) return set_error(SP_E_INVALID, "null items");
  if (n > 0xFFFFFFFFull) return set_error(SP_E_LIMIT, "too many items");
  if (schedule != SP_SCHED_PERSISTENT && schedule != SP_SCHED_FLAT) return set_error(SP_E_INVALID, "unknown schedule");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  size_t lds_max = 0;
  uint32_t n_meas_max = 0;
  std::vector<size_t> live;
  for (size_t i = 0; i < n; ++i) {
    const sp_batch_item& it = items[i];
    const std::string at = "item " + std::to_string(i) + ": ";
    if (!it.model) return set_error(SP_E_INVALID, at + "null model");
    if (it.model->device != dev) return set_error(SP_E_INVALID, at + "model on another device");
    lds_max = it.model->lds_max;
    if (it.shots == 0 || it.model->n_meas == 0) continue;
    if (!it.d_out || ((uintptr_t)it.d_out & 7u)) return set_error(SP_E_INVALID, at + "bad output pointer");
    const uint64_t words = (it.shots + 63) / 64;
    if (it.ld_words < words) return set_error(SP_E_INVALID, at + "ld_words < words");
    if (words > 0x7FFFFFFFull) return set_error(SP_E_LIMIT, at + "too many shots");
    if (it.first_shot + it.shots < it.first_shot) return set_error(SP_E_INVALID, at + "shot range overflows");
    n_meas_max = std::max(n_meas_max, it.model->rows_max);
    live.push_back(i);
  }
  if (launch) {
    P.launch = *launch;
  } else {
    P.launch.waves_per_group = 8;
    P.launch.words_per_group =
        (lds_max == 0 || sp::lds_bytes(n_meas_max, 2, 8, SP_PATH_SPARSE) * 3 <= lds_max) ? 2 : 1;
  }
  const sp_launch& L = P.launch;
  if (L.waves_per_group < 1 || L.waves_per_group > 16) return set_error(SP_E_INVALID, "waves_per_group must be 1..16");
  if (L.words_per_group != 1 && L.words_per_group != 2 && L.words_per_group != 4)
    return set_error(SP_E_INVALID, "words_per_group must be 1, 2 or 4");
  if (lds_max && sp::lds_bytes(n_meas_max, L.words_per_group, L.waves_per_group, SP_PATH_SPARSE) > lds_max)
    return set_error(SP_E_LIMIT, "the largest model's slabs exceed the LDS of one workgroup");
  // Heavier groups first: with either schedule the light ones fill the tail.
  std::stable_sort(live.begin(), live.end(), [&](size_t x, size_t y) {
    return items[x].model->nb > items[y].model->nb;
  });
  for (int p : {SP_PATH_SPARSE, SP_PATH_DENSE}) {
    SubPlan S;
    S.path = p;
    for (size_t i : live) {
      const sp_batch_item& it = items[i];
      if (it.model->path != p) continue;
      for (size_t t = 0; t < it.model->tiles.size(); ++t) {   // one job per row tile
      sp::BatchJob J{};
      J.a.m = it.model->tiles[t];
      J.a.out = it.d_out + (size_t)it.model->row0[t] * it.ld_words;
      J.a.ld = it.ld_words;
      J.a.first_shot = it.first_shot;
      J.a.shots = it.shots;
      J.a.key0 = (uint32_t)it.seed;
      J.a.key1 = (uint32_t)(it.seed >> 32);
      const uint64_t words = (it.shots + 63) / 64;
      J.a.n_words = (uint32_t)words;
      J.a.n_groups = (uint32_t)((words + L.words_per_group - 1) / L.words_per_group);
      J.group_base = (uint32_t)S.total_groups;
      S.total_groups += J.a.n_groups;
      if (S.total_groups >= 0x7FFFFFFFull) return set_error(SP_E_LIMIT, "more than 2^31 groups in one batch");
      S.n_meas_max = std::max(S.n_meas_max, J.a.m.n_meas);
      const uint32_t j = (uint32_t)S.jobs.size();
      if (schedule == SP_SCHED_PERSISTENT) {
        const uint32_t k = task_groups(J.a.m.nb);
        for (uint32_t g = 0; g < J.a.n_groups; g += k) S.tasks.push_back({j, g, std::min(k, J.a.n_groups - g), 0});
      } else {
        S.group_job.insert(S.group_job.end(), J.a.n_groups, j);
      }
      S.jobs.push_back(J);
      }
    }
    if (!S.jobs.empty()) P.sub[P.n_sub++] = std::move(S);
  }
  size_t off = 0;
  for (int i = 0; i < P.n_sub; ++i) {
    SubPlan& S = P.sub[i];
    S.off_ctr = off;   off = align256(off + sizeof(sp::BatchCounters));
    S.off_jobs = off;  off = align256(off + sizeof(sp::BatchJob) * S.jobs.size());
    S.off_tasks = off; off = align256(off + sizeof(sp::BatchTask) * S.tasks.size());
    S.off_map = off;   off = align256(off + sizeof(uint32_t) * S.group_job.size());
  }
  P.total_bytes = std::max<size_t>(off, 256);
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_batch_work_bytes(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule, size_t* bytes) {
  if (!bytes) return set_error(SP_E_INVALID, "null argument");
  Plan P;
  try {
    int rc = make_plan(items, n, launch, schedule, P);
    if (rc) return rc;
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  *bytes = P.total_bytes;
  return SP_OK;
}

int sp_batch_create(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule, void* d_work,
                    size_t work_bytes, void* stream, sp_batch** out) {
  if (!out || !d_work) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  if (((uintptr_t)d_work & 255u) != 0) return set_error(SP_E_INVALID, "work buffer must be 256-byte aligned");
  Plan P;
  std::vector<uint8_t> host;
  try {
    int rc = make_plan(items, n, launch, schedule, P);
    if (rc) return rc;
    if (work_bytes < P.total_bytes)
      return set_error(SP_E_INVALID, "work buffer of " + std::to_string(work_bytes) + " bytes, need " +
                                         std::to_string(P.total_bytes));
    host.assign(P.total_bytes, 0);   // counters start at zero
    for (int i = 0; i < P.n_sub; ++i) {
      const SubPlan& S = P.sub[i];
      std::memcpy(&host[S.off_jobs], S.jobs.data(), sizeof(sp::BatchJob) * S.jobs.size());
      if (!S.tasks.empty()) std::memcpy(&host[S.off_tasks], S.tasks.data(), sizeof(sp::BatchTask) * S.tasks.size());
      if (!S.group_job.empty()) std::memcpy(&host[S.off_map], S.group_job.data(), sizeof(uint32_t) * S.group_job.size());
    }
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  uint32_t grids[2] = {0, 0};
  if (schedule == SP_SCHED_PERSISTENT)
    for (int i = 0; i < P.n_sub; ++i) {
      int rc = sp::batch_grid(P.launch, P.sub[i].n_meas_max, P.sub[i].path, &grids[i]);
      if (rc) return rc;
    }
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(d_work, host.data(), P.total_bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  auto* b = new (std::nothrow) sp_batch();
  if (!b) return set_error(SP_E_NOMEM, "out of host memory");
  uint8_t* base = (uint8_t*)d_work;
  b->n_sub = P.n_sub;
  for (int i = 0; i < P.n_sub; ++i) {
    const SubPlan& S = P.sub[i];
    SubBatch& B = b->sub[i];
    B.path = S.path;
    B.ctr = (sp::BatchCounters*)(base + S.off_ctr);
    B.jobs = (sp::BatchJob*)(base + S.off_jobs);
    B.tasks = (sp::BatchTask*)(base + S.off_tasks);
    B.group_job = (uint32_t*)(base + S.off_map);
    B.n_jobs = (uint32_t)S.jobs.size();
    B.n_tasks = (uint32_t)S.tasks.size();
    B.total_groups = (uint32_t)S.total_groups;
    B.n_meas_max = S.n_meas_max;
    B.grid = std::min<uint32_t>(grids[i], std::max<uint32_t>(B.n_tasks, 1));
  }
  b->schedule = schedule;
  b->launch = P.launch;
  HIP_TRY(hipGetDevice(&b->device));
  *out = b;
  return SP_OK;
}

int sp_batch_info(const sp_batch* b, uint32_t* n_jobs, uint32_t* total_groups, uint32_t* grid, sp_launch* launch) {
  if (!b) return set_error(SP_E_INVALID, "null batch");
  uint32_t nj = 0, tg = 0, gr = 0;
  for (int i = 0; i < b->n_sub; ++i) {
    nj += b->sub[i].n_jobs;
    tg += b->sub[i].total_groups;
    gr += b->schedule == SP_SCHED_PERSISTENT ? b->sub[i].grid : b->sub[i].total_groups;
  }
  if (n_jobs) *n_jobs = nj;
  if (total_groups) *total_groups = tg;
  if (grid) *grid = gr;
  if (launch) *launch = b->launch;
  return SP_OK;
}

int sp_batch_launch(const sp_batch* b, void* stream) {
  if (!b) return set_error(SP_E_INVALID, "null batch");
  if (b->n_sub == 0) return SP_OK;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != b->device) return set_error(SP_E_INVALID, "current device differs from the batch's device");
  for (int i = 0; i < b->n_sub; ++i) {
    const SubBatch& B = b->sub[i];
    int rc = b->schedule == SP_SCHED_PERSISTENT
                 ? sp::launch_batch_persistent(B.jobs, B.tasks, B.n_tasks, B.ctr, B.n_meas_max, B.path, b->launch,
                                               B.grid, (hipStream_t)stream)
                 : sp::launch_batch_flat(B.jobs, B.group_job, B.total_groups, B.n_meas_max, B.path, b->launch,
                                         (hipStream_t)stream);
    if (rc) return rc;
  }
  return SP_OK;
}

void sp_batch_free(sp_batch* b) { delete b; }

}  // extern "C"

// ---- batched sampling without device allocation ---------------------------
//
// sp_sample_batch_static keeps a batch's job table, task list (or group map)
// and work counters in `scratch`, a fixed array in the library's device
// image: each GPU the library runs on holds its own copy for the life of the
// process, and every call on that GPU reuses it.  In host code the array's
// name is not a device address; the address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// handed to copies and kernels.

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch (the current device).
int scratch_ptr(int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(SP_E_LIMIT, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(SP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = (uint8_t*)g_scratch_ptr[dev];
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_sample_batch_static(const sp_batch_item* items, size_t n, const sp_launch* launch, int schedule,
                           void* stream) {
  Plan P;
  std::vector<uint8_t> host;
  try {
    int rc = make_plan(items, n, launch, schedule, P);
    if (rc) return rc;
    if (P.n_sub == 0) return SP_OK;
    if (P.total_bytes > kScratchBytes)
      return set_error(SP_E_LIMIT, "batch tables of " + std::to_string(P.total_bytes) + " bytes exceed the " +
                                       std::to_string(kScratchBytes) + "-byte static scratch");
    host.assign(P.total_bytes, 0);   // the work counters start at zero
    for (int i = 0; i < P.n_sub; ++i) {
      const SubPlan& S = P.sub[i];
      std::memcpy(&host[S.off_jobs], S.jobs.data(), sizeof(sp::BatchJob) * S.jobs.size());
      if (!S.tasks.empty()) std::memcpy(&host[S.off_tasks], S.tasks.data(), sizeof(sp::BatchTask) * S.tasks.size());
      if (!S.group_job.empty()) std::memcpy(&host[S.off_map], S.group_job.data(), sizeof(uint32_t) * S.group_job.size());
    }
  } catch (const std::bad_alloc&) {
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  uint8_t* base = nullptr;
  if (int rc = scratch_ptr(dev, &base)) return rc;
  uint32_t grids[2] = {0, 0};
  if (schedule == SP_SCHED_PERSISTENT)
    for (int i = 0; i < P.n_sub; ++i) {
      int rc = sp::batch_grid(P.launch, P.sub[i].n_meas_max, P.sub[i].path, &grids[i]);
      if (rc) return rc;
    }
  // Stream order puts this copy after any earlier launch on `stream` that
  // still reads the scratch; the wait lets the host image go.
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(base, host.data(), P.total_bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < P.n_sub; ++i) {
    const SubPlan& S = P.sub[i];
    const uint32_t n_tasks = (uint32_t)S.tasks.size();
    const int rc =
        schedule == SP_SCHED_PERSISTENT
            ? sp::launch_batch_persistent((const sp::BatchJob*)(base + S.off_jobs),
                                          (const sp::BatchTask*)(base + S.off_tasks), n_tasks,
                                          (sp::BatchCounters*)(base + S.off_ctr), S.n_meas_max, S.path, P.launch,
                                          std::min<uint32_t>(grids[i], std::max<uint32_t>(n_tasks, 1)), s)
            : sp::launch_batch_flat((const sp::BatchJob*)(base + S.off_jobs), (const uint32_t*)(base + S.off_map),
                                    (uint32_t)S.total_groups, S.n_meas_max, S.path, P.launch, s);
    if (rc) return rc;
  }
  return SP_OK;
}

}  // extern "C"

namespace {

// Captures fn(stream) on a private non-blocking stream into an executable graph.
template <class F>
int capture(F fn, sp_graph** out) {
  if (!out) return set_error(SP_E_INVALID, "null argument");
  *out = nullptr;
  hipStream_t s = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(s);
    return set_error(SP_E_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  int rc = fn(s);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  (void)hipStreamDestroy(s);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return set_error(SP_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return set_error(SP_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  auto* G = new (std::nothrow) sp_graph();
  if (!G) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return set_error(SP_E_NOMEM, "out of host memory");
  }
  G->graph = g;
  G->exec = x;
  *out = G;
  return SP_OK;
}

}  // namespace

extern "C" {

int sp_graph_capture_batch(const sp_batch* b, sp_graph** out) {
  if (!b) return set_error(SP_E_INVALID, "null batch");
  return capture([&](hipStream_t s) { return sp_batch_launch(b, (void*)s); }, out);
}

int sp_graph_capture_plain(const sp_batch_item* items, size_t n, sp_graph** out) {
  if (n && !items) return set_error(SP_E_INVALID, "null items");
  return capture(
      [&](hipStream_t s) {
        for (size_t i = 0; i < n; ++i) {
          const sp_batch_item& it = items[i];
          int rc = sp_sample(it.model, it.seed, it.first_shot, it.shots, it.d_out, it.ld_words, (void*)s);
          if (rc) return rc;
        }
        return (int)SP_OK;
      },
      out);
}

int sp_graph_launch(const sp_graph* g, void* stream) {
  if (!g) return set_error(SP_E_INVALID, "null graph");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return SP_OK;
}

void sp_graph_free(sp_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
