// Host runtime and C ABI of the MPM substep library (declared in
// include/mpm.h). One handle = one scene or a batch of scenes: device
// buffers, the stream, the tool tables, the solver, the binning schedule, the
// recorded graphs, the substep driver and the differentiable rollout.
//
// mpm_step(n) enqueues, for substeps k = 0..n-1 (Algorithm 1 of the paper):
//   k == 0:                    [binning] -> P2G(k)
//   re-binning due, in place:  binning by the positions in memory -> fused
//                              G2P(k-1) + P2G(k)
//   re-binning due, advance:   G2P(k-1) -> binning -> P2G(k)
//   otherwise:                 fused G2P(k-1) + P2G(k)
//   then the grid update of substep k (tools at their substep-k pose),
// and a final G2P, so that x, v, C, F are materialised when the call's work
// completes. Each G2P's position update is followed by the particle push-out
// of the tools that have it on. A PB-MPM substep is one step of `iterations` passes: the first
// as above, then iterations - 1 times fused G2P + P2G within the step, each
// followed by a grid update. Runs of plain substeps replay a recorded HIP
// graph. Nothing here waits on the device except mpm_read_state,
// mpm_get_info, mpm_profile_read, mpm_eval_stress, mpm_autotune, the batch
// particle upload and mpm_destroy.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mpm.h"
#include "mpm_internal.h"
#include "diff_internal.h"

using namespace mpm;

namespace {

// Re-binning interval when mpm_params gives none. Adaptive re-binning (below)
// re-bins earlier where particles drift out of their tiles, and particles
// one cell out still scatter into their tile's shell, so the interval is a
// backstop: on c3 (500 substeps), 256 substeps measured 259.2 us per
// substep against 262.3 at 128 and 260.6 at 512, and 128 against 32 had
// saved more in binning (about 7 us per substep) than the extra particles
// on the global path cost (about 4).
constexpr int kDefaultResort = 256;
// Adaptive re-binning: re-bin before the interval ends once the particles on
// the global path (outside their tiles) average more than this many per
// million per substep since the last binning. Such a particle costs about 25
// times one in its tile (108 global atomics instead of LDS ones), so at
// 0.5% the fused kernel is already about 10% slower, while one in-place
// re-binning costs about one and a half substeps.
constexpr int kDefaultRebinDrift = 5000;
// A drift-triggered re-binning waits at least this many substeps after the
// previous one.
constexpr int kMinDriftInterval = 2;
// With adaptive re-binning on, mpm_step keeps at most this many substeps
// enqueued ahead of the device (so that the fallback count it reads is
// recent): before each launch it waits for the work enqueued kDriftLag
// substeps earlier. The device then still has that many substeps queued.
constexpr int kDriftLag = 8;
constexpr int kDriftEvents = 32;
// Substeps launched one by one leave a progress mark every kDriftMarkEvery
// substeps (an event recorded on the stream costs a few microseconds of GPU
// time), so the host runs at most kDriftLag + kDriftMarkEvery - 1 ahead.
constexpr int kDriftMarkEvery = 4;
constexpr int kDefaultGraphChunk = 8;

struct HostTool {
  mpm_tool t;
  int64_t set_at = 0;
  double R[9];
  bool active = false;
  std::vector<double> vtab;  // optional per-substep linear velocities (rows of 3) from set_at on
  std::vector<double> vpre;  // prefix sums of vtab: vpre[3 j + a] = sum of rows < j
};

// Device buffers of the differentiable rollout (allocated on first use,
// grown as needed) and the record of the last rollout.
struct DiffBufs {
  int64_t generation = 0;  // rollouts recorded since mpm_create
  DiffGrid g;
  int grid_n = 0;
  int64_t part_cap = 0;   // particles the per-particle buffers hold
  float* E = nullptr;     // E per particle, caller order
  float* work = nullptr;  // two particle states
  float* adj = nullptr;   // one adjoint state
  float* ckpt = nullptr;
  int64_t ckpt_slots = 0;
  float* seg = nullptr;
  int64_t seg_slots = 0;
  double* tool_red = nullptr;
  int64_t tool_red_n = 0;
  float4* grids = nullptr;  // per substep: velocity after the grid update, then pre-contact velocity and mass
  int64_t grid_slots = 0;
  bool grids_kept = false;  // the forward kept the grid of every substep (checkpoint_every == 1)
  // Particle orders of the forward pass, one slot per order period (the
  // reverse pass reuses them): sorted caller indices, block ranges, work
  // items and {work items, first position outside the grid}.
  uint32_t* ord_idx = nullptr;
  int64_t ord_idx_n = 0;
  uint32_t* ord_begin = nullptr;
  int64_t ord_begin_n = 0;
  uint32_t* ord_end = nullptr;
  int64_t ord_end_n = 0;
  uint2* ord_work = nullptr;
  int64_t ord_work_n = 0;
  uint32_t* ord_info = nullptr;
  int64_t ord_info_n = 0;
  bool valid = false;     // a rollout is recorded and nothing it depends on changed
  int T = 0, K = 1;
  int64_t start = 0;      // substep counter when the rollout began
  int64_t N = 0;
};

struct ProfEvent {
  int kind;
  hipEvent_t a, b;
};

thread_local std::string g_create_error;

}  // namespace

struct mpm_handle {
  mpm_params p{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int cus = 256;
  Buffers b;
  int nb = 0;
  uint32_t n_blocks = 0;
  int key_bits = 0;
  int64_t N = 0;
  bool has_E = false;
  float mass = 0.0f, vol0 = 0.0f;
  SimK sim{};
  int n_scenes = 1;
  std::vector<HostTool> tools;                // n_scenes x kMaxTools (scene-major)
  std::vector<double*> tool_tables;           // device copies of the velocity tables (vtab then vpre)
  bool tools_dirty = true;                    // device tool descriptors need an upload
  std::vector<int64_t> scene_n;               // particles per scene
  int64_t substep = 0;
  int64_t updates = 0;                        // grid updates since mpm_create (their parity picks the overflow list)
  int pb_iterations = 10;                     // PB-MPM transfer passes per step
  int64_t since_sort = 0;
  bool dirty = true;
  bool fresh_order = true;                    // particles replaced since the last binning: no block counts yet
  int resort_interval = kDefaultResort;
  int64_t resorts = 0;
  int transfer_wgs = 512;
  std::string err;
  bool prof = false;
  int prof_every = 1;   // time the transfer and grid kernels of every prof_every-th substep
  bool prof_now = false;  // this substep's kernels are timed
  std::vector<ProfEvent> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  double prof_ms[MPM_KERNEL_KINDS] = {0, 0, 0, 0, 0};
  int64_t prof_n[MPM_KERNEL_KINDS] = {0, 0, 0, 0, 0};
  unsigned long long* scratch_u64 = nullptr;  // device word for on-demand reductions
  double* imp_sum = nullptr;                  // device: impulse totals of the last mpm_step
  DiffBufs d;
  // Runs of plain substeps (fused transfer + grid update) replayed as HIP
  // graphs: one instance per particle ping-pong half and parity of the first
  // grid update of the run (the kernels take the parity as an argument).
  int graph_chunk = kDefaultGraphChunk;
  int rebin_mode = MPM_REBIN_AUTO;
  int rebin_drift = kDefaultRebinDrift;       // ppm of N per substep on the global path; 0: off
  int64_t sort_substep = 0;                   // substep of the last binning
  // progress marks of the enqueued work (adaptive re-binning): an event after
  // each run of launches and the substep count it ends at, oldest first
  hipEvent_t drift_ev[kDriftEvents] = {};
  int64_t drift_sub[kDriftEvents] = {};
  int drift_head = 0, drift_n = 0;
  hipStream_t cap_stream = nullptr;
  // The rollout backward recomputes the next segment on rec_stream while
  // the adjoint of the current one runs on `stream`.
  hipStream_t rec_stream = nullptr;
  std::vector<hipEvent_t> seg_ev;  // two events per segment: recomputed, differentiated
  hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
};

namespace {

int fail(mpm_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

int hip_fail(mpm_handle* h, hipError_t e, const char* what) {
  return fail(h, MPM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_RETURN(h, expr)                       \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(h, e_, #expr); \
  } while (0)

hipError_t select_device(const mpm_handle* h) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != h->device) return hipSetDevice(h->device);
  return hipSuccess;
}

void quat_to_R(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  const double n = std::sqrt(w * w + x * x + y * y + z * z);
  w /= n, x /= n, y /= n, z /= n;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

// Centre and linear velocity of a tool during global substep k (FP64). The
// pose follows the velocities kinematically: closed form c + (k - set_at) dt v
// without a table; with a table of T rows, substep set_at + j uses row j and
// the centre is c plus dt times the sum of the earlier rows; after the table
// the constant velocity resumes from where the table left the tool.
void tool_kinematics(const HostTool& ht, int64_t k, double dt, double* pose, double* vel) {
  const int64_t rel = k - ht.set_at;
  const int64_t T = (int64_t)(ht.vtab.size() / 3);
  if (T == 0) {
    const double el = (double)rel * dt;
    for (int a = 0; a < 3; ++a) pose[a] = ht.t.center[a] + el * ht.t.lin_vel[a], vel[a] = ht.t.lin_vel[a];
    return;
  }
  const int64_t m = rel < T ? rel : T;
  for (int a = 0; a < 3; ++a) {
    pose[a] = ht.t.center[a] + dt * ht.vpre[3 * m + a] + (double)(rel - m) * dt * ht.t.lin_vel[a];
    vel[a] = rel < T ? ht.vtab[3 * rel + a] : ht.t.lin_vel[a];
  }
}

// Squared distance from the tool centre beyond which no point is in contact
// (a conservative bound with slack for FP32 rounding); -1 for the unbounded
// plane.
float reach2_of(const mpm_tool& t) {
  const double m = t.margin > 0.0f ? (double)t.margin : 0.0;
  double r;
  switch (t.type) {
    case MPM_TOOL_CAPSULE: r = t.size[0] + t.size[1] + m; break;
    case MPM_TOOL_BOX: r = std::sqrt(t.size[0] * t.size[0] + t.size[1] * t.size[1] + t.size[2] * t.size[2]) + m; break;
    case MPM_TOOL_SLICER: r = std::sqrt(t.size[0] * t.size[0] + t.size[1] * t.size[1]) + m; break;
    case MPM_TOOL_SEGMENT: r = t.size[0] + t.size[1]; break;
    case MPM_TOOL_ARC: r = t.size[0] + t.size[2]; break;
    default: return -1.0f;
  }
  r = r * 1.001 + 1e-6;
  return (float)(r * r);
}

// Tools at the pose of global substep `k` (FP64 kinematics, then rounded to
// FP32).
ToolSetK tools_at(const mpm_handle* h, int64_t k) {
  ToolSetK ts;
  std::memset(&ts, 0, sizeof(ts));
  ts.n = 0;
  for (int i = 0; i < kMaxTools; ++i) {
    const HostTool& ht = h->tools[i];
    ToolK& t = ts.t[i];
    if (!ht.active) {
      t.type = TOOL_NONE;
      continue;
    }
    ts.n = i + 1;
    t.type = ht.t.type;
    double pose[3], vel[3];
    tool_kinematics(ht, k, (double)h->p.dt, pose, vel);
    for (int a = 0; a < 3; ++a) {
      t.c[a] = (float)pose[a];
      t.size[a] = (float)ht.t.size[a];
      t.lv[a] = (float)vel[a];
      t.av[a] = (float)ht.t.ang_vel[a];
    }
    for (int i2 = 0; i2 < 9; ++i2) t.R[i2] = (float)ht.R[i2];
    t.mu = ht.t.mu;
    t.drag = ht.t.drag;
    t.margin = ht.t.margin;
    t.reach2 = reach2_of(ht.t);
  }
  return ts;
}

hipEvent_t prof_event(mpm_handle* h) {
  if (!h->prof_pool.empty()) {
    hipEvent_t e = h->prof_pool.back();
    h->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  mpm_handle* h;
  int kind;
  hipEvent_t a = nullptr;
  ProfScope(mpm_handle* hh, int k) : h(hh), kind(k) {
    if (h->prof) {
      a = prof_event(h);
      if (a) (void)hipEventRecord(a, h->stream);
    }
  }
  ~ProfScope() {
    if (h->prof && a) {
      hipEvent_t b = prof_event(h);
      if (b) {
        (void)hipEventRecord(b, h->stream);
        h->prof_pending.push_back({kind, a, b});
      } else {
        h->prof_pool.push_back(a);
      }
    }
  }
};

// The events of one timed kernel launch, recorded by the launch itself
// (KernelEvents; none when not timing), queued for prof_collect.
struct KernelTimer {
  mpm_handle* h;
  int kind;
  KernelEvents ev;
  KernelTimer(mpm_handle* hh, int k) : h(hh), kind(k) {
    if (!h->prof_now) return;
    ev.start = prof_event(h);
    ev.stop = ev.start ? prof_event(h) : nullptr;
    if (!ev.stop) {
      if (ev.start) h->prof_pool.push_back(ev.start);
      ev = KernelEvents();
    }
  }
  ~KernelTimer() {
    if (ev.start) h->prof_pending.push_back({kind, ev.start, ev.stop});
  }
};

void prof_collect(mpm_handle* h) {
  for (auto& pe : h->prof_pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
      h->prof_ms[pe.kind] += ms;
      h->prof_n[pe.kind] += 1;
    }
    h->prof_pool.push_back(pe.a);
    h->prof_pool.push_back(pe.b);
  }
  h->prof_pending.clear();
}

void drop_graphs(mpm_handle* h) {
  for (int i = 0; i < 2; ++i)
    for (int p = 0; p < 2; ++p)
      if (h->graph[i][p]) {
        (void)hipGraphExecDestroy(h->graph[i][p]);
        h->graph[i][p] = nullptr;
      }
}

// Persistent transfer workgroups for a work tile edge: two 512-thread
// workgroups per CU for 8-cell tiles (their 44 KB LDS tiles bound it), eight
// 128-thread ones for 4-cell tiles (registers bound it at 16 waves per CU);
// a multiple of 8 (one share per XCD).
int default_transfer_wgs(const mpm_handle* h, int tile) {
  const int per_cu = tile == 4 ? 8 : 2;
  return (per_cu * h->cus + 7) / 8 * 8;
}

// Particles per transfer work item: about N / (4 x workgroups), so that
// even a scene of a few dense tiles gives every persistent workgroup several
// items, as a power of two in [kItemMin, kItemMax] for 8-cell tiles and a
// quarter of that for 4-cell tiles (whose workgroups are a quarter the
// size). A change re-bins and drops the recorded graphs.
void choose_item_size(mpm_handle* h) {
  const int64_t target = h->N / (4 * (int64_t)h->transfer_wgs);
  const unsigned lo = h->sim.tile == 4 ? kItemMin / 4 : kItemMin, hi = h->sim.tile == 4 ? kItemMax / 4 : kItemMax;
  unsigned item = lo;
  while (item < hi && (int64_t)item * 2 <= target) item *= 2;
  if (item != h->sim.item_particles) {
    h->sim.item_particles = item;
    h->dirty = true;
    drop_graphs(h);
  }
}

// Use work tiles of edge `tile` (4 or 8) from the next binning on: the tile
// ranges of the previous sort are in the other indexing, so new orders are
// built as for new particles, and recorded graphs are dropped.
void set_tile(mpm_handle* h, int tile) {
  if (tile == h->sim.tile) return;
  h->sim.tile = tile;
  h->sim.unit_shift = tile == 4 ? 3 : 0;
  h->dirty = true;
  h->fresh_order = true;
  drop_graphs(h);
  choose_item_size(h);  // item sizes are bounded per tile edge
}

void free_buffers(Buffers& b) {
  void* ptrs[] = {b.part[0], b.part[1], b.id[0], b.id[1], b.keys[0], b.keys[1], b.vals[0], b.vals[1],
                  b.hist, b.scan_tmp, b.blk_begin, b.blk_end, b.flags, b.occ_list, b.work, b.work_tmp, b.act_list, b.mark,
                  b.ovf_list[0], b.ovf_list[1], b.node_cnt, b.imp_blocks, b.acc_m, b.acc_p[0], b.acc_p[1], b.acc_p[2], b.vel,
                  b.status, b.scene_off, b.tools, b.clock, b.pbound[0], b.pbound[1]};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (b.drift_host) (void)hipHostFree(b.drift_host);
  b = Buffers();
}

void free_diff(DiffBufs& d) {
  void* ptrs[] = {d.g.m, d.g.p[0], d.g.p[1], d.g.p[2], d.g.vel, d.g.vb[0], d.g.vb[1], d.g.vb[2], d.g.pb,
                  d.g.skip, d.E, d.work, d.adj, d.ckpt, d.seg, d.tool_red, d.grids,
                  d.ord_idx, d.ord_begin, d.ord_end, d.ord_work, d.ord_info};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  d = DiffBufs();
}

__global__ void k_reset_status(Status* st) {
  st->n_inverted = 0ull;
  st->n_domain = 0ull;
  st->n_nonfinite = 0ull;
  st->n_fallback = 0ull;
  st->n_range = 0ull;
  st->n_occ = 0u;
  st->n_work = 0u;
  st->n_act = 0u;
  st->ovf_count[0] = 0u;
  st->ovf_count[1] = 0u;
  st->fb_at_sort = 0ull;
  for (int i = 0; i < kXcds; ++i) st->claim[i] = st->claim_done[i] = 0u;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_zero_f4(float4* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

int pending_status(mpm_handle* h, Status* out) {
  Status st;
  HIP_OR_RETURN(h, hipMemcpy(&st, h->b.status, sizeof(Status), hipMemcpyDeviceToHost));
  if (out) *out = st;
  if (st.n_nonfinite) return fail(h, MPM_ENONFINITE, "non-finite particle state");
  if (st.n_domain) return fail(h, MPM_EDOMAIN, "a particle stencil left the grid");
  if (st.n_range) return fail(h, MPM_ERANGE, "a P2G contribution exceeded the fixed-point range");
  if (st.n_inverted) return fail(h, MPM_EINVERTED, "det F <= 0 in the stress evaluation");
  return MPM_OK;
}

int sync(mpm_handle* h) {
  HIP_OR_RETURN(h, hipStreamSynchronize(h->stream));
  HIP_OR_RETURN(h, hipGetLastError());
  return MPM_OK;
}

}  // namespace

// ====================================================================== C ABI
namespace {

// (Re)allocate a device buffer to hold at least `need` elements of `elem`
// bytes; `have` tracks the current capacity in elements.
int alloc_fail(mpm_handle* h, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(h, MPM_ENOMEM, std::string(what) + ": out of device memory");
  return hip_fail(h, e, what);
}

#define ALLOC_OR_RETURN(h, expr)                         \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return alloc_fail(h, e_, #expr); \
  } while (0)

template <typename T>
hipError_t ensure(T** p, int64_t* have, int64_t need, size_t elem = sizeof(T)) {
  if (*p && *have >= need) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipMalloc((void**)p, (size_t)(need > 0 ? need : 1) * elem);
  if (e == hipSuccess) *have = need;
  return e;
}

hipError_t diff_alloc_base(mpm_handle* h) {
  DiffBufs& d = h->d;
  const int n = h->p.n_grid;
  const int64_t nn = (int64_t)n * n * n;
  if (d.grid_n != n) {
    void* ptrs[] = {d.g.m, d.g.p[0], d.g.p[1], d.g.p[2], d.g.vel, d.g.vb[0], d.g.vb[1], d.g.vb[2], d.g.pb};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    DiffGrid z;
    z.skip = d.g.skip;
    d.g = z;
    d.grid_n = 0;
    hipError_t e;
    if ((e = hipMalloc((void**)&d.g.m, sizeof(float) * nn)) != hipSuccess) return e;
    for (int a = 0; a < 3; ++a) {
      if ((e = hipMalloc((void**)&d.g.p[a], sizeof(float) * nn)) != hipSuccess) return e;
      if ((e = hipMalloc((void**)&d.g.vb[a], sizeof(float) * nn)) != hipSuccess) return e;
    }
    if ((e = hipMalloc((void**)&d.g.vel, sizeof(float4) * nn)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&d.g.pb, sizeof(float4) * nn)) != hipSuccess) return e;
    d.grid_n = n;
  }
  const int64_t N = h->N;
  if (d.part_cap < N) {
    void* ptrs[] = {d.g.skip, d.E, d.work, d.adj};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    d.g.skip = nullptr, d.E = nullptr, d.work = nullptr, d.adj = nullptr;
    d.part_cap = 0;
    hipError_t e;
    if ((e = hipMalloc((void**)&d.g.skip, (size_t)N)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&d.E, sizeof(float) * N)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&d.work, sizeof(float) * 2 * kStateFloats * N)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&d.adj, sizeof(float) * kStateFloats * N)) != hipSuccess) return e;
    d.part_cap = N;
  }
  // Accumulators the kernels expect to find cleared.
  for (int a = 0; a < 3; ++a) {
    launch_fill_f32(d.g.p[a], nn, 0.0f, h->stream);
    launch_fill_f32(d.g.vb[a], nn, 0.0f, h->stream);
  }
  launch_fill_f32(d.g.m, nn, 0.0f, h->stream);
  return hipGetLastError();
}

// Substeps that share one particle order in a rollout: a multiple of the
// checkpoint interval (so that the state an order is taken from is a
// checkpoint in the reverse pass too) near 16.
int order_period(int K) { return K * std::max(1, 16 / K); }

// Work items an order can hold: one partial run per block plus one per
// kItemRollout particles.
int64_t order_work_cap(const mpm_handle* h) { return (int64_t)h->sim.nb3 + h->N / kItemRollout + 1; }

// Room for `periods` orders of the current particle set.
hipError_t alloc_orders(mpm_handle* h, int periods) {
  DiffBufs& d = h->d;
  const int64_t P = periods > 0 ? periods : 1;
  hipError_t e = ensure(&d.ord_idx, &d.ord_idx_n, P * (h->N > 0 ? h->N : 1));
  if (e == hipSuccess) e = ensure(&d.ord_begin, &d.ord_begin_n, P * (int64_t)h->sim.nb3);
  if (e == hipSuccess) e = ensure(&d.ord_end, &d.ord_end_n, P * (int64_t)h->sim.nb3);
  if (e == hipSuccess) e = ensure(&d.ord_work, &d.ord_work_n, P * order_work_cap(h));
  if (e == hipSuccess) e = ensure(&d.ord_info, &d.ord_info_n, P * 2);
  return e;
}

// Order slot `period` as the scatter kernels take it.
DiffOrder order_slot(const mpm_handle* h, int period) {
  const DiffBufs& d = h->d;
  return DiffOrder{d.ord_idx + (int64_t)period * h->N, d.ord_end + (int64_t)period * h->sim.nb3,
                   d.ord_work + (int64_t)period * order_work_cap(h), d.ord_info + 2 * (int64_t)period};
}

// Spatial order of the rollout state `x` (caller order) for the scatters,
// computed into order slot `period`.
hipError_t rollout_order(mpm_handle* h, const float* x, int period) {
  DiffBufs& d = h->d;
  return launch_order(h->b, h->N, h->sim, x, h->key_bits, kItemRollout, d.ord_idx + (int64_t)period * h->N,
                      d.ord_begin + (int64_t)period * h->sim.nb3, d.ord_end + (int64_t)period * h->sim.nb3,
                      d.ord_work + (int64_t)period * order_work_cap(h), d.ord_info + 2 * (int64_t)period,
                      h->stream);
}

}  // namespace

extern "C" {

namespace {

int create_impl(const mpm_params* p, int32_t n_scenes, uint64_t hip_stream, mpm_handle** out) {
  g_create_error.clear();
  noalloc_clear_error();
  if (!out) {
    g_create_error = "out is NULL";
    return MPM_EINVAL;
  }
  *out = nullptr;
  if (!p) {
    g_create_error = "params is NULL";
    return MPM_EINVAL;
  }
  if (p->n_grid < 8 || p->n_grid > 1024 || !(p->dt > 0.0f) || !std::isfinite(p->dt) ||
      !(p->nu >= 0.0f && p->nu < 0.5f) || !(p->E_default >= 0.0f) || !std::isfinite(p->E_default) ||
      p->wall_band < 0 || p->wall_band > p->n_grid / 2 ||
      !(p->accum_mode == MPM_ACCUM_F32 || p->accum_mode == MPM_ACCUM_FIXED) ||
      !(p->tile == 0 || p->tile == 4 || p->tile == 8) ||
      p->resort_interval < 0 || p->max_particles < 0 || p->max_particles > 0x7fffffffLL ||
      !std::isfinite(p->gravity[0]) || !std::isfinite(p->gravity[1]) || !std::isfinite(p->gravity[2]) ||
      n_scenes < 1) {
    g_create_error = "parameter out of range";
    return MPM_EINVAL;
  }
  {
    // Node indices of the whole batch must fit an int.
    const int64_t nb = (p->n_grid + kTile - 1) / kTile;
    if ((int64_t)n_scenes * nb * nb * nb * kBlockNodes >= (1ll << 31)) {
      g_create_error = "n_scenes x grid nodes exceeds 2^31";
      return MPM_EINVAL;
    }
  }
  mpm_handle* h = new (std::nothrow) mpm_handle();
  if (!h) {
    g_create_error = "host allocation failed";
    return MPM_ENOMEM;
  }
  h->p = *p;
  if (h->p.tile == 0) h->p.tile = 8;
  h->n_scenes = n_scenes;
  h->tools.assign((size_t)n_scenes * kMaxTools, HostTool());
  h->tool_tables.assign((size_t)n_scenes * kMaxTools, nullptr);
  h->scene_n.assign((size_t)n_scenes, 0);
  h->resort_interval = p->resort_interval > 0 ? p->resort_interval : kDefaultResort;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
    delete h;
    return MPM_EHIP;
  }
  if (hip_stream) {
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreate(&h->stream);
    if (e != hipSuccess) {
      g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
      delete h;
      return MPM_EHIP;
    }
    h->own_stream = true;
  }
  const int n = p->n_grid;
  h->nb = (n + kTile - 1) / kTile;
  const uint32_t nb3 = (uint32_t)h->nb * h->nb * h->nb;
  h->n_blocks = nb3 * (uint32_t)n_scenes;
  int bits = 1;
  while ((1u << bits) < h->n_blocks + 1u) ++bits;
  h->key_bits = bits;
  // Persistent transfer grid: two 8-cell-tile workgroups per CU (LDS bound)
  // or eight 4-cell-tile ones (VGPR bound), a multiple of 8.
  h->transfer_wgs = default_transfer_wgs(h, h->p.tile);

  const int64_t cap = p->max_particles > 0 ? p->max_particles : 1;
  Buffers& b = h->b;
  b.cap = cap;
  const int64_t n_tiles = (cap + 4095) / 4096;
  const int64_t hist_n = 256 * n_tiles;
  const int64_t n_units_max = (int64_t)h->n_blocks << kMaxUnitShift;  // 4-cell work tiles
  const int64_t scan_part = (std::max<int64_t>(hist_n, n_units_max) + 2047) / 2048 + 1;
  const size_t grid_nodes = (size_t)h->n_blocks * kBlockNodes;
  bool ok = true;
  auto alloc = [&](void** ptr, size_t bytes) {
    if (!ok) return;
    if (hipMalloc(ptr, bytes) != hipSuccess) ok = false;
  };
  for (int i = 0; i < 2; ++i) {
    alloc((void**)&b.part[i], sizeof(float) * kFields * cap);
    alloc((void**)&b.id[i], sizeof(uint32_t) * cap);
    alloc((void**)&b.keys[i], sizeof(uint32_t) * cap);
    alloc((void**)&b.vals[i], sizeof(uint32_t) * cap);
    alloc((void**)&b.ovf_list[i], sizeof(uint32_t) * h->n_blocks);
    alloc((void**)&b.pbound[i], sizeof(unsigned long long) * n_units_max);
  }
  alloc((void**)&b.hist, sizeof(uint32_t) * hist_n);
  alloc((void**)&b.scan_tmp, sizeof(uint32_t) * scan_part);
  alloc((void**)&b.blk_begin, sizeof(uint32_t) * n_units_max);
  alloc((void**)&b.blk_end, sizeof(uint32_t) * n_units_max);
  alloc((void**)&b.flags, sizeof(uint32_t) * n_units_max);
  alloc((void**)&b.occ_list, sizeof(uint32_t) * n_units_max);
  // at most one partial item per occupied work tile plus one per
  // kItemMinAny (the smallest item of any tile edge or of the rollout) particles
  alloc((void**)&b.work, sizeof(uint2) * ((size_t)n_units_max + (size_t)(cap / kItemMinAny) + 1));
  alloc((void**)&b.work_tmp, sizeof(uint2) * ((size_t)n_units_max + (size_t)(cap / kItemMinAny) + 1));
  alloc((void**)&b.act_list, sizeof(uint32_t) * h->n_blocks);
  alloc((void**)&b.mark, sizeof(uint32_t) * h->n_blocks);
  alloc((void**)&b.node_cnt, sizeof(uint32_t) * h->n_blocks);
  alloc((void**)&b.imp_blocks, sizeof(float) * (size_t)h->n_blocks * kImpulseRows * 3);
  alloc((void**)&b.scene_off, sizeof(uint32_t) * ((size_t)n_scenes + 1));
  alloc((void**)&b.tools, sizeof(ToolDesc) * (size_t)n_scenes * kMaxTools);
  alloc((void**)&b.clock, 2 * sizeof(Clock));
  if (ok && hipHostMalloc((void**)&b.drift_host, 4 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
    ok = false;
  if (ok) std::memset(b.drift_host, 0, 4 * sizeof(unsigned long long));
  alloc((void**)&h->imp_sum, sizeof(double) * kImpulseRows * 3);
  alloc((void**)&h->scratch_u64, sizeof(unsigned long long));
  const size_t mom_bytes = p->accum_mode == MPM_ACCUM_FIXED ? sizeof(long long) : sizeof(float);
  alloc(&b.acc_m, sizeof(float) * grid_nodes);  // weights: float or u32
  for (int a = 0; a < 3; ++a) alloc(&b.acc_p[a], mom_bytes * grid_nodes);
  alloc((void**)&b.vel, sizeof(float4) * grid_nodes);
  alloc((void**)&b.status, sizeof(Status));
  if (!ok) {
    free_buffers(b);
    if (h->scratch_u64) (void)hipFree(h->scratch_u64);
    if (h->imp_sum) (void)hipFree(h->imp_sum);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    g_create_error = "device allocation failed";
    return MPM_ENOMEM;
  }
  // The accumulator must start (and stay, outside a substep) at zero.
  hipLaunchKernelGGL(k_zero_u32, dim3(4096), dim3(256), 0, h->stream, (uint32_t*)b.acc_m, (int64_t)grid_nodes);
  for (int a = 0; a < 3; ++a)
    hipLaunchKernelGGL(k_zero_u32, dim3(4096), dim3(256), 0, h->stream, (uint32_t*)b.acc_p[a],
                       (int64_t)(grid_nodes * mom_bytes / 4));
  hipLaunchKernelGGL(k_zero_f4, dim3(4096), dim3(256), 0, h->stream, b.vel, (int64_t)grid_nodes);
  // Block ranges of the previous sort, read by the binning keys: none yet.
  hipLaunchKernelGGL(k_zero_u32, dim3(256), dim3(256), 0, h->stream, b.blk_begin, n_units_max);
  hipLaunchKernelGGL(k_zero_u32, dim3(256), dim3(256), 0, h->stream, b.blk_end, n_units_max);
  for (int i = 0; i < 2; ++i)  // no bound recorded yet (substep stamp 0, value 0)
    hipLaunchKernelGGL(k_zero_u32, dim3(256), dim3(256), 0, h->stream, (uint32_t*)b.pbound[i], 2 * n_units_max);
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(1), 0, h->stream, b.status);
  launch_set_clock(b, 0, 0, h->stream);
  // Scene constants.
  SimK& s = h->sim;
  s.n = n;
  s.nb = h->nb;
  s.n_scenes = n_scenes;
  s.nb3 = nb3;
  s.n3 = (int)(nb3 * kBlockNodes);
  s.solver = SOLVER_MLS;
  s.pb_beta = 0.5f;
  s.item_particles = kItemMax;
  set_tile(h, h->p.tile);
  launch_clear_impulses(b, s, h->stream);
  e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    g_create_error = std::string("initialisation: ") + hipGetErrorString(e);
    free_buffers(b);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return MPM_EHIP;
  }
  s.dx = (float)(1.0 / n);
  s.inv_dx = (float)n;
  s.dt = p->dt;
  s.band = p->wall_band;
  s.E_default = p->E_default;
  const double nu = p->nu;
  s.c_mu = (float)(1.0 / (2.0 * (1.0 + nu)));
  s.c_la = (float)(nu / ((1.0 + nu) * (1.0 - 2.0 * nu)));
  for (int a = 0; a < 3; ++a) s.g[a] = p->gravity[a];
  s.fixed = p->accum_mode == MPM_ACCUM_FIXED ? 1 : 0;
  *out = h;
  return MPM_OK;
}

}  // namespace

int mpm_create(const mpm_params* p, uint64_t hip_stream, mpm_handle** out) {
  return create_impl(p, 1, hip_stream, out);
}

int mpm_create_batch(const mpm_params* p, int32_t n_scenes, uint64_t hip_stream, mpm_handle** out) {
  return create_impl(p, n_scenes, hip_stream, out);
}

int mpm_destroy(mpm_handle* h) {
  if (!h) return MPM_OK;
  int rc = MPM_OK;
  if (select_device(h) == hipSuccess && hipStreamSynchronize(h->stream) == hipSuccess) {
    rc = pending_status(h, nullptr);
  } else {
    rc = MPM_EHIP;
  }
  for (auto& pe : h->prof_pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  for (auto e : h->prof_pool) (void)hipEventDestroy(e);
  for (auto e : h->drift_ev)
    if (e) (void)hipEventDestroy(e);
  drop_graphs(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->rec_stream) (void)hipStreamDestroy(h->rec_stream);
  for (auto e : h->seg_ev) (void)hipEventDestroy(e);
  free_buffers(h->b);
  free_diff(h->d);
  for (double* t : h->tool_tables)
    if (t) (void)hipFree(t);
  if (h->scratch_u64) (void)hipFree(h->scratch_u64);
  if (h->imp_sum) (void)hipFree(h->imp_sum);
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return rc;
}

namespace {

int set_particles_impl(mpm_handle* h, const int64_t* counts, const float* x, const float* v, const float* C,
                       const float* F, const float* E, float mass, float vol0, int32_t where) {
  int64_t n = 0;
  for (int sc = 0; sc < h->n_scenes; ++sc) {
    if (counts[sc] < 0) return fail(h, MPM_EINVAL, "mpm_set_particles: negative count");
    n += counts[sc];
  }
  if (n > h->b.cap || (n > 0 && !x) || !(mass > 0.0f) || !(vol0 > 0.0f) ||
      !std::isfinite(mass) || !std::isfinite(vol0) || (where != MPM_HOST && where != MPM_DEVICE))
    return fail(h, MPM_EINVAL, "mpm_set_particles: argument out of range");
  HIP_OR_RETURN(h, select_device(h));
  if (h->n_scenes > 1) {
    // Scene offsets for the key generation (original particle order).
    std::vector<uint32_t> off((size_t)h->n_scenes + 1, 0u);
    for (int sc = 0; sc < h->n_scenes; ++sc) off[sc + 1] = off[sc] + (uint32_t)counts[sc];
    HIP_OR_RETURN(h, hipMemcpyAsync(h->b.scene_off, off.data(), sizeof(uint32_t) * off.size(),
                                    hipMemcpyHostToDevice, h->stream));
    HIP_OR_RETURN(h, hipStreamSynchronize(h->stream));
  }
  for (int sc = 0; sc < h->n_scenes; ++sc) h->scene_n[sc] = counts[sc];
  Buffers& b = h->b;
  const float* dx = x;
  const float* dv = v;
  const float* dC = C;
  const float* dF = F;
  const float* dE = E;
  if (where == MPM_HOST && n > 0) {
    // Stage the AoS inputs in the idle half of the particle ping-pong.
    float* stg = b.part[b.cur ^ 1];
    float* sx = stg;
    float* sv = stg + 3 * n;
    float* sC = stg + 6 * n;
    float* sF = stg + 15 * n;
    float* sE = stg + 24 * n;
    HIP_OR_RETURN(h, hipMemcpyAsync(sx, x, sizeof(float) * 3 * n, hipMemcpyHostToDevice, h->stream));
    if (v) HIP_OR_RETURN(h, hipMemcpyAsync(sv, v, sizeof(float) * 3 * n, hipMemcpyHostToDevice, h->stream));
    if (C) HIP_OR_RETURN(h, hipMemcpyAsync(sC, C, sizeof(float) * 9 * n, hipMemcpyHostToDevice, h->stream));
    if (F) HIP_OR_RETURN(h, hipMemcpyAsync(sF, F, sizeof(float) * 9 * n, hipMemcpyHostToDevice, h->stream));
    if (E) HIP_OR_RETURN(h, hipMemcpyAsync(sE, E, sizeof(float) * n, hipMemcpyHostToDevice, h->stream));
    dx = sx;
    dv = v ? sv : nullptr;
    dC = C ? sC : nullptr;
    dF = F ? sF : nullptr;
    dE = E ? sE : nullptr;
  }
  launch_load_particles(b, n, dx, dv, dC, dF, dE, h->stream);
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(1), 0, h->stream, b.status);
  HIP_OR_RETURN(h, hipGetLastError());
  if (where == MPM_HOST && n > 0) HIP_OR_RETURN(h, hipStreamSynchronize(h->stream));
  h->N = n;
  h->has_E = (E != nullptr);
  h->mass = mass;
  h->vol0 = vol0;
  h->sim.mass = mass;
  h->sim.has_E = h->has_E ? 1 : 0;
  h->sim.p2g_stress = (float)((double)h->p.dt * (double)vol0 * 4.0 * (double)h->p.n_grid * (double)h->p.n_grid);
  h->sim.pic_force = (float)((double)h->p.dt * (double)vol0 * (double)h->p.n_grid);
  // Fixed-point units: a weight is 2^-22; momentum units are chosen so that
  // one particle at 1 m/s is 2^40 units (exact powers of two).
  h->sim.m_unit = std::ldexp(mass, -22);
  const int shift = 40 - std::ilogb(mass);
  h->sim.fx_p = std::ldexp(1.0, shift);
  h->sim.fx_p_inv = std::ldexp(1.0, -shift);
  h->sim.p_limit = (float)std::ldexp(1.0, 50 - shift);
  h->since_sort = 0;
  h->dirty = true;
  h->fresh_order = true;
  h->d.valid = false;
  drop_graphs(h);  // the recorded launches hold the old scene constants
  choose_item_size(h);
  h->err.clear();
  return MPM_OK;
}

// Free the device copy of a tool's velocity table once the stream no longer
// needs it.
int drop_tool_table(mpm_handle* h, size_t slot) {
  if (h->tool_tables[slot]) {
    HIP_OR_RETURN(h, hipStreamSynchronize(h->stream));
    HIP_OR_RETURN(h, hipFree(h->tool_tables[slot]));
    h->tool_tables[slot] = nullptr;
  }
  return MPM_OK;
}

int set_tool_impl(mpm_handle* h, int32_t scene, int32_t tool_id, const mpm_tool* t) {
  if (scene < 0 || scene >= h->n_scenes || tool_id < 0 || tool_id >= kMaxTools || !t)
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: bad scene or tool id");
  const size_t slot = (size_t)scene * kMaxTools + tool_id;
  HostTool& ht = h->tools[slot];
  if (t->type == MPM_TOOL_NONE) {
    ht.active = false;
    ht.vtab.clear();
    ht.vpre.clear();
    h->d.valid = false;
    h->tools_dirty = true;
    return drop_tool_table(h, slot);
  }
  if (t->type < MPM_TOOL_CAPSULE || t->type > MPM_TOOL_ARC)
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: bad type");
  bool fin = std::isfinite(t->mu) && std::isfinite(t->drag) && std::isfinite(t->margin);
  for (int a = 0; a < 3; ++a)
    fin = fin && std::isfinite(t->center[a]) && std::isfinite(t->size[a]) && std::isfinite(t->lin_vel[a]) &&
          std::isfinite(t->ang_vel[a]);
  double qn = 0.0;
  for (int a = 0; a < 4; ++a) {
    fin = fin && std::isfinite(t->quat[a]);
    qn += t->quat[a] * t->quat[a];
  }
  if (!fin || !(qn > 0.0) || t->mu < 0.0f || t->drag < 0.0f || t->drag > 1.0f)
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: value out of range");
  if (t->type == MPM_TOOL_CAPSULE && (!(t->size[0] >= 0.0) || !(t->size[1] > 0.0)))
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: capsule needs half_length >= 0, radius > 0");
  if (t->type == MPM_TOOL_BOX && (!(t->size[0] > 0.0) || !(t->size[1] > 0.0) || !(t->size[2] > 0.0)))
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: box needs positive half extents");
  if (t->type == MPM_TOOL_SLICER && (!(t->size[0] > 0.0) || !(t->size[1] > 0.0) || !(t->margin > 0.0f)))
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: slicer needs positive half width, half height and margin");
  if (t->type == MPM_TOOL_SEGMENT && (!(t->size[0] >= 0.0) || !(t->size[1] > 0.0)))
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: segment needs half_length >= 0, thickness > 0");
  if (t->type == MPM_TOOL_ARC && (!(t->size[0] > 0.0) || !(t->size[1] > 0.0) || !(t->size[1] <= M_PI) ||
                                  !(t->size[2] > 0.0)))
    return fail(h, MPM_EINVAL, "mpm_set_tool_sdf: arc needs radius > 0, 0 < half angle <= pi, thickness > 0");
  ht.t = *t;
  ht.set_at = h->substep;
  quat_to_R(t->quat, ht.R);
  ht.active = true;
  ht.vtab.clear();
  ht.vpre.clear();
  h->d.valid = false;
  h->tools_dirty = true;
  return drop_tool_table(h, slot);
}

int set_table_impl(mpm_handle* h, int32_t scene, int32_t tool_id, int64_t n_rows, const double* table) {
  if (scene < 0 || scene >= h->n_scenes || tool_id < 0 || tool_id >= kMaxTools || n_rows < 0 ||
      (n_rows > 0 && !table))
    return fail(h, MPM_EINVAL, "mpm_set_tool_velocity_table: bad argument");
  const size_t slot = (size_t)scene * kMaxTools + tool_id;
  HostTool& ht = h->tools[slot];
  if (!ht.active) return fail(h, MPM_EINVAL, "mpm_set_tool_velocity_table: no tool with this id");
  for (int64_t i = 0; i < 3 * n_rows; ++i)
    if (!std::isfinite(table[i])) return fail(h, MPM_EINVAL, "mpm_set_tool_velocity_table: non-finite entry");
  // Re-anchor at the current pose, then follow the table.
  double pose[3], vel[3];
  tool_kinematics(ht, h->substep, (double)h->p.dt, pose, vel);
  for (int a = 0; a < 3; ++a) ht.t.center[a] = pose[a];
  ht.set_at = h->substep;
  ht.vtab.assign(table, table + 3 * n_rows);
  ht.vpre.assign(3 * (n_rows + 1), 0.0);
  for (int64_t j = 0; j < n_rows; ++j)
    for (int a = 0; a < 3; ++a) ht.vpre[3 * (j + 1) + a] = ht.vpre[3 * j + a] + ht.vtab[3 * j + a];
  h->d.valid = false;
  h->tools_dirty = true;
  int rc = drop_tool_table(h, slot);
  if (rc != MPM_OK || n_rows == 0) return rc;
  double* dev = nullptr;
  const size_t nd = ht.vtab.size() + ht.vpre.size();
  ALLOC_OR_RETURN(h, hipMalloc((void**)&dev, sizeof(double) * nd));
  h->tool_tables[slot] = dev;
  HIP_OR_RETURN(h, hipMemcpy(dev, ht.vtab.data(), sizeof(double) * ht.vtab.size(), hipMemcpyHostToDevice));
  HIP_OR_RETURN(h, hipMemcpy(dev + ht.vtab.size(), ht.vpre.data(), sizeof(double) * ht.vpre.size(),
                             hipMemcpyHostToDevice));
  return MPM_OK;
}

// Device descriptors of every scene's tools (uploaded when a tool changed).
int upload_tools(mpm_handle* h) {
  if (!h->tools_dirty) return MPM_OK;
  std::vector<ToolDesc> desc((size_t)h->n_scenes * kMaxTools);
  for (size_t slot = 0; slot < desc.size(); ++slot) {
    const HostTool& ht = h->tools[slot];
    ToolDesc& d = desc[slot];
    std::memset(&d, 0, sizeof(d));
    d.k.type = ht.active ? ht.t.type : TOOL_NONE;
    if (!ht.active) continue;
    for (int a = 0; a < 3; ++a) {
      d.k.size[a] = (float)ht.t.size[a];
      d.k.av[a] = (float)ht.t.ang_vel[a];
      d.c0[a] = ht.t.center[a];
      d.lv[a] = ht.t.lin_vel[a];
    }
    for (int i = 0; i < 9; ++i) d.k.R[i] = (float)ht.R[i];
    d.k.mu = ht.t.mu;
    d.k.drag = ht.t.drag;
    d.k.margin = ht.t.margin;
    d.k.reach2 = reach2_of(ht.t);
    d.k.push = (ht.t.push_out != 0 &&
                (ht.t.type == TOOL_CAPSULE || ht.t.type == TOOL_BOX || ht.t.type == TOOL_PLANE)) ? 1 : 0;
    d.set_at = ht.set_at;
    d.rows = (long long)(ht.vtab.size() / 3);
    d.vtab = h->tool_tables[slot];
    d.vpre = h->tool_tables[slot] ? h->tool_tables[slot] + ht.vtab.size() : nullptr;
  }
  // A pageable source is staged before the call returns, so `desc` may go.
  HIP_OR_RETURN(h, hipMemcpyAsync(h->b.tools, desc.data(), sizeof(ToolDesc) * desc.size(), hipMemcpyHostToDevice,
                                  h->stream));
  h->tools_dirty = false;
  // The grid update scans the slots up to the highest one in use; the
  // transfer kernels check positions when some tool pushes particles out.
  int slots = 0, push = 0;
  for (size_t slot = 0; slot < desc.size(); ++slot) {
    if (h->tools[slot].active) slots = std::max(slots, (int)(slot % kMaxTools) + 1);
    if (desc[slot].k.push) push = 1;
  }
  if (slots != h->sim.tool_slots || push != h->sim.push_out) {
    h->sim.tool_slots = slots;
    h->sim.push_out = push;
    drop_graphs(h);  // the recorded launches hold the scene constants
  }
  return MPM_OK;
}

}  // namespace

int mpm_set_particles(mpm_handle* h, int64_t n, const float* x, const float* v, const float* C, const float* F,
                      const float* E, float mass, float vol0, int32_t where) {
  if (!h) return MPM_EINVAL;
  if (h->n_scenes != 1) return fail(h, MPM_EINVAL, "mpm_set_particles: several scenes, use mpm_set_batch_particles");
  if (n < 0) return fail(h, MPM_EINVAL, "mpm_set_particles: argument out of range");
  return set_particles_impl(h, &n, x, v, C, F, E, mass, vol0, where);
}

int mpm_set_batch_particles(mpm_handle* h, const int64_t* counts, const float* x, const float* v, const float* C,
                            const float* F, const float* E, float mass, float vol0, int32_t where) {
  if (!h) return MPM_EINVAL;
  if (!counts) return fail(h, MPM_EINVAL, "mpm_set_batch_particles: counts is NULL");
  return set_particles_impl(h, counts, x, v, C, F, E, mass, vol0, where);
}

int mpm_set_tool_sdf(mpm_handle* h, int32_t tool_id, const mpm_tool* t) {
  if (!h) return MPM_EINVAL;
  return set_tool_impl(h, 0, tool_id, t);
}

int mpm_set_scene_tool(mpm_handle* h, int32_t scene, int32_t tool_id, const mpm_tool* t) {
  if (!h) return MPM_EINVAL;
  return set_tool_impl(h, scene, tool_id, t);
}

int mpm_set_tool_velocity_table(mpm_handle* h, int32_t tool_id, int64_t n_rows, const double* table) {
  if (!h) return MPM_EINVAL;
  return set_table_impl(h, 0, tool_id, n_rows, table);
}

int mpm_set_scene_tool_velocity_table(mpm_handle* h, int32_t scene, int32_t tool_id, int64_t n_rows,
                                      const double* table) {
  if (!h) return MPM_EINVAL;
  return set_table_impl(h, scene, tool_id, n_rows, table);
}

namespace {

// Grid updates per substep: the PB-MPM iterations, else one.
int transfer_passes(const mpm_handle* h) { return h->sim.solver == SOLVER_PB ? h->pb_iterations : 1; }

// Whether a re-binning inside mpm_step sorts by the positions in memory
// (MPM_REBIN_IN_PLACE) rather than after a G2P pass (MPM_REBIN_ADVANCE).
bool rebin_in_place(const mpm_handle* h) {
  if (h->rebin_mode != MPM_REBIN_AUTO) return h->rebin_mode == MPM_REBIN_IN_PLACE;
  return h->sim.solver != SOLVER_PB && h->resort_interval >= 4;
}

// Adaptive re-binning keeps the host at most kDriftLag substeps ahead of the
// device: wait for the progress marks that end kDriftLag or more substeps
// before the current count (the device still has that many queued).
hipError_t drift_throttle(mpm_handle* h) {
  while (h->drift_n > 0 && h->drift_sub[h->drift_head] <= h->substep - kDriftLag) {
    const hipError_t e = hipEventSynchronize(h->drift_ev[h->drift_head]);
    if (e != hipSuccess) return e;
    h->drift_head = (h->drift_head + 1) % kDriftEvents;
    h->drift_n--;
  }
  return hipSuccess;
}

// A progress mark after a run of launches that ends at substep h->substep.
hipError_t drift_mark(mpm_handle* h) {
  if (h->drift_n == kDriftEvents) {  // ring full: retire the oldest
    const hipError_t e = hipEventSynchronize(h->drift_ev[h->drift_head]);
    if (e != hipSuccess) return e;
    h->drift_head = (h->drift_head + 1) % kDriftEvents;
    h->drift_n--;
  }
  const int slot = (h->drift_head + h->drift_n) % kDriftEvents;
  if (!h->drift_ev[slot]) {
    const hipError_t e = hipEventCreateWithFlags(&h->drift_ev[slot], hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  const hipError_t e = hipEventRecord(h->drift_ev[slot], h->stream);
  if (e != hipSuccess) return e;
  h->drift_sub[slot] = h->substep;
  h->drift_n++;
  return hipSuccess;
}

// Whether the particles on the global path since the last binning call for
// a re-binning before the interval ends: the grid update mirrors the
// device's fallback count into pinned host memory after every substep, and
// this reads the latest mirror without waiting on the stream (it lags the
// enqueued work by however far the device is behind).
bool drift_rebin(const mpm_handle* h) {
  if (h->rebin_drift <= 0 || h->dirty || h->since_sort < kMinDriftInterval) return false;
  const volatile unsigned long long* m = h->b.drift_host;
  const int64_t sub = (int64_t)__atomic_load_n(&m[0], __ATOMIC_ACQUIRE);
  const unsigned long long fb = m[1], fb0 = m[2];
  if (sub <= h->sort_substep || sub > h->substep || fb < fb0) return false;  // none since the binning
  const double per_substep = (double)(fb - fb0) / (double)(sub - h->sort_substep);
  return per_substep * 1e6 > (double)h->rebin_drift * (double)h->N;
}

// Grid update `it` of `passes` in a substep, of parity `parity`: PB-MPM
// leaves gravity out (it is added to the particles) and keeps the impulses of
// the last pass only; the clock's substep advances after the last pass.
void launch_grid_pass(mpm_handle* h, int it, int passes, int parity, hipStream_t st, KernelEvents ev = {}) {
  const bool last = it == passes - 1;
  launch_grid(h->b, h->sim, (int)h->n_blocks, parity, st, h->sim.solver != SOLVER_PB, last, last, ev);
}

// Record `chunk` plain substeps (fused transfer + grid update) as a graph
// for the current particle half, starting at grid-update parity `p0`.
int record_graph(mpm_handle* h, int p0) {
  if (!h->cap_stream) HIP_OR_RETURN(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  Buffers& b = h->b;
  hipGraph_t g = nullptr;
  HIP_OR_RETURN(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const int passes = transfer_passes(h);
  int parity = p0;
  for (int i = 0; i < h->graph_chunk; ++i) {
    launch_g2p2g(b, h->N, h->sim, h->transfer_wgs, parity, h->cap_stream, PB_FIRST);
    for (int it = 0; it < passes; ++it) {
      if (it > 0) launch_g2p2g(b, h->N, h->sim, h->transfer_wgs, parity, h->cap_stream, PB_ITER);
      launch_grid_pass(h, it, passes, parity, h->cap_stream);
      parity ^= 1;
    }
  }
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&h->graph[b.cur][p0], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph[b.cur][p0] = nullptr;
    return hip_fail(h, e, "hipGraphInstantiate");
  }
  return MPM_OK;
}

}  // namespace

int mpm_step(mpm_handle* h, int32_t n_substeps) {
  if (!h) return MPM_EINVAL;
  if (n_substeps < 0) return fail(h, MPM_EINVAL, "mpm_step: n_substeps < 0");
  if (n_substeps == 0) return MPM_OK;
  h->d.valid = false;
  if (h->N == 0) {
    HIP_OR_RETURN(h, select_device(h));
    launch_clear_impulses(h->b, h->sim, h->stream);
    h->substep += n_substeps;
    return MPM_OK;
  }
  HIP_OR_RETURN(h, select_device(h));
  Buffers& b = h->b;
  const int64_t N = h->N;
  const int wgs = h->transfer_wgs;
  int rc = upload_tools(h);
  if (rc != MPM_OK) return rc;
  launch_clear_impulses(b, h->sim, h->stream);
  launch_set_clock(b, (long long)h->substep, (int)(h->updates & 1), h->stream);
  const int passes = transfer_passes(h);
  const bool in_place = rebin_in_place(h);
  const bool adaptive = h->rebin_drift > 0;
  for (int k = 0; k < n_substeps;) {
    if (adaptive) HIP_OR_RETURN(h, drift_throttle(h));
    const bool rebin = h->dirty || h->since_sort >= h->resort_interval || drift_rebin(h);
    // Within a call the particle memory holds x and F as the next G2P reads
    // them (v and C live in registers between G2P and P2G). A re-binning in
    // place sorts by those positions, so every G2P stencil of the next fused
    // substep lies in its block's tile; otherwise a G2P pass first writes
    // the advanced state and the P2G below scatters from it. At the first
    // substep the memory holds the full state (v, C included).
    const bool advance = rebin && k > 0 && !in_place;
    const int parity = (int)(h->updates & 1);
    h->prof_now = h->prof && h->substep % h->prof_every == 0;
    if (advance) {
      KernelTimer kt(h, 3);
      launch_g2p(b, N, h->sim, wgs, parity, h->stream, kt.ev);
    }
    if (rebin) {
      ProfScope ps(h, 0);
      // Binning orders a block's particles by sub-cell class when the block
      // held few enough particles at the previous sort; for new particles a
      // sort of their keys alone gives those counts first.
      const int bits = h->key_bits + h->sim.unit_shift;  // bits of a work tile id or the sentinel
      if (h->fresh_order) launch_tile_counts(b, N, h->sim, bits, h->stream);
      h->fresh_order = false;
      launch_binning(b, N, h->sim, bits, k == 0 || advance, h->stream);
      h->dirty = false;
      h->since_sort = 0;
      h->sort_substep = h->substep;
      h->resorts++;
    }
    if (k == 0 || advance) {
      KernelTimer kt(h, 1);
      launch_p2g(b, N, h->sim, wgs, parity, h->stream, kt.ev);
    } else {
      // Plain substeps until the next re-binning or the end of the call:
      // whole chunks replay the recorded graph (not while timing kernels).
      const int64_t run = std::min<int64_t>(n_substeps - k, h->resort_interval - h->since_sort);
      if (!h->prof && h->graph_chunk > 0 && run >= h->graph_chunk) {
        if (!h->graph[b.cur][parity]) {
          rc = record_graph(h, parity);
          if (rc != MPM_OK) return rc;
        }
        HIP_OR_RETURN(h, hipGraphLaunch(h->graph[b.cur][parity], h->stream));
        k += h->graph_chunk;
        h->substep += h->graph_chunk;
        h->updates += (int64_t)h->graph_chunk * passes;
        h->since_sort += h->graph_chunk;
        if (adaptive) HIP_OR_RETURN(h, drift_mark(h));
        continue;
      }
      KernelTimer kt(h, 2);
      launch_g2p2g(b, N, h->sim, wgs, parity, h->stream, PB_FIRST, kt.ev);
    }
    for (int it = 0; it < passes; ++it) {
      const int pit = (parity + it) & 1;
      if (it > 0) {
        KernelTimer kt(h, 2);
        launch_g2p2g(b, N, h->sim, wgs, pit, h->stream, PB_ITER, kt.ev);
      }
      KernelTimer kt(h, 4);
      launch_grid_pass(h, it, passes, pit, h->stream, kt.ev);
    }
    h->updates += passes;
    h->substep++;
    h->since_sort++;
    ++k;
    if (adaptive && (h->substep % kDriftMarkEvery == 0 || k == n_substeps)) HIP_OR_RETURN(h, drift_mark(h));
  }
  {
    h->prof_now = h->prof;  // the closing G2P, once per call
    KernelTimer kt(h, 3);
    launch_g2p(b, N, h->sim, wgs, (int)(h->updates & 1), h->stream, kt.ev);
  }
  h->prof_now = false;
  HIP_OR_RETURN(h, hipGetLastError());
  return MPM_OK;
}

int mpm_set_solver(mpm_handle* h, int32_t solver, int32_t iterations, float beta) {
  if (!h) return MPM_EINVAL;
  if (solver != MPM_SOLVER_MLS && solver != MPM_SOLVER_PIC && solver != MPM_SOLVER_PB)
    return fail(h, MPM_EINVAL, "mpm_set_solver: unknown solver");
  if (solver == MPM_SOLVER_PB && (iterations < 1 || iterations > 1024 || !(beta >= 0.0f && beta <= 1.0f)))
    return fail(h, MPM_EINVAL, "mpm_set_solver: PB-MPM needs 1 <= iterations <= 1024 and 0 <= beta <= 1");
  static_assert(MPM_SOLVER_MLS == SOLVER_MLS && MPM_SOLVER_PIC == SOLVER_PIC && MPM_SOLVER_PB == SOLVER_PB,
                "solver codes");
  h->sim.solver = solver;
  if (solver == MPM_SOLVER_PB) {
    h->pb_iterations = iterations;
    h->sim.pb_beta = beta;
  }
  h->d.valid = false;
  drop_graphs(h);  // the recorded launches are those of the previous solver
  return MPM_OK;
}

int mpm_get_solver(const mpm_handle* h, int32_t* solver, int32_t* iterations, float* beta) {
  if (!h) return MPM_EINVAL;
  if (solver) *solver = h->sim.solver;
  if (iterations) *iterations = h->pb_iterations;
  if (beta) *beta = h->sim.pb_beta;
  return MPM_OK;
}

int mpm_get_launch_config(const mpm_handle* h, mpm_launch_config* out) {
  if (!h || !out) return MPM_EINVAL;
  out->resort_interval = h->resort_interval;
  out->transfer_wgs = h->transfer_wgs;
  out->graph_chunk = h->graph_chunk;
  out->rebin_mode = h->rebin_mode;
  out->tile = h->sim.tile;
  out->rebin_drift = h->rebin_drift;
  return MPM_OK;
}

int mpm_set_launch_config(mpm_handle* h, const mpm_launch_config* c) {
  if (!h) return MPM_EINVAL;
  if (!c || c->resort_interval < 1 || c->transfer_wgs < 8 || c->transfer_wgs % 8 != 0 || c->transfer_wgs > 65536 ||
      c->graph_chunk < 0 || c->graph_chunk > 256 || c->rebin_mode < MPM_REBIN_AUTO ||
      c->rebin_mode > MPM_REBIN_IN_PLACE || !(c->tile == 0 || c->tile == 4 || c->tile == 8) ||
      c->rebin_drift < 0 || c->rebin_drift > 1000000)
    return fail(h, MPM_EINVAL, "mpm_set_launch_config: value out of range");
  h->rebin_drift = c->rebin_drift;
  if (c->tile != 0) set_tile(h, c->tile);
  h->resort_interval = c->resort_interval;
  h->rebin_mode = c->rebin_mode;
  if (c->transfer_wgs != h->transfer_wgs || c->graph_chunk != h->graph_chunk) drop_graphs(h);
  h->transfer_wgs = c->transfer_wgs;
  h->graph_chunk = c->graph_chunk;
  choose_item_size(h);  // the work list is rebuilt before the next transfer if the item size changed
  return MPM_OK;
}

int mpm_autotune(mpm_handle* h, int32_t trial_substeps, mpm_launch_config* chosen) {
  if (!h) return MPM_EINVAL;
  if (trial_substeps < 1) return fail(h, MPM_EINVAL, "mpm_autotune: trial_substeps < 1");
  if (h->N == 0) return fail(h, MPM_EINVAL, "mpm_autotune: no particles");
  HIP_OR_RETURN(h, select_device(h));
  int rc = sync(h);
  if (rc != MPM_OK) return rc;
  Buffers& b = h->b;
  // Save what the trials change: the particles (and their order), the status
  // word and the clocks; restore them after every trial.
  const size_t part_bytes = sizeof(float) * kFields * (size_t)b.cap;
  float* save_part = nullptr;
  uint32_t* save_id = nullptr;
  Status* save_st = nullptr;
  ALLOC_OR_RETURN(h, hipMalloc((void**)&save_part, part_bytes));
  hipError_t e = hipMalloc((void**)&save_id, sizeof(uint32_t) * (size_t)b.cap);
  if (e == hipSuccess) e = hipMalloc((void**)&save_st, sizeof(Status));
  auto release = [&]() {
    (void)hipFree(save_part);
    (void)hipFree(save_id);
    (void)hipFree(save_st);
  };
  if (e != hipSuccess) {
    release();
    return alloc_fail(h, e, "mpm_autotune");
  }
  const int cur0 = b.cur;
  const int64_t substep0 = h->substep, since0 = h->since_sort, resorts0 = h->resorts;
  const bool dirty0 = h->dirty, prof0 = h->prof;
  const mpm_launch_config orig = {h->resort_interval, h->transfer_wgs, h->graph_chunk, h->rebin_mode, h->sim.tile,
                                   h->rebin_drift};
  e = hipMemcpyAsync(save_part, b.part[cur0], part_bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(save_id, b.id[cur0], sizeof(uint32_t) * b.cap, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(save_st, b.status, sizeof(Status), hipMemcpyDeviceToDevice, h->stream);
  auto restore = [&]() -> hipError_t {
    b.cur = cur0;
    hipError_t r = hipMemcpyAsync(b.part[cur0], save_part, part_bytes, hipMemcpyDeviceToDevice, h->stream);
    if (r == hipSuccess) r = hipMemcpyAsync(b.id[cur0], save_id, sizeof(uint32_t) * b.cap, hipMemcpyDeviceToDevice, h->stream);
    if (r == hipSuccess) r = hipMemcpyAsync(b.status, save_st, sizeof(Status), hipMemcpyDeviceToDevice, h->stream);
    // The tile bounds carry substep stamps that the trials ran past.
    for (int i = 0; i < 2 && r == hipSuccess; ++i) {
      hipLaunchKernelGGL(k_zero_u32, dim3(256), dim3(256), 0, h->stream, (uint32_t*)b.pbound[i],
                         (int64_t)(2 * ((int64_t)h->n_blocks << kMaxUnitShift)));
      r = hipGetLastError();
    }
    h->substep = substep0;
    h->since_sort = since0;
    h->resorts = resorts0;
    h->dirty = true;  // block lists are rebuilt for the restored order
    return r;
  };
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  h->prof = false;
  // Candidates: work tile edge, re-binning interval, persistent workgroups
  // per CU, graph replay on or off.
  // Fast-moving scenes leave their tiles within a few substeps (the global
  // path then takes the scatter), so the short intervals are candidates too.
  const int resorts[] = {1, 2, 4, 8, 16, 32, 64};
  const int n_resorts = (int)(sizeof(resorts) / sizeof(resorts[0]));
  const int per_cu[] = {1, 2, 3, 4};  // 8-cell tiles; four times as many 4-cell-tile workgroups
  const int tiles[] = {8, 4};
  const int chunks[] = {0, kDefaultGraphChunk};
  mpm_launch_config best = orig;
  float best_ms = 0.0f;
  bool have = false;
  // For each workgroup count and graph setting the re-binning intervals are
  // tried in increasing order; a candidate more than kSlow times slower than
  // the best so far ends that run of intervals (longer intervals only let more
  // particles drift out of their tiles), and a warm-up call that slow skips
  // the timed one. This bounds the cost of scenes whose particles move fast.
  constexpr float kSlow = 3.0f;
  auto timed_step = [&](float* ms) -> bool {
    e = hipEventRecord(ev0, h->stream);
    if (e != hipSuccess) return false;
    rc = mpm_step(h, trial_substeps);
    if (rc != MPM_OK) return false;
    e = hipEventRecord(ev1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev0, ev1);
    return e == hipSuccess;
  };
  // The configuration in use is the incumbent. Short trials on the current
  // state cannot resolve small differences (and the scene's later state may
  // rank them otherwise), so a candidate replaces it only if it is faster by
  // more than kKeep.
  constexpr float kKeep = 0.05f;
  auto same = [](const mpm_launch_config& a, const mpm_launch_config& c) {
    return a.resort_interval == c.resort_interval && a.transfer_wgs == c.transfer_wgs &&
           a.graph_chunk == c.graph_chunk && a.rebin_mode == c.rebin_mode && a.tile == c.tile &&
           a.rebin_drift == c.rebin_drift;
  };
  // warm-up (records graphs) and timed call of configuration c
  auto trial = [&](const mpm_launch_config& c, float* ms) -> bool {
    mpm_launch_config cc = c;
    rc = mpm_set_launch_config(h, &cc);
    if (rc != MPM_OK) return false;
    float warm = 0.0f;
    if ((e = restore()) != hipSuccess || !timed_step(&warm)) return false;
    if ((e = restore()) != hipSuccess) return false;
    return timed_step(ms);
  };
  float orig_ms = 0.0f;
  if (e == hipSuccess && trial(orig, &orig_ms)) {
    best_ms = orig_ms;
    have = true;
  }
  for (int ti = 0; ti < 2 && e == hipSuccess && rc == MPM_OK; ++ti)
  for (int wi = 0; wi < 4 && e == hipSuccess && rc == MPM_OK; ++wi)
    for (int ci = 0; ci < 2 && e == hipSuccess && rc == MPM_OK; ++ci)
      for (int ri = 0; ri < n_resorts && e == hipSuccess && rc == MPM_OK; ++ri) {
        const int wg_per_cu = per_cu[wi] * (tiles[ti] == 4 ? 4 : 1);
        mpm_launch_config c = {resorts[ri], (wg_per_cu * h->cus + 7) / 8 * 8, chunks[ci], MPM_REBIN_AUTO, tiles[ti],
                               h->rebin_drift};
        rc = mpm_set_launch_config(h, &c);
        if (rc != MPM_OK) break;
        e = restore();
        if (e != hipSuccess) break;
        // a warm-up call (records graphs), then the timed one
        float warm = 0.0f, ms = 0.0f;
        if (!timed_step(&warm)) break;
        if (have && warm > kSlow * best_ms) break;
        e = restore();
        if (e != hipSuccess) break;
        if (!timed_step(&ms)) break;
        if (!have || ms < best_ms) {
          best = c;
          best_ms = ms;
          have = true;
        } else if (ms > kSlow * best_ms) {
          break;
        }
      }
  // The fastest candidate with the re-binning mode that AUTO did not pick.
  if (have && e == hipSuccess && rc == MPM_OK) {
    mpm_launch_config c = best;
    rc = mpm_set_launch_config(h, &c);
    if (rc == MPM_OK) {
      c.rebin_mode = rebin_in_place(h) ? MPM_REBIN_ADVANCE : MPM_REBIN_IN_PLACE;
      rc = mpm_set_launch_config(h, &c);
    }
    float warm = 0.0f, ms = 0.0f;
    if (rc == MPM_OK && (e = restore()) == hipSuccess && timed_step(&warm) && warm <= kSlow * best_ms &&
        (e = restore()) == hipSuccess && timed_step(&ms) && ms < best_ms) {
      best = c;
      best_ms = ms;
    }
  }
  // The winner against the incumbent: each timed once more (the better of
  // two timings counts); a switch needs a gain above kKeep.
  if (have && e == hipSuccess && rc == MPM_OK && !same(best, orig)) {
    float again = 0.0f;
    if (trial(best, &again)) best_ms = std::min(best_ms, again);
    if (e == hipSuccess && rc == MPM_OK && trial(orig, &again)) orig_ms = std::min(orig_ms, again);
    if (e == hipSuccess && rc == MPM_OK && !(best_ms < (1.0f - kKeep) * orig_ms)) best = orig;
  }
  hipError_t e2 = restore();
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  // the trials' fallback counts and progress marks must not count later
  if (e == hipSuccess) std::memset(h->b.drift_host, 0, 4 * sizeof(unsigned long long));
  h->drift_n = 0;
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  release();
  h->prof = prof0;
  if (rc == MPM_OK && e == hipSuccess) rc = mpm_set_launch_config(h, have ? &best : &orig);
  else (void)mpm_set_launch_config(h, &orig);
  if (!dirty0) h->dirty = true;
  launch_clear_impulses(b, h->sim, h->stream);
  if (rc != MPM_OK) return rc;
  if (e != hipSuccess) return hip_fail(h, e, "mpm_autotune");
  if (chosen) *chosen = have ? best : orig;
  return MPM_OK;
}

int mpm_rollout_forward(mpm_handle* h, int32_t n_substeps, int32_t checkpoint_every, const float* theta) {
  if (!h) return MPM_EINVAL;
  if (n_substeps < 0 || checkpoint_every < 1)
    return fail(h, MPM_EINVAL, "mpm_rollout_forward: need n_substeps >= 0 and checkpoint_every >= 1");
  if (h->N == 0) return fail(h, MPM_EINVAL, "mpm_rollout_forward: no particles");
  if (h->n_scenes != 1) return fail(h, MPM_EINVAL, "mpm_rollout_forward: one scene only");
  if (h->sim.solver != SOLVER_MLS) return fail(h, MPM_EINVAL, "mpm_rollout_forward: needs the MLS-MPM solver");
  for (const HostTool& t : h->tools)
    if (t.active && t.t.push_out)
      return fail(h, MPM_EINVAL, "mpm_rollout_forward: particle push-out is not differentiated");
  HIP_OR_RETURN(h, select_device(h));
  DiffBufs& d = h->d;
  d.valid = false;
  const int64_t N = h->N;
  const int T = n_substeps, K = checkpoint_every;
  const int64_t SF = (int64_t)kStateFloats * N;
  const int64_t nn = (int64_t)h->p.n_grid * h->p.n_grid * h->p.n_grid;
  ALLOC_OR_RETURN(h, diff_alloc_base(h));
  ALLOC_OR_RETURN(h, ensure(&d.ckpt, &d.ckpt_slots, (int64_t)(T / K + 1), sizeof(float) * SF));
  // With a checkpoint at every substep the grids are kept too, and the
  // reverse pass recomputes nothing.
  d.grids_kept = (K == 1);
  if (d.grids_kept) ALLOC_OR_RETURN(h, ensure(&d.grids, &d.grid_slots, (int64_t)(T > 0 ? T : 1), sizeof(float4) * 2 * nn));
  if (theta)
    launch_exp(theta, d.E, N, h->stream);
  else
    launch_unpermute_E(h->b, N, h->sim, d.E, h->stream);
  auto slot = [&](int k) -> DState {
    if (k % K == 0) return dstate(d.ckpt + (int64_t)(k / K) * SF, N);
    return dstate(d.work + (int64_t)(k % 2) * SF, N);
  };
  DState s0 = slot(0);
  launch_unpermute(h->b, N, s0.x, s0.v, s0.C, s0.F, h->stream);
  launch_clear_impulses(h->b, h->sim, h->stream);
  // The orders are sorted in the binning scratch of the handle; mpm_step
  // re-bins afterwards.
  h->dirty = true;
  const int R = order_period(K);
  ALLOC_OR_RETURN(h, alloc_orders(h, (T + R - 1) / R));
  DiffOrder ord{};
  for (int k = 0; k < T; ++k) {
    if (k % R == 0) {
      HIP_OR_RETURN(h, rollout_order(h, slot(k).x, k / R));
      ord = order_slot(h, k / R);
    }
    float4* vel = d.grids_kept ? d.grids + (int64_t)k * 2 * nn : d.g.vel;
    float4* hat = d.grids_kept ? vel + nn : nullptr;
    launch_diff_substep(d.g, vel, hat, h->sim, tools_at(h, h->substep), N, slot(k), d.E, slot(k + 1), true,
                        h->b.status, ord, h->stream);
    h->substep++;
  }
  DState sT = slot(T);
  const bool keep_E = theta || h->has_E;
  launch_load_particles(h->b, N, sT.x, sT.v, sT.C, sT.F, keep_E ? d.E : nullptr, h->stream);
  HIP_OR_RETURN(h, hipGetLastError());
  if (theta) {
    h->has_E = true;
    h->sim.has_E = 1;
  }
  h->since_sort = 0;
  h->dirty = true;
  d.T = T, d.K = K, d.start = h->substep - T, d.N = N;
  d.valid = true;
  d.generation++;
  return MPM_OK;
}

int mpm_rollout_backward(mpm_handle* h, const float* xb, const float* vb, const float* Cb, const float* Fb,
                         float* theta_bar, double* vel_bar, float* xb0, float* vb0, float* Cb0, float* Fb0) {
  if (!h) return MPM_EINVAL;
  DiffBufs& d = h->d;
  if (!d.valid || d.N != h->N)
    return fail(h, MPM_EINVAL,
                "mpm_rollout_backward: no rollout to differentiate (particles, tools or the clock changed since)");
  if (!theta_bar) return fail(h, MPM_EINVAL, "mpm_rollout_backward: theta_bar is required");
  HIP_OR_RETURN(h, select_device(h));
  const int64_t N = d.N;
  const int T = d.T, K = d.K;
  const int64_t SF = (int64_t)kStateFloats * N;
  const int64_t nn = (int64_t)h->p.n_grid * h->p.n_grid * h->p.n_grid;
  const int nseg = d.grids_kept ? 0 : (T + K - 1) / K;
  if (!d.grids_kept) {
    // two sets of segment states and grids: the segment being differentiated
    // and the one being recomputed
    ALLOC_OR_RETURN(h, ensure(&d.seg, &d.seg_slots, 2 * (int64_t)K, sizeof(float) * SF));
    ALLOC_OR_RETURN(h, ensure(&d.grids, &d.grid_slots, 2 * (int64_t)K, sizeof(float4) * 2 * nn));
    if (!h->rec_stream) HIP_OR_RETURN(h, hipStreamCreateWithFlags(&h->rec_stream, hipStreamNonBlocking));
    while ((int)h->seg_ev.size() < 2 * nseg + 1) {
      hipEvent_t e;
      HIP_OR_RETURN(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      h->seg_ev.push_back(e);
    }
  }
  // per substep: kToolRedCopies partial sums, then (after them, for all
  // substeps) the totals
  const int64_t red_row = (int64_t)kMaxTools * 6;
  ALLOC_OR_RETURN(h, ensure(&d.tool_red, &d.tool_red_n, (int64_t)(T > 0 ? T : 1) * red_row * (kToolRedCopies + 1)));
  double* tool_tot = d.tool_red + (int64_t)T * red_row * kToolRedCopies;
  DState adj = dstate(d.adj, N);
  const float* seeds[4] = {xb, vb, Cb, Fb};
  float* dst[4] = {adj.x, adj.v, adj.C, adj.F};
  const int64_t len[4] = {3 * N, 3 * N, 9 * N, 9 * N};
  for (int f = 0; f < 4; ++f) {
    if (seeds[f])
      HIP_OR_RETURN(h, hipMemcpyAsync(dst[f], seeds[f], sizeof(float) * len[f], hipMemcpyDeviceToDevice, h->stream));
    else
      launch_fill_f32(dst[f], len[f], 0.0f, h->stream);
  }
  launch_fill_f32(theta_bar, N, 0.0f, h->stream);
  launch_fill_f64(d.tool_red, (int64_t)T * red_row * kToolRedCopies, 0.0, h->stream);
  auto grid_of = [&](int slot_index) -> float4* { return d.grids + (int64_t)slot_index * 2 * nn; };
  // The forward pass's particle orders: one per order_period(K) substeps.
  const int R = order_period(K);
  DiffOrder ord{};
  auto order_for = [&](int j) { ord = order_slot(h, j / R); };
  h->dirty = true;
  // The P2G reverse of substep j + 1 (its tail) runs inside the G2P reverse
  // of substep j; only the tail of substep 0 runs on its own.
  if (d.grids_kept) {
    for (int j = T - 1; j >= 0; --j) {
      float4* vel = grid_of(j);
      order_for(j);
      const DState next = dstate(d.ckpt + (int64_t)(j + 1) * SF, N);
      launch_adjoint_head(d.g, vel, vel + nn, h->sim, tools_at(h, d.start + j), N, dstate(d.ckpt + (int64_t)j * SF, N),
                          d.E, adj, theta_bar, d.tool_red + (int64_t)j * red_row * kToolRedCopies, ord,
                          j + 1 < T ? &next : nullptr, h->stream);
    }
  } else {
    // Segments from the last: each is recomputed from its checkpoint (the
    // states and grids of its substeps kept in slot set a & 1), then
    // differentiated. The recomputation of segment a - 1 runs on rec_stream
    // while segment a is differentiated on the main stream: they share no
    // buffer (the forward substep uses the P2G accumulator and the skip
    // flags, the adjoint the cotangent grids), and a slot set is refilled
    // only after the adjoint of the segment that used it is done.
    const DState none = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t start = h->seg_ev[2 * nseg];
    HIP_OR_RETURN(h, hipEventRecord(start, h->stream));  // seeds, fills and the forward pass are enqueued
    HIP_OR_RETURN(h, hipStreamWaitEvent(h->rec_stream, start, 0));
    for (int a = nseg - 1; a >= 0; --a) {
      const int s0 = a * K;
      const int n_in = (T - s0) < K ? (T - s0) : K;
      const int64_t set = (int64_t)(a & 1) * K;
      auto st = [&](int i) -> DState {
        return i == 0 ? dstate(d.ckpt + (int64_t)a * SF, N) : dstate(d.seg + (set + i) * SF, N);
      };
      hipEvent_t recomputed = h->seg_ev[2 * a], differentiated = h->seg_ev[2 * a + 1];
      if (a + 2 < nseg) HIP_OR_RETURN(h, hipStreamWaitEvent(h->rec_stream, h->seg_ev[2 * (a + 2) + 1], 0));
      // Recompute the segment from its checkpoint, keeping states and grids.
      // (A segment lies inside one order period.)
      const DiffOrder seg_ord = order_slot(h, s0 / R);
      for (int i = 0; i < n_in; ++i) {
        float4* vel = grid_of((int)set + i);
        launch_diff_substep(d.g, vel, vel + nn, h->sim, tools_at(h, d.start + s0 + i), N, st(i), d.E,
                            i + 1 < n_in ? st(i + 1) : none, false, h->b.status, seg_ord, h->rec_stream);
      }
      HIP_OR_RETURN(h, hipEventRecord(recomputed, h->rec_stream));
      HIP_OR_RETURN(h, hipStreamWaitEvent(h->stream, recomputed, 0));
      for (int i = n_in - 1; i >= 0; --i) {
        const int j = s0 + i;
        float4* vel = grid_of((int)set + i);
        // the state after substep j: the next segment's checkpoint at the end
        const DState next = i + 1 < n_in ? st(i + 1) : dstate(d.ckpt + (int64_t)(a + 1) * SF, N);
        launch_adjoint_head(d.g, vel, vel + nn, h->sim, tools_at(h, d.start + j), N, st(i), d.E, adj, theta_bar,
                            d.tool_red + (int64_t)j * red_row * kToolRedCopies, seg_ord,
                            j + 1 < T ? &next : nullptr, h->stream);
      }
      HIP_OR_RETURN(h, hipEventRecord(differentiated, h->stream));
    }
  }
  if (T > 0) launch_adjoint_tail(d.g, h->sim, N, dstate(d.ckpt, N), d.E, adj, theta_bar, h->stream);
  float* outs[4] = {xb0, vb0, Cb0, Fb0};
  for (int f = 0; f < 4; ++f)
    if (outs[f])
      HIP_OR_RETURN(h, hipMemcpyAsync(outs[f], dst[f], sizeof(float) * len[f], hipMemcpyDeviceToDevice, h->stream));
  HIP_OR_RETURN(h, hipGetLastError());
  if (vel_bar) {
    std::vector<double> red((size_t)T * kMaxTools * 6);
    launch_sum_tool_copies(d.tool_red, T, tool_tot, h->stream);
    if (T > 0)
      HIP_OR_RETURN(h, hipMemcpyAsync(red.data(), tool_tot, sizeof(double) * red.size(), hipMemcpyDeviceToHost,
                                      h->stream));
    HIP_OR_RETURN(h, hipStreamSynchronize(h->stream));
    // The centre in substep i is the centre at the rollout start plus dt
    // times the velocities of the substeps before i.
    const double dt = (double)h->p.dt;
    for (int q = 0; q < kMaxTools; ++q) {
      double suffix[3] = {0.0, 0.0, 0.0};
      for (int j = T - 1; j >= 0; --j) {
        const double* r = &red[((size_t)j * kMaxTools + q) * 6];
        for (int c = 0; c < 3; ++c) {
          vel_bar[((size_t)q * T + j) * 3 + c] = r[c] + dt * suffix[c];
          suffix[c] += r[3 + c];
        }
      }
    }
  }
  return MPM_OK;
}

int mpm_read_state(mpm_handle* h, float* x, float* v, float* C, float* F, int32_t where) {
  if (!h) return MPM_EINVAL;
  if (where != MPM_HOST && where != MPM_DEVICE) return fail(h, MPM_EINVAL, "mpm_read_state: bad where");
  HIP_OR_RETURN(h, select_device(h));
  const int64_t N = h->N;
  Buffers& b = h->b;
  if (N > 0 && (x || v || C || F)) {
    if (where == MPM_DEVICE) {
      launch_unpermute(b, N, x, v, C, F, h->stream);
    } else {
      float* stg = b.part[b.cur ^ 1];
      float* sx = stg;
      float* sv = stg + 3 * N;
      float* sC = stg + 6 * N;
      float* sF = stg + 15 * N;
      launch_unpermute(b, N, x ? sx : nullptr, v ? sv : nullptr, C ? sC : nullptr, F ? sF : nullptr,
                       h->stream);
      if (x) HIP_OR_RETURN(h, hipMemcpyAsync(x, sx, sizeof(float) * 3 * N, hipMemcpyDeviceToHost, h->stream));
      if (v) HIP_OR_RETURN(h, hipMemcpyAsync(v, sv, sizeof(float) * 3 * N, hipMemcpyDeviceToHost, h->stream));
      if (C) HIP_OR_RETURN(h, hipMemcpyAsync(C, sC, sizeof(float) * 9 * N, hipMemcpyDeviceToHost, h->stream));
      if (F) HIP_OR_RETURN(h, hipMemcpyAsync(F, sF, sizeof(float) * 9 * N, hipMemcpyDeviceToHost, h->stream));
    }
  }
  int rc = sync(h);
  if (rc != MPM_OK) return rc;
  return pending_status(h, nullptr);
}

int mpm_get_info(mpm_handle* h, mpm_info* info) {
  if (!h || !info) return fail(h, MPM_EINVAL, "mpm_get_info: NULL");
  HIP_OR_RETURN(h, select_device(h));
  int rc = sync(h);
  if (rc != MPM_OK) return rc;
  Status st;
  HIP_OR_RETURN(h, hipMemcpy(&st, h->b.status, sizeof(Status), hipMemcpyDeviceToHost));
  std::memset(info, 0, sizeof(*info));
  info->n_particles = h->N;
  info->substeps = h->substep;
  info->resorts = h->resorts;
  info->occupied_blocks = st.n_occ;
  info->active_blocks = st.n_act;
  info->active_nodes = 0;
  if (h->N > 0 && h->substep > 0 && !h->dirty) {
    launch_count_active_nodes(h->b, (int)((h->updates - 1) & 1), h->scratch_u64, h->stream);
    unsigned long long cnt = 0;
    HIP_OR_RETURN(h, hipMemcpyAsync(&cnt, h->scratch_u64, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_RETURN(h, hipStreamSynchronize(h->stream));
    info->active_nodes = (int64_t)cnt;
  }
  info->n_inverted = (int64_t)st.n_inverted;
  info->n_domain = (int64_t)st.n_domain;
  info->n_nonfinite = (int64_t)st.n_nonfinite;
  info->n_fallback = (int64_t)st.n_fallback;
  info->n_range = (int64_t)st.n_range;
  info->tile = h->sim.tile;
  info->resort_interval = h->resort_interval;
  info->accum_mode = h->p.accum_mode;
  int nt = 0;
  for (const HostTool& t : h->tools)
    if (t.active) nt++;
  info->n_tools = nt;
  info->rollouts = h->d.generation;
  return MPM_OK;
}

const char* mpm_last_error(const mpm_handle* h) {
  if (!h) {
    const char* m = noalloc_last_error();
    return m ? m : g_create_error.c_str();
  }
  return h->err.c_str();
}

int mpm_eval_stress(int64_t n, const float* F, const float* E, float nu, float* tau, int32_t where) {
  if (n < 0 || (n > 0 && (!F || !E || !tau)) || !(nu >= 0.0f && nu < 0.5f) ||
      (where != MPM_HOST && where != MPM_DEVICE))
    return MPM_EINVAL;
  if (n == 0) return MPM_OK;
  if (where == MPM_DEVICE) {
    launch_eval_stress(n, F, E, nu, tau, nullptr);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? MPM_OK : MPM_EHIP;
  }
  float *dF = nullptr, *dE = nullptr, *dT = nullptr;
  if (hipMalloc((void**)&dF, sizeof(float) * 9 * n) != hipSuccess ||
      hipMalloc((void**)&dE, sizeof(float) * n) != hipSuccess ||
      hipMalloc((void**)&dT, sizeof(float) * 9 * n) != hipSuccess) {
    (void)hipFree(dF);
    (void)hipFree(dE);
    (void)hipFree(dT);
    return MPM_ENOMEM;
  }
  hipError_t e = hipMemcpy(dF, F, sizeof(float) * 9 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dE, E, sizeof(float) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_eval_stress(n, dF, dE, nu, dT, nullptr);
    e = hipDeviceSynchronize();
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(tau, dT, sizeof(float) * 9 * n, hipMemcpyDeviceToHost);
  (void)hipFree(dF);
  (void)hipFree(dE);
  (void)hipFree(dT);
  return e == hipSuccess ? MPM_OK : MPM_EHIP;
}

int mpm_read_scene_tool_impulses(mpm_handle* h, int32_t scene, double* out) {
  if (!h || !out) return fail(h, MPM_EINVAL, "mpm_read_tool_impulses: NULL");
  if (scene < 0 || scene >= h->n_scenes) return fail(h, MPM_EINVAL, "mpm_read_tool_impulses: bad scene");
  HIP_OR_RETURN(h, select_device(h));
  launch_sum_impulses(h->b, h->sim, scene, h->imp_sum, h->stream);
  double sums[kImpulseRows * 3];
  HIP_OR_RETURN(h, hipMemcpyAsync(sums, h->imp_sum, sizeof(sums), hipMemcpyDeviceToHost, h->stream));
  int rc = sync(h);
  if (rc != MPM_OK) return rc;
  // Block sums hold the momentum given to the material; the tool receives the opposite.
  for (int i = 0; i < kImpulseRows * 3; ++i) out[i] = -sums[i];
  return MPM_OK;
}

int mpm_read_tool_impulses(mpm_handle* h, double* out) { return mpm_read_scene_tool_impulses(h, 0, out); }

int mpm_profile(mpm_handle* h, int32_t enable) {
  if (!h) return MPM_EINVAL;
  if (enable < 0) return fail(h, MPM_EINVAL, "mpm_profile: enable < 0");
  if (enable) {
    HIP_OR_RETURN(h, select_device(h));
    int rc = sync(h);
    if (rc != MPM_OK) return rc;
    prof_collect(h);
    for (int k = 0; k < MPM_KERNEL_KINDS; ++k) {
      h->prof_ms[k] = 0.0;
      h->prof_n[k] = 0;
    }
  }
  h->prof = enable != 0;
  h->prof_every = enable > 1 ? enable : 1;
  return MPM_OK;
}

int mpm_profile_read(mpm_handle* h, mpm_kernel_times* out) {
  if (!h || !out) return fail(h, MPM_EINVAL, "mpm_profile_read: NULL");
  HIP_OR_RETURN(h, select_device(h));
  int rc = sync(h);
  if (rc != MPM_OK) return rc;
  prof_collect(h);
  for (int k = 0; k < MPM_KERNEL_KINDS; ++k) {
    out->total_ms[k] = h->prof_ms[k];
    out->launches[k] = h->prof_n[k];
  }
  return MPM_OK;
}

}  // extern "C"
