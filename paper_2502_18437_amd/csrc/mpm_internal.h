// Internal declarations shared by the translation units of the library:
// kernel-argument structs, the device status word and host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace mpm {

// Grid blocks are kTile^3 nodes, stored contiguously (x fastest inside a
// block, blocks x fastest); the grid update, the active and overflow lists
// and the impulse sums work per block. The transfers work per work tile: a
// cube of TileShape<T>::kEdge cells (T = 8: one block; T = 4: one of its
// eight sub-blocks), whose particles share a tile of (T + 2)^3 nodes in LDS
// (the 3-node stencils of its cells). Particles that drift out of their tile
// since binning take the global-memory path.
constexpr int kTile = 8;
constexpr int kTileLog2 = 3;
// Low bits of a binning key below the work tile id: the particle's sub-cell
// class (a half of the base cell per axis, 3 bits) and the base cell's z
// layer in the tile (3 bits), in either order. Handles keep n_blocks below
// 2^22 (work tile ids below 2^25), so a key stays below 2^31.
constexpr int kClassBits = 6;
// The differentiable rollout's scatters work on 8-cell tiles: 10^3 nodes.
constexpr int kSpan = kTile + 2;                   // 10
constexpr int kSpanNodes = kSpan * kSpan * kSpan;  // 1000
constexpr int kBlockNodes = kTile * kTile * kTile;  // 512

// Shape of a transfer work tile of edge T (4 or 8 cells): its LDS span, the
// workgroup size of the transfer kernels, the shift from block ids to work
// tile ids (a 4-cell tile is block * 8 + sub-block, sub-block = sx + 2 sy +
// 4 sz), and the particle count above which a tile counts as dense (8 per
// cell; see kDenseFlag).
template <int T>
struct TileShape {
  static_assert(T == 4 || T == 8, "work tiles are 4 or 8 cells wide");
  static constexpr int kEdge = T;
  static constexpr int kLog2 = T == 8 ? 3 : 2;
  static constexpr int kSpan = T + 2;
  static constexpr int kSpanNodes = kSpan * kSpan * kSpan;
  static constexpr int kWG = T == 8 ? 512 : 128;
  static constexpr int kUnitShift = T == 8 ? 0 : 3;
  static constexpr unsigned kDense = 8u * T * T * T;
};
// Sub-blocks per block for the finest work tile: the per-tile tables
// (ranges, flags, work items) are sized for it.
constexpr int kMaxUnitShift = 3;
constexpr int kMaxTools = 8;
constexpr int kImpulseRows = kMaxTools + 1;  // tools, then the walls
constexpr int kGridSlots = 8192;             // largest grid-update launch
constexpr int kFields = 25;  // x3 v3 C9 F9 E1, SoA
// A transfer work item is one work tile's particles or, for a tile holding
// more than SimK::item_particles, a run of that many of them: dense tiles
// are shared by several workgroups (each with its own LDS tile) instead of
// serialising on one. The run length is a power of two in [kItemMin / k,
// kItemMax / k] (k = 1 for 8-cell tiles, 4 for 4-cell tiles, whose
// workgroups are a quarter the size) chosen from the particle and workgroup
// counts.
constexpr int kItemMin = 512;
constexpr int kItemMax = 2048;
// Work items of a tile holding more than TileShape<T>::kDense particles (8
// per cell on average) carry kDenseFlag in their tile id: their particles
// are dealt to the lanes of a wave kWG / 64 apart, so that one wave's LDS
// atomics do not pile onto the same nodes.
constexpr unsigned kDenseFlag = 0x80000000u;
// The differentiable rollout's scatters take runs of kItemRollout particles
// (its scenes are small, so shorter runs keep every workgroup busy).
constexpr int kItemRollout = 256;
// The smallest work item of any kind (sizes the work list).
constexpr int kItemMinAny = 128;
static_assert(kItemMin / 4 >= kItemMinAny && kItemRollout >= kItemMinAny, "work list capacity");

// Field offsets in the particle SoA (each field is `cap` floats).
enum Field { FX = 0, FV = 3, FC = 6, FF = 15, FE = 24 };

enum ToolType { TOOL_NONE = 0, TOOL_CAPSULE = 1, TOOL_BOX = 2, TOOL_PLANE = 3, TOOL_SLICER = 4, TOOL_SEGMENT = 5, TOOL_ARC = 6 };

// One tool as the grid kernel sees it (FP32, pose of the current substep).
struct ToolK {
  int type;
  float c[3];      // centre at the start of the substep
  float R[9];      // body-to-world rotation, row-major
  float size[3];
  float lv[3];
  float av[3];
  float mu, drag, margin;
  float reach2;    // squared radius around c outside which no node is in contact; < 0: unbounded
  int push;        // particle push-out after each substep (solid tools only)
};

struct ToolSetK {
  int n;           // tools 0..n-1 are scanned; NONE entries are skipped
  ToolK t[kMaxTools];
};

// One tool of one scene as the device keeps it: the constant part of ToolK
// plus what its pose at any substep is computed from (FP64 kinematics, the
// same formula as the host's).
struct ToolDesc {
  ToolK k;               // type, R, size, av, mu, drag, margin, reach2 (c and lv are per substep)
  double c0[3];          // centre at set_at
  double lv[3];          // constant linear velocity
  long long set_at;      // substep counter when set (or re-anchored)
  long long rows;        // velocity-table rows (0: none)
  const double* vtab;    // rows x 3 (device)
  const double* vpre;    // (rows + 1) x 3 prefix sums (device)
};

// Scene constants for the transfer kernels.
//
// P2G accumulates in integers (LDS float atomics are slow on gfx950, and
// integer sums are exact and order independent): the mass channel as the sum
// of the B-spline weights in units of 2^-22 (u32), the momentum channels as
// int64 in units of 2^-fx_shift kg m/s, where fx_shift is chosen per scene
// so that one particle moving at 1 m/s is about 2^40 units. The conversion
// of a value to int64 is the round-to-nearest of an FP64 sum with 1.5 * 2^52,
// exact for magnitudes below 2^51 units.
struct SimK {
  int n;           // nodes per axis (of every scene)
  int nb;          // blocks per axis
  int n_scenes;    // scenes of the batch; scene s owns blocks [s nb^3, (s+1) nb^3) and nodes [s n^3, (s+1) n^3)
  unsigned nb3;    // blocks per scene
  int n3;          // nodes per scene
  float dx, inv_dx, dt;
  float mass;      // per particle
  float p2g_stress;  // dt * vol0 * 4 / dx^2
  float c_mu, c_la;  // mu = c_mu E, lambda = c_la E
  float E_default;
  int has_E;         // per-particle E stored in field FE
  int band;          // wall band
  float g[3];
  int fixed;         // global accumulator: 0 FP32, 1 integer (bit-reproducible)
  float m_unit;      // kg per weight unit: mass * 2^-22
  double fx_p;       // 2^fx_shift (momentum units per kg m/s)
  double fx_p_inv;   // 2^-fx_shift
  float p_limit;     // largest |contribution| (kg m/s) kept in range
  int solver;        // Solver: which transfer scheme and constitutive model the kernels run
  float pic_force;   // standard MPM: dt * vol0 / dx (internal force per unit of tau grad N dx)
  float pb_beta;     // PB-MPM: rotation weight of the co-rotational constraint
  int tool_slots;    // 1 + the highest tool slot in use in any scene (0: no tools)
  int push_out;      // some tool pushes particles out: the transfer kernels check positions
  unsigned item_particles;  // particles per transfer work item (at most)
  int tile;          // transfer work tile edge in cells: 8 (a block) or 4 (a sub-block)
  int unit_shift;    // work tile ids = block ids << unit_shift (3 for 4-cell tiles, else 0)
};

// Solvers of Sec. III: MLS-MPM (APIC transfers, fixed-corotated stress in the
// affine momentum), standard MPM (PIC transfers, Neo-Hookean stress as a grid
// force) and PB-MPM (iterated APIC transfers with a co-rotational constraint
// projection of C, no stress).
enum Solver { SOLVER_MLS = 0, SOLVER_PIC = 1, SOLVER_PB = 2 };

// Which transfer pass a PB-MPM launch is: the first of a step (finishes the
// previous step's F and x update, adds gravity) or a later iteration.
enum PBPass { PB_FIRST = 0, PB_ITER = 1 };

// Device status word (one per handle).
// XCDs of the chip. Workgroups of a launch are dealt round-robin to them, so
// workgroup w runs on XCD w % kXcds, each with its own L2.
constexpr int kXcds = 8;

struct Status {
  unsigned long long n_inverted;
  unsigned long long n_domain;
  unsigned long long n_nonfinite;
  unsigned long long n_fallback;
  unsigned long long n_range;      // P2G contributions outside the fixed-point range
  unsigned int n_occ;               // occupied work tiles (this binning)
  unsigned int n_work;              // transfer work items (this binning)
  unsigned int n_act;               // active blocks (this binning)
  unsigned int ovf_count[2];        // overflow blocks claimed, per parity
  unsigned long long fb_at_sort;    // n_fallback when the last binning ended
  // Work items claimed beyond the first one per workgroup, and workgroups
  // done, per XCD, in the persistent transfer kernels. Zero between launches:
  // the last workgroup of an XCD to finish puts both back to zero.
  unsigned int claim[kXcds];
  unsigned int claim_done[kXcds];
};

// Substep clock on the device, one entry per parity of the grid update
// (grid updates alternate the parity, which also picks the overflow list):
// the transfer and grid kernels of parity p read the substep (tool poses)
// from entry p rather than from their arguments, so that a run of substeps
// can be recorded once and replayed. The grid update of parity p writes entry
// p ^ 1 for the kernels after it: the same substep, or the next one after the
// last grid update of a substep (PB-MPM runs several per substep).
struct Clock {
  long long substep;
};

// Device buffers of one handle.
struct Buffers {
  float* part[2] = {nullptr, nullptr};      // particle SoA ping-pong, kFields * cap
  uint32_t* id[2] = {nullptr, nullptr};     // original particle index
  int cur = 0;                              // which ping-pong half is live
  int64_t cap = 0;
  uint32_t* keys[2] = {nullptr, nullptr};   // sort keys ping-pong
  uint32_t* vals[2] = {nullptr, nullptr};   // sort values ping-pong
  uint32_t* hist = nullptr;                 // radix histograms
  uint32_t* scan_tmp = nullptr;             // scan partials
  uint32_t* blk_begin = nullptr;            // per work tile [begin, end) (n_blocks << kMaxUnitShift entries)
  uint32_t* blk_end = nullptr;
  uint32_t* flags = nullptr;                // per work tile scratch for compaction
  uint32_t* occ_list = nullptr;             // occupied work tiles
  uint2* work = nullptr;                    // transfer work items {work tile, first particle}
  uint2* work_tmp = nullptr;                // the items as emitted, before ordering by size
  uint32_t* act_list = nullptr;             // active (dilated) blocks
  uint32_t* mark = nullptr;                 // per block: 0 idle, 1 active, 2 overflow
  // Per work tile, one per grid-update parity: the largest P2G contribution
  // bound of the tile's particles in the substep of that parity, as
  // (substep << 32) | FP32 bits, merged with atomicMax (FP32 accumulation,
  // MLS-MPM only; sets the scale of the packed LDS sums of the next substep).
  unsigned long long* pbound[2] = {nullptr, nullptr};
  uint32_t* node_cnt = nullptr;             // per block: nodes with mass, last grid update
  float* imp_blocks = nullptr;              // per grid block: impulse sums (kImpulseRows x 3)
  uint32_t* scene_off = nullptr;            // n_scenes + 1 particle offsets (original order)
  ToolDesc* tools = nullptr;                // n_scenes x kMaxTools
  uint32_t* ovf_list[2] = {nullptr, nullptr};
  void* acc_m = nullptr;                    // grid accumulator, mass channel (float or u32)
  void* acc_p[3] = {nullptr, nullptr, nullptr};  // momentum channels (float or int64)
  float4* vel = nullptr;                    // grid velocity
  Status* status = nullptr;
  Clock* clock = nullptr;                   // two entries, by parity
  // Pinned host words the grid update writes after a substep's last pass:
  // {substep, n_fallback, fb_at_sort}, so that the host can see how many
  // particles take the global path since the last binning without waiting
  // on the stream (adaptive re-binning).
  unsigned long long* drift_host = nullptr;
};

// ---------------------------------------------------------------- launchers
// Binning pipeline: keys from positions (block, then sub-cell class), radix
// sort, permutation, block ranges, occupied and active block lists. Resets
// the overflow lists. key_bits: bits of a block id or the sentinel. with_vc:
// also permute v and C (false between fused substeps, where only x, F, E are
// held in memory).
void launch_binning(Buffers& b, int64_t N, const SimK& s, int key_bits, bool with_vc, hipStream_t st);
// The tile counts that launch_binning's ordering rule reads, for particles
// without a previous sort (blk_begin / blk_end; nothing else changes).
void launch_tile_counts(Buffers& b, int64_t N, const SimK& s, int key_bits, hipStream_t st);

// Optional HIP events that a launcher records around its one kernel as part
// of the kernel's dispatch (hipExtLaunchKernel), for per-kernel timing
// without marker packets of their own; both null: a plain launch.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

template <class F, class... Args>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, hipStream_t st, KernelEvents ev, Args... args) {
  if (ev.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ev.start, ev.stop, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// Transfers before the grid update of parity `parity` (its overflow list
// takes drifted particles; push-out reads its clock entry). The solver is
// s.solver; `pass` selects the PB-MPM pass (PBPass) and is ignored by the
// other solvers.
void launch_p2g(Buffers& b, int64_t N, const SimK& s, int grid_wgs, int parity, hipStream_t st,
                KernelEvents ev = {});
void launch_g2p2g(Buffers& b, int64_t N, const SimK& s, int grid_wgs, int parity, hipStream_t st,
                  int pass = PB_FIRST, KernelEvents ev = {});
void launch_g2p(Buffers& b, int64_t N, const SimK& s, int grid_wgs, int parity, hipStream_t st,
                KernelEvents ev = {});

// Grid update of parity `parity` over active blocks and that parity's
// overflow blocks, with each scene's tools at their pose of the clock
// entry's substep; it sets the other parity's clock entry to the same
// substep or, when `last`, the next. `gravity` adds dt g to the node
// velocities; `record` adds the tools' and walls' momentum changes to the
// impulse sums.
void launch_grid(Buffers& b, const SimK& s, int max_act, int parity, hipStream_t st, bool gravity = true,
                 bool record = true, bool last = true, KernelEvents ev = {});
// The grid update after a substep's last pass also mirrors {substep,
// n_fallback, fb_at_sort} into Buffers::drift_host.
// Set the clock entry of `parity` to `substep`.
void launch_set_clock(Buffers& b, long long substep, int parity, hipStream_t st);

// Spatial order of a one-scene particle set held as an AoS x (N x 3) in the
// caller's order, for the rollout's tiled scatters. Sorts the particles by the
// grid block of their base cell (particles whose stencil leaves the grid or
// whose x is not finite last) in the handle's binning scratch, then writes the
// sorted caller indices to order (N entries), the block ranges to begin / end
// (nb3 entries each), the work items to work (runs of at most `item`
// particles of one block; at most nb3 + N / item + 1 of them), info[0] = the
// number of items and info[1] = the first sorted position of the particles
// left out. Every output is caller-owned device memory. Returns the error of
// the final copy (kernel launch errors show in hipGetLastError).
hipError_t launch_order(Buffers& b, int64_t N, const SimK& s, const float* x, int key_bits, uint32_t item,
                        uint32_t* order, uint32_t* begin, uint32_t* end, uint2* work, uint32_t* info,
                        hipStream_t st);

// Nodes with mass in the last grid update (sum of node_cnt over the active
// and overflow blocks of `parity`), written to *out (device memory).
void launch_count_active_nodes(Buffers& b, int parity, unsigned long long* out, hipStream_t st);

// Clear the per-block impulse sums; sum those of one scene into
// out[kImpulseRows * 3] (device).
void launch_clear_impulses(Buffers& b, const SimK& s, hipStream_t st);
void launch_sum_impulses(Buffers& b, const SimK& s, int scene, double* out, hipStream_t st);

// Stress evaluation (diagnostic entry point).
void launch_eval_stress(int64_t n, const float* F, const float* E, float nu, float* tau,
                        hipStream_t st);
// Message of the last failed mpm_eval_stress_noalloc call on this thread
// (nullptr if none since the last clear), and its reset.
const char* noalloc_last_error();
void noalloc_clear_error();

// Gather particles back into the caller's order (AoS outputs).
void launch_unpermute(const Buffers& b, int64_t N, float* x, float* v, float* C, float* F,
                      hipStream_t st);
// Scatter caller AoS inputs into the SoA (identity order, id = index).
void launch_load_particles(Buffers& b, int64_t N, const float* x, const float* v, const float* C,
                           const float* F, const float* E, hipStream_t st);

}  // namespace mpm
