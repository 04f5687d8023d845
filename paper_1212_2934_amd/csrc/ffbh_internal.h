// Internal declarations of libffbh (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <functional>
#include <type_traits>

#include "../../include/ffbh.h"

namespace ffbh {

constexpr int kBits = 21;                       // quantisation bits per axis
constexpr uint32_t kQMax = (1u << kBits) - 1u;  // largest quantised coordinate
constexpr int kMaxLevel = 21;                   // deepest cell level
constexpr int kWave = 64;                       // CDNA wavefront width
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixPasses = 8;                 // 8 x 8 bits cover the 63-bit codes
constexpr int kTieBits = 32;                    // low code bits the tiled sort leaves to k_fix_ties
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                  // most keys per thread per tile
constexpr int kMinTpw = 16;                     // fewest targets an adjoint wave owns
constexpr int kStackMax = 64;                   // one traversal stack entry per lane of a wave
// Largest theta^2 for which the acceptance test alone rejects every cell holding the target: target and
// centre lie in the cell's cube of side s, so d^2 <= 3 s^2, and theta^2 d^2 < s^2 holds with a margin of
// at least 10 %, far above rounding.  Up to it the traversals skip the explicit test for the target.
constexpr double kSelfRejectTheta2 = 0.3;

// Form of the acceptance test s^2 < theta^2 d^2 that a handle's traversals evaluate.
//   kMacInside: as written, plus the explicit test for cells holding the target (theta^2 above
//     kSelfRejectTheta2);
//   kMacPlain: as written; the test itself rejects the cells holding the target;
//   kMacScaled: theta^2 a power of two up to kSelfRejectTheta2 (theta = 1/2, 1/4, ...): the node records
//     hold s^2 / theta^2, which is exact, and the test is s2 < d^2.  Multiplying by a power of two is exact
//     (d^2 is never near the FP64 underflow threshold), so the decision is the same, with one FP64
//     multiplication fewer per node visit.
enum MacForm { kMacInside = 0, kMacPlain = 1, kMacScaled = 2 };
inline int mac_form(double theta2)
{
    if (theta2 > kSelfRejectTheta2) return kMacInside;
    int e = 0;
    return theta2 > 0.0 && std::frexp(theta2, &e) == 0.5 ? kMacScaled : kMacPlain;
}
// Factor of the squared cell sides in the node records (bbox slot 5 of each system).
inline double node_s2_scale(double theta2) { return mac_form(theta2) == kMacScaled ? 1.0 / theta2 : 1.0; }
constexpr int kHilbertBits = 8;                 // bits per axis of the Hilbert keys that group targets
constexpr int64_t kTargetOrderMin = 2049;       // systems from this size group targets in Hilbert order
constexpr int64_t kForkMinParticles = 1 << 14;  // fewer particles over the batch stay on one stream

// Node record read by the traversal: one 64-byte line, fetched with a single scalar load.
struct alignas(64) NodeRec {
    double cx, cy, cz;  // pseudo-particle position (geometric centre of the members)
    double s2;          // squared side of the cell's cube
    float mx, my, mz;   // moment sum rounded to FP32 (mixed-precision traversal)
    int32_t first;      // first member, global sorted position
    int32_t count;      // number of members
    int32_t child;      // first child node (children contiguous, octant order); -1 for a leaf
    int32_t nchild;     // 0 for a leaf
    int32_t parent;     // -1 for a root
};
static_assert(sizeof(NodeRec) == 64, "node record must be one 64-byte line");

// Device workspace, carved from the caller's buffer.  All arrays are global over the B systems.
struct Workspace {
    uint32_t *status;        // [0] flags, [1] scan total, [2] node count, [12] calls in flight
    double *bbox;            // B x 8: lo xyz, side, quantisation scale, node s^2 factor, (pad)
    double *bbox_part;       // B x kBboxBlocks x 6 partial min/max
    uint64_t *keys[2];       // N_tot sort keys (ping-pong)
    uint32_t *vals[2];       // N_tot sort values: global original index (ping-pong)
    uint32_t *hist;          // radix histograms (B x 256 x tiles_per_system)
    uint32_t *scan_tmp;      // per-tile partial sums of the device-wide scan
    uint32_t *perm;          // sorted position -> global original index (alias of the final vals)
    uint64_t *hkeys;         // N_tot Hilbert keys of the sorted particles (target-order sort)
    uint32_t *tgt_order;     // N_tot: the traversal's targets of each system in Hilbert order (sorted positions)
    uint32_t *hscan_tmp;     // per-tile partial sums of the target-order sort's scan
    uint64_t *codes;         // sorted codes (alias of the final keys)
    double *spos;            // 3 x N_tot sorted positions (SoA: x block, y block, z block)
    double *smom;            // 3 x N_tot sorted moments FP64
    void *src64;             // N_tot sorted source records (position, moment FP64), 48 bytes each (FP64)
    void *src32;             // the same buffer as records of position FP64, moment FP32 (FP32-mixed)
    // binary radix tree (per system: n-1 internal nodes, n leaves)
    int32_t *bin_left;       // internal node -> left child (>= 0 internal, < 0: leaf ~idx)
    int32_t *bin_right;
    int32_t *bin_first;      // range of an internal node (segment-local sorted positions)
    int32_t *bin_last;
    int32_t *bin_delta;      // common prefix length in bits (63 + x for equal codes)
    int32_t *bin_parent;     // internal node -> parent internal node (-1 root)
    int32_t *leaf_parent;    // sorted particle -> parent internal node (-1 if n == 1)
    int32_t *bin_nchild;     // octree children of an internal node (0 if not an in-tree internal)
    uint32_t *bin_scan;      // exclusive scan of bin_nchild
    // octree
    int32_t *bin_octid;      // internal node -> octree node id (in-tree internal nodes only)
    NodeRec *nodes;          // max_nodes
    int32_t *node_level;     // max_nodes: cell level (side = side_root / 2^level)
    double *node_m64;        // 4 x max_nodes: moment sum FP64 (x, y, z, pad) per node
    uint2 *cells;            // short-range grid: member range [start, end) of each cell (B x cell_T)
    double *part_buf;        // (parts, 6, ntot) partial sums of split adjoint walks
    uint32_t *wave_cost;     // per adjoint wave item: work of the last launch (orders the next one)
    uint32_t *wave_order;    // item order of the next persistent launch
    uint32_t *sched_ctr;     // [0]: work counter of the persistent launch
    uint32_t *field_cost;    // per forward-walk wave item: work of the last walk (orders the next one)
    uint32_t *field_order;   // wave -> item order of the next forward walk
    uint32_t *field_ctr;     // counters the ordering kernel resets (unused by the forward walk)
    double *node_q64;        // max_nodes x 16: first moment D (row-major 3x3, then pad) per node, FP64
    float *node_q32;         // max_nodes x 16: the same rounded to FP32 (mixed-precision traversal)
    double *node_adjq;       // max_nodes x 8: dL/dD of each node, symmetric (xx, yy, zz, xy, xz, yz)
    double *ones;            // B: constant 1.0 (dL/dE for the MD force)
    uint32_t *lvl;           // 128: per-bucket node counts [0,23), bucket starts [32,56), cursors [64,87)
    int32_t *lvl_nodes;      // max_nodes: node ids bucketed (internal nodes by level 0..21, leaves in 22)
    int32_t *leaf_of;        // N_tot: sorted particle -> its leaf
    // traversal outputs and adjoint accumulators
    double *e_part;          // per wave energy partials
    double *node_adj;        // 8 x max_nodes: A (3), B (3) per node, padded; also upward-pass sums
    double *g_gather;        // 3 x N_tot: per-target gathered position adjoint (sorted order)
    double *g_rm;            // N_tot x 8: scattered position (3) and moment (3) adjoint per sorted particle
    double *hbar;            // 3 x N_tot: upstream field gradient (sorted order)
    double *Hs;              // 3 x N_tot: field in sorted order
    double *H_scratch;       // B x 3 x n: field in caller order when the caller does not want it
    double *md_force;        // 3 x N_tot: short-range forces (caller order) for the MD step
    double *md_grad_r;       // B x 3 x n
    double *md_grad_m;       // B x 3 x n
};

constexpr int kBboxBlocks = 512;  // partial bounding boxes per system (two workgroups per CU)

struct Layout {
    int64_t n, B, ntot, max_nodes, tiles, num_waves, hist_len, bin_int;
    int sort_items;         // keys per thread per radix-sort tile (1..kSortItems)
    int adj_parts;          // parts of a split adjoint walk that the workspace holds (0: none)
    int expansion;          // 2: first moments are kept (order-2 cells); else 1
    int cell_lcap;       // finest level of the short-range cell grid
    int64_t cell_T;      // grid entries per system, 2^(3 cell_lcap)
    size_t bytes;
};

Layout plan_layout(const bh_params &p);
void carve(const Layout &L, void *base, Workspace &w);

// Host-side handle.
struct Handle {
    bh_params p;
    Layout L;
    Workspace w;
    int device;
    int built;           // a bh_build has been enqueued
    int owned;           // 1: made by bh_create (host memory, side stream and events are the library's);
                         // 0: made by bh_init in the caller's memory (nothing allocated, no side stream)
    int waves_per_block; // traversal launch shape
    int adj_tpw;         // targets per independent adjoint wave (16, 32 or 64)
    int adj_parts;       // independent adjoint walks split over the root's children (8) or not (1)
    int adj_sched;       // adjoint waves: 0 one per item in index order, 1 one persistent launch in the
                         // previous launch's cost order, 2 one per item in that order
    int adj_resident;    // workgroups of that launch resident at once (grid of the persistent launch)
    int field_sched;     // the last bh_build ordered the forward walk's wave items (bh_field follows it)
    int32_t *cnt_far, *cnt_near;  // optional per-target counters (device)
    hipEvent_t ev[4];             // optional timing events around the traversal kernels
    // The MD step's side stream (default priority, non-blocking) and its fork/join events: the wave
    // ordering and the short-range forces run there, beside the tree build.
    hipStream_t side;
    hipEvent_t fork_ev, sorted_ev, join_ev;
};

// ---- shared device helpers -----------------------------------------------------------------------

__host__ __device__ inline uint64_t spread3(uint32_t v)
{
    // Spread the low 21 bits of v so that bit k moves to bit 3k.
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Inverse of spread3: gather bits 0, 3, 6, ... of x into the low 21 bits.
__host__ __device__ inline uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x001f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x001f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

__host__ __device__ inline uint64_t morton(uint32_t qx, uint32_t qy, uint32_t qz)
{
    return (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

__device__ inline void set_flag(uint32_t *status, uint32_t bit)
{
    atomicOr(status, bit);
}

// Calls in flight on a handle's workspace.  Every entry point that uses the workspace counts itself in
// with its first kernel and out with its last, in its stream's order, so calls on one stream never see
// each other.  A call that finds another one in flight (calls on one handle overlapping on streams that
// are not ordered with each other) sets BH_FLAG_OVERLAP.  This detects the misuse; it does not prevent
// the race.
constexpr int kStatusInFlight = 12;  // status word slot of the count
__device__ inline void call_enter(uint32_t *status)
{
    if (atomicAdd(status + kStatusInFlight, 1u) != 0u) set_flag(status, BH_FLAG_OVERLAP);
}
__device__ inline void call_leave(uint32_t *status) { atomicSub(status + kStatusInFlight, 1u); }

inline unsigned grid_for(int64_t work, int threads, int64_t cap = (int64_t)1 << 30)
{
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Whether the traversals of this layout take their targets in Hilbert order (w.tgt_order) rather than in
// sorted (Morton) order.
inline bool uses_target_order(const Layout &L) { return L.n >= kTargetOrderMin; }

// Launch helpers implemented per source file.
// Tree build; with d_mom the moments are gathered and summed in the same upward pass (the MD step).
// With a side stream, h.sorted_ev is recorded once the sorted codes, permutation, positions and cube are
// final, the side stream waits for it and computes the traversal's target order, then enqueues
// after_sort's work (which needs only the sorted particles), beside the rest of the build; with join the
// caller's stream then waits for the side stream at the end of the build, without it the caller joins
// the side stream itself (h.join_ev) before the traversal.  Without a side stream everything runs on s.
// With enter, the build's first kernel counts the call in (call_enter).
using SortedWork = std::function<hipError_t(hipStream_t)>;
hipError_t launch_build(Handle &h, const double *d_pos, hipStream_t s, const double *d_mom = nullptr,
                        hipStream_t side = nullptr, bool join = true, bool enter = false,
                        const SortedWork &after_sort = nullptr);
// Targets of every system in Hilbert order (the positions' cells at kHilbertBits bits per axis), sorted
// positions as values: consecutive targets of a traversal wave then lie close together.
void launch_target_order(Handle &h, hipStream_t s);
hipError_t launch_upward_moments(Handle &h, const double *d_mom, hipStream_t s);
hipError_t launch_upward_first_moments(Handle &h, hipStream_t s);
hipError_t launch_field(Handle &h, const double *d_mom, const double *d_hext, double *d_H,
                        double *d_E, hipStream_t s);
// moments_done: the build already summed the moments (launch_build with d_mom).
// order_done: the wave order of the persistent launch was already enqueued (launch_order_waves).
hipError_t launch_backward(Handle &h, const double *d_mom, const double *d_hext, const double *d_gH,
                           const double *d_gE, double *d_dpos, double *d_dmom, double *d_dhext,
                           hipStream_t s, double *d_H = nullptr, double *d_E = nullptr, bool moments_done = false,
                           bool order_done = false);
// Whether the fused traversal of this handle runs the persistent, cost-ordered launch, and the launch
// that orders its items from the costs the previous traversal recorded.
bool uses_wave_order(const Handle &h);
void launch_order_waves(Handle &h, hipStream_t s);
// The same ordering for any list of wave items: item order from per-item costs, work counters reset.
void launch_order_items(const uint32_t *cost, int nw, uint32_t *order, uint32_t *work_ctr, hipStream_t s);
// Order of the forward walk's items from the costs the previous forward walk recorded.
void launch_order_field(Handle &h, hipStream_t s);
void launch_energy_final(Handle &h, double *d_E, hipStream_t s, int targets_per_wave);
hipError_t adjoint_resident_blocks(Handle &h, int &blocks);
hipError_t launch_ap(int64_t n, int32_t batch, int32_t precision, const double *pos, const double *mom,
                     const double *hext, double *H, double *dEdr, double *E, hipStream_t s);
hipError_t launch_md(Handle &h, const md_state *st, const md_params *mp, hipStream_t s);

}  // namespace ffbh
