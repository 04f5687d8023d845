/*
 * ffbh.h -- C ABI of libffbh: Barnes-Hut dipolar field, its adjoint, and a Langevin MD step on one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem is the one stated in Sec. 2 of Polyakov et al., "Large-scale ferrofluid simulations on
 * graphics processing units" (arXiv:1212.2934): N identical particles with positions r_i and moments
 * m_i interact through the dipole field of Eq. (H_dip),
 *     H_i = sum_{j != i} [3 r_ij (m_j . r_ij) - m_j |r_ij|^2] / |r_ij|^5 ,   r_ij = r_i - r_j ,
 * in reduced units (diameter 1, no mu0/4pi prefactor).  The sum is approximated with the Barnes-Hut
 * scheme of Sec. 3.2: an octree over a bounding cube, cell pseudo-particles whose moment is the sum of
 * the members' moments and whose position is the members' geometric centre (Eq. magCenter), and a
 * per-target traversal that uses a cell's pseudo-particle when the target is far enough from it and
 * opens the cell otherwise.  "Far enough" (the paper gives no criterion) is, per target i and cell C:
 *     i is not a member of C  and  s_C^2 < (theta*theta) * d^2 ,
 * s_C the side of C's cube and d the distance from r_i to C's pseudo-particle.  Leaves hold at most
 * leaf_size particles; an unaccepted leaf is summed particle by particle (j != i).
 *
 * Memory.  Every pointer argument named d_* is DEVICE memory on the current HIP device; all other
 * pointers are host memory.  Vector fields are FP64 structure-of-arrays: a batch of B systems of n
 * particles is laid out (B, 3, n) -- x components of system b at [3bn, 3bn+n), y next, z next.
 * Device buffers are owned by the caller (e.g. torch tensors); the library never allocates or frees
 * device memory.  Its only device state is the caller-provided workspace, sized by
 * bh_workspace_bytes, which must stay allocated while the handle is used.  All work is enqueued on the
 * caller's stream (a hipStream_t passed as void*, NULL = the null stream); no call synchronises with
 * the host except bh_check_status.  All calls on one handle -- and replays of graphs captured from it --
 * share its workspace, so they must be ordered: enqueue them on one stream or order the streams.  Each
 * such call counts itself in and out on the device (its first and last kernels); a call that starts
 * while another one is in flight on the handle sets BH_FLAG_OVERLAP, so the misuse is reported, though
 * not prevented.  Two handles never share state and may run concurrently.
 *
 * Errors.  Arguments that can be checked on the host are checked before anything is enqueued; a
 * failing call returns a negative bh_status and enqueues nothing.  Conditions only the device can see
 * (non-finite input, two distinct particles at the same position, a cell that cannot be split below
 * leaf_size, traversal stack overflow, overlapping calls) set bits in a device status word that
 * bh_check_status reads and clears.
 */
#ifndef FFBH_H
#define FFBH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bh_status;

enum {
    BH_OK = 0,
    BH_EINVAL = -1,       /* bad argument (null pointer, n < 1, theta < 0, leaf_size outside 1..64),
                             or a call the handle's parameters do not support                        */
    BH_EWORKSPACE = -2,   /* workspace missing, misaligned or smaller than bh_workspace_bytes       */
    BH_EDEVICE = -3,      /* a HIP runtime call failed                                              */
    BH_EDEGENERATE = -4,  /* bh_check_status: the device flagged degenerate input                   */
    BH_ESTATE = -5        /* bh_field / bh_field_backward / md_step before a successful bh_build    */
};

/* Device status word bits (bh_check_status). */
enum {
    BH_FLAG_NONFINITE = 1u << 0,   /* a position or moment was NaN or infinite                      */
    BH_FLAG_COINCIDENT = 1u << 1,  /* two distinct particles at zero distance (pair skipped)         */
    BH_FLAG_DEEP_LEAF = 1u << 2,   /* a level-21 cell holds more than leaf_size particles            */
    BH_FLAG_STACK = 1u << 3,       /* traversal stack overflow (cannot happen for depth <= 21)       */
    BH_FLAG_TREE = 1u << 4,        /* internal consistency check failed; the affected walk stopped  */
    BH_FLAG_OVERLAP = 1u << 5      /* a call on the handle ran while another was in flight on it (calls
                                      on different streams not ordered with each other): both raced on
                                      the workspace and their results are void                      */
};

enum { BH_FP64 = 0, BH_FP32_MIXED = 1 };

/* Run parameters, fixed for the life of a handle. */
typedef struct bh_params {
    int64_t n;          /* particles per system, >= 1                                                 */
    int32_t batch;      /* independent systems B, >= 1                                                */
    int32_t leaf_size;  /* maximum particles per leaf, 1..64                                          */
    double theta;       /* opening parameter, >= 0 (0 gives the all-pairs sum)                        */
    int32_t precision;  /* BH_FP64: all arithmetic FP64.  BH_FP32_MIXED: pair arithmetic in FP32 on
                           FP64 offsets, FP64 acceptance test, FP64 cell sums and accumulation; the
                           walk of bh_field_backward and md_step evaluates direct pairs closer than
                           1.25 diameters in FP64 (up to six per target)                             */
    int32_t tuning_id;  /* traversal launch shape (see bh_num_tunings); -1 = default                  */
    int32_t expansion;  /* cells of the field, its adjoint and md_step: 0 or 1 = the paper's
                           pseudo-particles (Eq. magCenter); 2 = plus each accepted cell's first moment
                           D = sum_j (r_j - c) m_j^T, the next term of the Taylor expansion of Eq. H_dip
                           about c (beyond the paper; field error one power of theta lower)           */
} bh_params;

typedef struct bh_handle bh_handle;

/* Bytes of device workspace a handle with these parameters needs. */
bh_status bh_workspace_bytes(const bh_params *p, size_t *out_bytes);

/* Number of traversal launch shapes that tuning_id may select (0..count-1).  Every shape gives the same
 * forward field (bitwise) and interaction counts; the adjoint agrees to rounding (its sums are reduced in
 * another order).  Some shapes split each adjoint walk over the root's children and hold a partial-sum
 * buffer of 384 bytes per particle in the workspace (bh_workspace_bytes depends on tuning_id).  Others
 * order the adjoint walk's wave items by the cost each had in the previous call on the handle (the first
 * call after bh_create runs them in index order), in one persistent launch or one wave per item.  The
 * forward walk of bh_field takes its items in the order of its previous call's costs in every shape, from
 * 16384 particles up (ordered by bh_build). */
int32_t bh_num_tunings(void);

/* Create a handle (host memory, owned by the caller until bh_destroy) bound to the current HIP device
 * and to d_workspace (>= bh_workspace_bytes, 256-byte aligned, owned by the caller).  The handle also
 * owns one non-blocking HIP stream of default priority and three events, which bh_build and md_step use
 * internally (forked from and joined back into the caller's stream within the call); bh_destroy waits for
 * that stream and releases them. */
bh_status bh_create(const bh_params *p, void *d_workspace, size_t workspace_bytes, bh_handle **out);
/* Release a handle made by bh_create (BH_EINVAL for one made by bh_init). */
bh_status bh_destroy(bh_handle *h);

/* Bytes of host memory a handle occupies (the mem argument of bh_init). */
size_t bh_handle_bytes(void);

/* A handle in caller-owned memory, for callers that do not let the library allocate.  mem (at least
 * bh_handle_bytes() bytes, 16-byte aligned, host memory owned by the caller) receives a handle bound to the
 * current HIP device and to d_workspace, as bh_create makes it, but nothing is allocated: no host memory,
 * no stream, no event.  Two small kernels that set the workspace's status word and constants are enqueued
 * on `stream`; later calls on the handle are ordered after them by the caller, as any two calls are.
 * Without a side stream bh_build and md_step enqueue all their work on the caller's stream: results equal
 * those of a bh_create handle (the adjoint's to the rounding of its atomics), and large MD steps lose the
 * overlap of the short-range forces with the tree build.  Errors: BH_EINVAL for a null, short or
 * misaligned mem, bad parameters or a null out; BH_EWORKSPACE as for bh_create; BH_EDEVICE on a HIP error
 * (mem then holds no handle).  End it with bh_fini. */
bh_status bh_init(void *mem, size_t mem_bytes, const bh_params *p, void *d_workspace, size_t workspace_bytes,
                  void *stream, bh_handle **out);

/* End a handle made by bh_init.  Frees nothing: mem and the workspace are the caller's again once the
 * handle's work enqueued so far has finished.  BH_EINVAL for a handle made by bh_create. */
bh_status bh_fini(bh_handle *h);

/* Build the tree for positions d_pos (B, 3, n): bounding cube, Morton codes, radix sort, octree and
 * the geometric centre of every cell (Sec. 3.2 kernels 1-4, Eq. magCenter positions).  Systems of more
 * than 2048 particles also get the order in which the traversals group their targets (Hilbert order of
 * the particles' cells); it changes results only through the order of rounding. */
bh_status bh_build(bh_handle *h, const double *d_pos, void *stream);

/* Dipolar field and energy with the tree of the last bh_build (Eq. H_dip summed by the Sec. 3.2
 * traversal).  d_mom (B, 3, n) moments; d_hext (B, 3) external field or NULL (zero); d_H (B, 3, n)
 * receives the dipolar field (without H_ext); d_E (B) receives
 *     E = -1/2 sum_i m_i . H_i - sum_i m_i . H_ext
 * or may be NULL. */
bh_status bh_field(bh_handle *h, const double *d_mom, const double *d_hext, double *d_H, double *d_E,
                   void *stream);

/* Reverse-mode derivative of the field and energy of bh_field, with the tree, cell membership and
 * acceptance decisions of the last bh_build held fixed (they are piecewise constant in the
 * positions).  Given upstream gradients d_gH (B, 3, n) = dL/dH (or NULL = 0) and d_gE (B) = dL/dE (or
 * NULL = 0), writes d_dpos = dL/dr and d_dmom = dL/dm (B, 3, n) and, if d_dhext is not NULL,
 * d_dhext = dL/dH_ext (B, 3).  Per interaction the position derivative uses the gradient kernel of
 * the reduced dipolar force f_dip (Sec. 2). */
bh_status bh_field_backward(bh_handle *h, const double *d_mom, const double *d_hext,
                            const double *d_gH, const double *d_gE, double *d_dpos, double *d_dmom,
                            double *d_dhext, void *stream);

/* Langevin dynamics state, all device FP64 (B, 3, n), updated in place by md_step. */
typedef struct md_state {
    double *pos, *vel, *mom, *omega;
    uint64_t *d_step;   /* device step counter (one uint64), incremented by md_step */
} md_state;

/* Integrator parameters (reduced units).  Forces: -dE/dr of the Barnes-Hut energy plus a short-range
 * force between particles and against the faces of the box [box_lo, box_hi] (distance centre-to-face,
 * wall sigma = sigma/2), with strength wca_eps and length wca_sigma:
 *   sr_kind 0 (default): WCA repulsion 24 eps [2 (s/r)^12 - (s/r)^6] / r, cut at 2^(1/6) s;
 *   sr_kind 1: the paper's form (Eq. LJ, Sec. 2) 24 eps [(s/r)^12 - (s/r)^6] / r, zero at s, attractive
 *   beyond, cut at sr_cut (0: 2.5 s); walls of the same form, cut at sr_cut / 2.
 * Torque m x (-dE/dm).
 * Euler-Maruyama step of size dt for (r, v) and (m, omega) with friction gamma_t, gamma_r and
 * Gaussian noise of variance 2 gamma kT dt per component; m is rotated by omega*dt and renormalised.
 * Noise: Philox4x32-10 keyed by (seed, system), counter (step, particle, component-stream). */
typedef struct md_params {
    double dt, kT, gamma_t, gamma_r, mass, inertia, wca_eps, wca_sigma;
    double box_lo[3], box_hi[3];
    const double *d_hext;   /* (B, 3) or NULL */
    uint64_t seed;
    int32_t sr_kind;        /* 0 WCA, 1 the paper's form (see above) */
    double sr_cut;          /* cut-off of sr_kind 1; 0 = 2.5 sigma */
} md_params;

/* One MD step: bh_build on the current positions, field + adjoint of the energy, WCA forces, and the
 * integrator update.  Enqueued on the stream with no host synchronisation (capturable in a graph).  From
 * 16384 particles over the batch, the short-range forces and the ordering of the traversal's work run on
 * the handle's own stream, forked from `stream` (event record + wait) and joined back to it before the
 * traversal; smaller steps run on `stream` alone.  Either way the step starts after everything enqueued
 * on `stream` before it and is complete for everything enqueued on `stream` after it. */
bh_status md_step(bh_handle *h, const md_state *s, const md_params *p, void *stream);

/* Capture one md_step (everything it enqueues: kernel launches, and any fork to and join from the
 * handle's stream, which become graph edges) into a HIP graph on `stream` and instantiate it into
 * *graph_exec.  The stream must not be the null stream.  Replaying the graph
 * with bh_graph_launch performs one MD step on the same state buffers with the same parameters; the
 * noise advances with the device step counter, so replays continue the trajectory.  The handle,
 * workspace and state buffers must outlive the graph.  Release with bh_graph_destroy. */
bh_status bh_graph_capture_md(bh_handle *h, const md_state *s, const md_params *p, void *stream,
                              void **graph_exec);
bh_status bh_graph_launch(void *graph_exec, void *stream);
bh_status bh_graph_destroy(void *graph_exec);

/* All-pairs reference (Sec. 3.1, the all-pairs GPU step of Alg. 1).  For `batch` systems of n
 * particles in caller order (d_pos, d_mom: (B, 3, n) FP64), writes d_H (B, 3, n) with
 * H_i = sum_{j != i} T(r_i - r_j) m_j (Eq. H_dip); if not NULL, d_dEdr (B, 3, n) with the all-pairs
 * energy gradient dE/dr_i = -sum_{j != i} f_dip(r_i - r_j; m_i, m_j) (Sec. 2), and d_E (B) with
 * E = -1/2 sum m.H - sum m.H_ext (d_hext (B, 3) or NULL for no external field).  precision BH_FP64, or
 * BH_FP32_MIXED: offsets formed in FP64, pair arithmetic in FP32, partial sums over 256 sources
 * accumulated in FP64.  Distinct particles at the same position contribute nothing to each other.
 * O(n^2) work per system; needs no handle or workspace; enqueued on `stream` without host
 * synchronisation.  Returns BH_EINVAL for n < 1, batch outside [1, 65535], an unknown precision, or a
 * NULL or misaligned required pointer; BH_EDEVICE if the launch fails. */
bh_status bh_allpairs(int64_t n, int32_t batch, int32_t precision, const double *d_pos, const double *d_mom,
                      const double *d_hext, double *d_H, double *d_dEdr, double *d_E, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): bh_build followed by bh_field in one call, with no handle, no caller workspace
 * and no allocation of any kind.  The workspace is a fixed 64 MiB array of device memory that the library
 * reserves on every device it runs on when its code is loaded there, and holds until the process ends;
 * the first call on a device also looks up that array's address (do it once outside graph capture).
 * Parameters as for bh_create (tuning_id selects the forward traversal's launch shape); d_pos, d_mom,
 * d_hext, d_H and d_E as for bh_build and bh_field; d_flags (one uint32, device, or NULL) receives the
 * device status word of this call (the BH_FLAG_* bits).  The results equal those of bh_create + bh_build +
 * bh_field with the same parameters.
 * Returns BH_EWORKSPACE, before anything is enqueued, when the parameters need more workspace than the
 * array holds (bh_workspace_bytes > 64 MiB: up to about 65536 particles over the batch at leaf size 16),
 * BH_EINVAL for bad parameters or pointers, BH_EDEVICE on a HIP failure.  Every call on one device uses
 * the same array and leaves its contents behind; calls that overlap on one device (two streams, two
 * threads, or a replayed graph overlapping another call) race and give wrong results: order them. */
bh_status bh_field_noalloc(const bh_params *p, const double *d_pos, const double *d_mom, const double *d_hext,
                           double *d_H, double *d_E, uint32_t *d_flags, void *stream);

/* Read (and clear) the device status word; synchronises the stream.  Returns BH_EDEGENERATE if any
 * flag was set, BH_OK otherwise; the raw bits go to *flags if not NULL. */
bh_status bh_check_status(bh_handle *h, void *stream, uint32_t *flags);

/* Per-target interaction counts of the last bh_field (sorted order is undone): far cells and direct
 * partners, each int32 (B, n) device arrays.  Requires the handle to have been created with
 * counters enabled (bh_enable_counters before the bh_field call); costs one extra write per target. */
bh_status bh_enable_counters(bh_handle *h, int32_t *d_n_far, int32_t *d_n_near);

/* ---- Introspection (tests and tools) ------------------------------------------------------------ */

/* Number of octree nodes of the last bh_build (synchronises the stream). */
bh_status bh_num_nodes(bh_handle *h, void *stream, int64_t *out_nodes);

/* Copy the tree of the last bh_build into caller device buffers (any may be NULL).  Sorted order is
 * (system, Morton code, index).  d_perm (B*n) int32: sorted position -> global original index b*n+i.
 * Per node (num_nodes entries): d_first, d_count (sorted positions, global), d_level, d_nchild (0 for a
 * leaf), d_child_first (-1 for a leaf) as int32; d_centroid (3*num_nodes, AoS xyz) FP64; d_bbox (B*5:
 * lo_x, lo_y, lo_z, side, scale) FP64.  Roots are nodes 0..B-1.  Unary cells are collapsed: a chain
 * of cells with one non-empty child each is stored once, at the level of its deepest cell. */
bh_status bh_export_tree(bh_handle *h, int32_t *d_perm, int32_t *d_first, int32_t *d_count,
                         int32_t *d_level, int32_t *d_nchild, int32_t *d_child_first,
                         double *d_centroid, double *d_bbox, void *stream);

/* Timing hook: when set, bh_field records fwd_start / fwd_stop (hipEvent_t, created by the caller)
 * on its stream immediately before and after its traversal kernel, and bh_field_backward records
 * adj_start / adj_stop around its adjoint traversal kernel.  Pass NULL to disable. */
bh_status bh_set_timing_events(bh_handle *h, void *fwd_start, void *fwd_stop, void *adj_start,
                               void *adj_stop);

/* Host-side reference of the code of a quantised position (21 bits per axis): bit 3k+2 = bit k of qx,
 * bit 3k+1 = bit k of qy, bit 3k = bit k of qz.  Same function the device uses; no GPU needed. */
uint64_t bh_morton_code(uint32_t qx, uint32_t qy, uint32_t qz);

/* Static description of a status code. */
const char *bh_status_str(bh_status s);

#ifdef __cplusplus
}
#endif
#endif /* FFBH_H */
