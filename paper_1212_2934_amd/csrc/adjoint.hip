// Adjoint of the Barnes-Hut field: dL/dr and dL/dm for L = sum_i Hbar_i . H_i (+ the explicit
// dependence of E on m), with the tree, memberships and acceptance decisions of the forward pass held
// fixed.  The traversal is recomputed (nothing is stored from the forward pass): the same per-lane
// decisions are taken in the same order, and for every interaction
//   far (i, C):  dL/dr_i += g(x; Hbar_i, M_C);  B_C -= g;  A_C += T(x) Hbar_i      (x = r_i - c_C)
//   near (i, k): dL/dr_i += g(x; Hbar_i, m_k);  dL/dr_k -= g;  dL/dm_k += T(x) Hbar_i
// where g is the summand of the reduced dipolar force f_dip (Sec. 2) and T the dipole-field tensor of
// Eq. (H_dip).  Cell adjoints reach the members in a downward pass: every member k of C receives
// A_C in dL/dm_k and B_C / n_C in dL/dr_k (c_C is the mean of the members, Eq. magCenter).
// Scatters are reduced across the wave before one FP64 atomic per value.  The records hold the sums of
// +g (S_C = -B_C for a cell, the sum of g over a source's partners for a particle), and the downward pass
// subtracts them, so the scattered values need no negation.
#include "traverse.h"

namespace ffbh {

__device__ inline void atomic_add_d(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Six scatter values of one wave added to six consecutive doubles at p (a 64-byte aligned record): the
// values are summed over the wave (lanes that do not contribute pass zeros) and the six lanes holding the
// totals add them with one atomic instruction, so the memory system sees one request per record.
// wcomp = total6_comp(lane).  Uniform control flow.
template <typename T>
__device__ inline void scatter6(uint64_t who, int lane, int wcomp, double *p, T v0, T v1, T v2, T v3, T v4, T v5)
{
    // reduced whatever `who` holds (no branch around the reduction, so the inputs need no copies); only
    // the atomic is skipped for an empty mask
    const T t = wave_total6<T>(lane, v0, v1, v2, v3, v4, v5);
    if (who != 0ull && wcomp >= 0) atomic_add_d(p + wcomp, (double)t);
}

// One pair of the fused traversal for a target with upstream field gradient a: adds the gathered dL/dr
// (g) and the field of b to the target's sums (FP32 partials since the last flush in MIXED mode, FP64
// otherwise) and returns g and T(x) a for the scatter.  Lanes with `use` false add and return zeros.
template <bool MIXED, typename T>
__device__ inline void fused_pair(bool use, T r2, T x, T y, T z, T ax, T ay, T az, T bx, T by, T bz, T &gx, T &gy,
                                  T &gz, T &tx, T &ty, T &tz, T &pgx, T &pgy, T &pgz, T &phx, T &phy, T &phz,
                                  double &grx, double &gry, double &grz, double &hx, double &hy, double &hz)
{
    if constexpr (MIXED) {
        T ug[3] = {pgx, pgy, pgz};
        adj_field_r2<T, true>(use, r2, x, y, z, ax, ay, az, bx, by, bz, gx, gy, gz, tx, ty, tz, phx, phy, phz, ug);
        pgx = ug[0]; pgy = ug[1]; pgz = ug[2];
    } else {
        adj_field_r2<T>(use, r2, x, y, z, ax, ay, az, bx, by, bz, gx, gy, gz, tx, ty, tz, hx, hy, hz);
        grx += gx; gry += gy; grz += gz;
    }
}

// Contact pairs of the FP32-mixed walk.  A chain bead's two neighbours pull it with forces of about 5 (in
// reduced units) in opposite directions, and its net force can be a thousand times smaller, so the FP32
// rounding of those two pairs (offset and arithmetic, about 1e-6 each) would dominate its error.  Direct
// pairs closer than 1.25 d (measured on the FP32 offset) are therefore listed per target during the walk
// and evaluated in FP64 after it, at most kCloseMax per target (any further ones stay FP32).
constexpr int kCloseMax = 6;
constexpr float kClose2 = 1.5625f;  // (1.25 d)^2
template <bool ON>
struct CloseList {
};
template <>
struct CloseList<true> {
    uint32_t n[kWave];             // listed partners per target lane
    int32_t k[kWave][kCloseMax];   // their sorted indices
};

// Per-wave LDS of the fused traversal (dynamic shared memory, one record per wave of the block).
template <typename T>
struct AdjLds {
    LdsTarget tgt[kWave];  // the wave's targets
    T hb[kWave][4];        // their upstream field gradients
    T acc[kWave][6];       // direct-sum g (0..2) and field (3..5) of the current leaf, by owner lane
    T sbuf[16][6];         // member totals of the current chunk: sum g (0..2), sum T(x) a (3..5)
    int list[kWave];       // lanes that opened the current leaf
    CloseList<std::is_same<T, float>::value> cl;  // contact pairs deferred to FP64 (FP32-mixed walk)
};

// Direct sums of one leaf (first, count) for the c listed lanes, in groups of G lanes (see the compacted
// direct sums in traverse.h).  Lane b of group g pairs member b with listed target t0 + g: the group's
// totals of g and of the field go to the target's LDS slot; the member's totals over all listed targets
// are summed across the groups and added to its record with one atomic per component.
template <int G, typename T, typename Src>
__device__ inline void adj_leaf(AdjLds<T> &W, int lane, const Src *__restrict__ sr, double *__restrict__ g_rm,
                                int first, int count, int c, bool &coincident)
{
    const int grp = lane / G, b = lane % G;
    for (int c0 = 0; c0 < count; c0 += G) {
        const int cn = min(G, count - c0);
        const bool sok = b < cn;
        const int k = first + c0 + (sok ? b : 0);
        const Src sk = sr[k];
        const T mx = (T)sk.mx, my = (T)sk.my, mz = (T)sk.mz;
        T s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
        for (int t0 = 0; t0 < c; t0 += kWave / G) {
            const int a = t0 + grp;
            const bool tok = a < c;
            const int tl = W.list[tok ? a : 0];
            const LdsTarget tg = W.tgt[tl];
            const T ax = W.hb[tl][0], ay = W.hb[tl][1], az = W.hb[tl][2];
            const T x = (T)(tg.rx - sk.x), y = (T)(tg.ry - sk.y), z = (T)(tg.rz - sk.z);
            const T r2 = norm2<T>(x, y, z);
            const bool other = tok && sok && k != tg.si;
            bool deferred = false;
            if constexpr (std::is_same<T, float>::value) {
                // a contact pair goes to the target's list (evaluated in FP64 after the walk) while it has room
                if (other && r2 > (T)0 && r2 < kClose2) {
                    const uint32_t q = __hip_atomic_fetch_add(&W.cl.n[tl], 1u, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_WAVEFRONT);
                    if (q < (uint32_t)kCloseMax) {
                        W.cl.k[tl][q] = k;
                        deferred = true;
                    }
                }
            }
            const bool use = other && r2 > (T)0 && !deferred;
            coincident |= other && !(r2 > (T)0);
            T qx, qy, qz, ux, uy, uz, hx = 0, hy = 0, hz = 0;
            adj_field_r2<T>(use, r2, x, y, z, ax, ay, az, mx, my, mz, qx, qy, qz, ux, uy, uz, hx, hy, hz);
            s0 += qx; s1 += qy; s2 += qz;
            s3 += ux; s4 += uy; s5 += uz;
            T o0, o1;
            group_sum6<G>(lane, qx, qy, qz, hx, hy, hz, o0, o1);
            if constexpr (G == 4) {
                const int j = lane & 3;  // holds slots 2j, 2j + 1
                if (tok && j < 3) {
                    lds_add(&W.acc[tl][2 * j], o0);
                    lds_add(&W.acc[tl][2 * j + 1], o1);
                }
            } else {
                if (tok && b < 6) lds_add(&W.acc[tl][b], o0);  // lane b < 6 holds slot b
            }
        }
        // sum g (subtracted from dL/dr_k downstream), dL/dm_k += sum T(x) a over the listed targets: the row
        // swaps move two of the six values each (rows 0..3 of x0 carry components 0, 2, 1, 3 and rows 0, 1 /
        // 2, 3 of x1 carry 4 / 5),
        // then lanes of equal member index inside a row are added
        const T w0 = swap32_pair(s0, s1), w1 = swap32_pair(s2, s3), w2 = swap32_pair(s4, s5);
        const T x0 = row_stride_sum<G>(swap16_pair(w0, w1)), x1 = row_stride_sum<G>(swap16_sum(w2));
        const int row = lane >> 4, p = lane & 15;
        if (p < cn) {
            W.sbuf[p][row == 0 ? 0 : row == 1 ? 2 : row == 2 ? 1 : 3] = x0;
            if ((row & 1) == 0) W.sbuf[p][4 + (row >> 1)] = x1;
        }
        wave_lds_sync();
        for (int base = 0; base < 6 * cn; base += kWave) {
            const int idx = base + lane;
            if (idx < 6 * cn) {
                const int m = idx / 6, comp = idx - 6 * m;
                const T v = W.sbuf[m][comp];
                if (v != (T)0) atomic_add_d(g_rm + 8 * (int64_t)(first + c0 + m) + comp, (double)v);
            }
        }
        wave_lds_sync();
    }
}

// The deferred contact pairs of one target lane, in FP64: offset from the FP64 positions, pair arithmetic
// with the FP64 upstream gradient and source moment; g and the field go to the lane's FP64 sums, the
// member's share (g and T(x) a) to its record with FP64 atomics.  Lanes walk their own lists together.
__device__ inline void close_pairs(AdjLds<float> &W, int lane, bool valid, int si, double rx, double ry, double rz,
                                   const double *__restrict__ spos, const double *__restrict__ smom,
                                   const double *__restrict__ hbar, int64_t ntot, double *__restrict__ g_rm,
                                   double &grx, double &gry, double &grz, double &hx, double &hy, double &hz)
{
    wave_lds_sync();
    const uint32_t listed = valid ? W.cl.n[lane] : 0u;
    const int cnt = listed < (uint32_t)kCloseMax ? (int)listed : kCloseMax;
    const double ax = valid ? hbar[si] : 0.0, ay = valid ? hbar[ntot + si] : 0.0,
                 az = valid ? hbar[2 * ntot + si] : 0.0;
    for (int q = 0; q < kCloseMax; ++q) {
        const bool on = q < cnt;
        if (ballot(on) == 0ull) break;
        const int k = on ? W.cl.k[lane][q] : si;
        const double x = rx - spos[k], y = ry - spos[ntot + k], z = rz - spos[2 * ntot + k];
        const double bx = smom[k], by = smom[ntot + k], bz = smom[2 * ntot + k];
        double gx, gy, gz, tx, ty, tz;
        adj_field_r2<double>(on, norm2<double>(x, y, z), x, y, z, ax, ay, az, bx, by, bz, gx, gy, gz, tx, ty, tz,
                             hx, hy, hz);
        grx += gx; gry += gy; grz += gz;
        if (on) {
            double *r = g_rm + 8 * (int64_t)k;
            atomic_add_d(r, gx); atomic_add_d(r + 1, gy); atomic_add_d(r + 2, gz);
            atomic_add_d(r + 3, tx); atomic_add_d(r + 4, ty); atomic_add_d(r + 5, tz);
        }
    }
}

#define FFBH_ADJ_PARAMS                                                                                         \
    const NodeRec *__restrict__ nodes, const double *__restrict__ node_m64, const double *__restrict__ spos,     \
        const double *__restrict__ smom, const void *__restrict__ src, const double *__restrict__ hbar,          \
        const uint32_t *__restrict__ perm, const double *__restrict__ hext, double *__restrict__ g_gather,       \
        double *__restrict__ g_rm, double *__restrict__ node_adj, double *__restrict__ Hs,                       \
        double *__restrict__ Hout, double *__restrict__ e_part, uint32_t *__restrict__ status, int64_t n,        \
        int64_t ntot, int waves_per_seg, int num_waves, double theta2, int max_nodes, int tpw, int parts,        \
        double *__restrict__ part_buf, uint32_t *__restrict__ wave_cost, const void *__restrict__ node_q,         \
        double *__restrict__ node_adjq, const uint32_t *__restrict__ tgt_order, int inside_test
#define FFBH_ADJ_ARGS                                                                                           \
    nodes, node_m64, spos, smom, src, hbar, perm, hext, g_gather, g_rm, node_adj, Hs, Hout, e_part, status, n,   \
        ntot, waves_per_seg, num_waves, theta2, max_nodes, tpw, parts, part_buf, wave_cost, node_q, node_adjq,  \
        tgt_order, inside_test

// The fused walk of wave item gw.  If wave_cost is not null, lane 0 stores there a deterministic measure of
// the item's work (node visits plus leaf pair rounds), which orders the next launch.  QUAD: order-2 cells
// (node_q holds each node's first moment D, stride 16); an accepted cell adds its first-moment field, its
// gradient to the target and (negated) to the cell centre, and d/dD to node_adjq (six values, stride 8).
// SCALED: the node records hold s^2 / theta^2 and the acceptance test is s2 < d^2 (kMacScaled).
template <bool MIXED, bool QUAD, bool SCALED>
__device__ __forceinline__ void adjoint_wave(int gw, FFBH_ADJ_PARAMS)
{
    using T = typename std::conditional<MIXED, float, double>::type;
    using Src = typename std::conditional<MIXED, Src32, Src64>::type;
    const Src *__restrict__ sr = (const Src *)src;
    const int lane = threadIdx.x & (kWave - 1);
    const int wcomp = total6_comp(lane);
    // a wave owns tpw consecutive targets (lanes at and above tpw stay idle) and, with parts > 1, walks
    // the subtree of one child of the root (part p: child p); the parts' sums meet in k_parts_sum
    const int per_seg = waves_per_seg * parts;
    const int seg = gw / per_seg;
    const int grp = (gw - seg * per_seg) / parts, part = gw - seg * per_seg - grp * parts;
    const int local = grp * tpw + lane;
    const bool valid = lane < tpw && local < n;
    const int si = target_of(tgt_order, seg, n, local, valid);
    const double rx = spos[si], ry = spos[ntot + si], rz = spos[2 * ntot + si];
    const T ax = valid ? (T)hbar[si] : (T)0, ay = valid ? (T)hbar[ntot + si] : (T)0,
            az = valid ? (T)hbar[2 * ntot + si] : (T)0;

    double grx = 0.0, gry = 0.0, grz = 0.0;  // gathered dL/dr of the target (FP64)
    double hx = 0.0, hy = 0.0, hz = 0.0;     // forward field of the target (FP64)
    T pgx = 0, pgy = 0, pgz = 0, phx = 0, phy = 0, phz = 0;  // partial sums since the last flush
    bool coincident = false;
    AdjLds<T> &W = ((AdjLds<T> *)ffbh_dyn_lds)[threadIdx.x / kWave];
    W.tgt[lane] = LdsTarget{rx, ry, rz, si, 0};
    W.hb[lane][0] = ax; W.hb[lane][1] = ay; W.hb[lane][2] = az;
#pragma unroll
    for (int j = 0; j < 6; ++j) W.acc[lane][j] = (T)0;
    if constexpr (MIXED) W.cl.n[lane] = 0u;

    LaneStack st;
    if (parts == 1) {
        st.init(seg, 1, ballot(valid));
    } else {
        // the root holds every target of the system, so it is always opened: start at child `part` (a leaf
        // root is walked by part 0 alone)
        const NodeRec r = nodes[seg];
        const bool leaf_root = r.nchild == 0;
        const int first = leaf_root ? seg : r.child + part;
        int cnt = leaf_root ? (part == 0 ? 1 : 0) : (part < r.nchild ? 1 : 0);
        if (cnt > 0 && (unsigned)first >= (unsigned)max_nodes) {
            if (lane == 0) set_flag(status, BH_FLAG_TREE);
            cnt = 0;
        }
        st.init(first, cnt, ballot(valid));
    }
    // Node indices are checked where they enter the stack (the root above, child ranges at the push), so
    // every visited node is in [0, max_nodes); a wave pushes each internal node's children at most once,
    // so at most max_nodes pushes keep the walk finite whatever the tree holds.
    int guard = max_nodes;
    uint32_t work = 0;      // node visits plus leaf pair rounds (wave-uniform)
    while (st.more_any()) {
        uint64_t mask;
        const int cur = st.pop(mask);
        const NodeRec nd = nodes[cur];
        ++work;
        // masks of the lanes that take part, of the targets inside the node (opened whatever the test
        // says; below kSelfRejectTheta2 the test rejects them itself) and of the acceptance test
        uint64_t insm = 0ull;
        if (inside_test) insm = ballot((unsigned)(si - nd.first) < (unsigned)nd.count);
        const double dx = rx - nd.cx, dy = ry - nd.cy, dz = rz - nd.cz;
        const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const uint64_t accm = mask & ~insm & ballot(SCALED ? nd.s2 < d2 : nd.s2 < theta2 * d2);
        const bool acc = lane_in(accm);
        if (accm != 0ull) {
            // the whole wave evaluates the pair (lanes that do not accept add zeros)
            T bx, by, bz;
            if (MIXED) {
                bx = (T)nd.mx; by = (T)nd.my; bz = (T)nd.mz;
            } else {
                const double *m = node_m64 + 4 * (int64_t)cur;
                bx = (T)m[0]; by = (T)m[1]; bz = (T)m[2];
            }
            T gx, gy, gz, tx, ty, tz;
            fused_pair<MIXED, T>(acc, (T)d2, (T)dx, (T)dy, (T)dz, ax, ay, az, bx, by, bz, gx, gy, gz, tx, ty, tz,
                                 pgx, pgy, pgz, phx, phy, phz, grx, gry, grz, hx, hy, hz);
            T e0 = 0, e1 = 0, e2 = 0, e3 = 0, e4 = 0, e5 = 0;
            if constexpr (QUAD) {
                const T *qd = (const T *)node_q + 16 * (int64_t)cur;
                T Gx, Gy, Gz;
                first_moment_adj_r2<T>(acc, (T)d2, (T)dx, (T)dy, (T)dz, qd, ax, ay, az, Gx, Gy, Gz, e0, e1, e2, e3, e4,
                                       e5);
                if constexpr (MIXED) {
                    first_moment_acc_r2<T>(acc, (T)d2, (T)dx, (T)dy, (T)dz, qd, phx, phy, phz);
                    pgx += Gx; pgy += Gy; pgz += Gz;
                } else {
                    first_moment_acc_r2<T>(acc, (T)d2, (T)dx, (T)dy, (T)dz, qd, hx, hy, hz);
                    grx += Gx; gry += Gy; grz += Gz;
                }
                gx += Gx; gy += Gy; gz += Gz;
            }
            // A_C += sum T(x) Hbar over the accepting lanes, S_C += sum g (B_C = -S_C)
            scatter6<T>(accm, lane, wcomp, node_adj + 8 * (int64_t)cur, tx, ty, tz, gx, gy, gz);
            if constexpr (QUAD) scatter6<T>(accm, lane, wcomp, node_adjq + 8 * (int64_t)cur, e0, e1, e2, e3, e4, e5);
        }
        // One loop exit and one back edge: error exits clear the stack instead of breaking, so that the
        // accumulators stay in the same registers on every path (no copies at the merges).
        const uint64_t open = mask & ~accm;
        if (open != 0ull) {
            if (nd.nchild != 0) {
                if (--guard < 0 || nd.child < 0 || nd.nchild > 8 || nd.child + nd.nchild > max_nodes) {
                    if (lane == 0) set_flag(status, BH_FLAG_TREE);
                    st.clear();
                } else if (st.sp >= kStackMax) {
                    if (lane == 0) set_flag(status, BH_FLAG_STACK);
                    st.clear();
                } else {
                    st.push(lane, nd.child, nd.nchild, open);
                }
            } else if (nd.first < 0 || nd.count < 1 || (uint32_t)nd.first + (uint32_t)nd.count > (uint32_t)ntot) {
                // the member range is checked here, where it is first used to index memory
                if (lane == 0) set_flag(status, BH_FLAG_TREE);
                st.clear();
            } else {
                // leaf: direct sums over its members, packed over the lanes that opened it
                if (lane_in(open)) W.list[lanes_below(open)] = lane;
                const int c = __builtin_popcountll(open);
                wave_lds_sync();
                if (nd.count <= 4) adj_leaf<4>(W, lane, sr, g_rm, nd.first, nd.count, c, coincident);
                else if (nd.count <= 8) adj_leaf<8>(W, lane, sr, g_rm, nd.first, nd.count, c, coincident);
                else adj_leaf<16>(W, lane, sr, g_rm, nd.first, nd.count, c, coincident);
                {
                    const int G = nd.count <= 4 ? 4 : nd.count <= 8 ? 8 : 16;
                    work += (uint32_t)(((nd.count + G - 1) / G) * ((c * G + kWave - 1) / kWave + 1));
                }
                T d[6];
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    d[j] = W.acc[lane][j];
                    W.acc[lane][j] = (T)0;
                }
                if (MIXED) {
                    grx += (double)(pgx + d[0]); gry += (double)(pgy + d[1]); grz += (double)(pgz + d[2]);
                    hx += (double)(phx + d[3]); hy += (double)(phy + d[4]); hz += (double)(phz + d[5]);
                    pgx = pgy = pgz = phx = phy = phz = (T)0;
                } else {
                    grx += (double)d[0]; gry += (double)d[1]; grz += (double)d[2];
                    hx += (double)d[3]; hy += (double)d[4]; hz += (double)d[5];
                }
            }
        }
    }
    if constexpr (MIXED) {
        grx += (double)pgx; gry += (double)pgy; grz += (double)pgz;
        hx += (double)phx; hy += (double)phy; hz += (double)phz;
        close_pairs(W, lane, valid, si, rx, ry, rz, spos, smom, hbar, ntot, g_rm, grx, gry, grz, hx, hy, hz);
    }
    if (ballot(coincident) != 0ull && lane == 0) set_flag(status, BH_FLAG_COINCIDENT);
    if (wave_cost && lane == 0) wave_cost[gw] = work;
    if (parts > 1) {
        if (valid) {
            double *q = part_buf + (int64_t)part * 6 * ntot;
            q[si] = grx; q[ntot + si] = gry; q[2 * ntot + si] = grz;
            q[3 * ntot + si] = hx; q[4 * ntot + si] = hy; q[5 * ntot + si] = hz;
        }
        return;
    }

    double e = 0.0;
    if (valid) {
        const double mx = smom[si], my = smom[ntot + si], mz = smom[2 * ntot + si];
        e = -0.5 * (mx * hx + my * hy + mz * hz);
        if (hext) e -= mx * hext[3 * seg] + my * hext[3 * seg + 1] + mz * hext[3 * seg + 2];
    }
    e = wave_sum(e);
    if (lane == 0) e_part[gw] = e;
    if (valid) {
        g_gather[si] = grx;
        g_gather[ntot + si] = gry;
        g_gather[2 * ntot + si] = grz;
        Hs[si] = hx;
        Hs[ntot + si] = hy;
        Hs[2 * ntot + si] = hz;
        const int64_t i = (int64_t)perm[si] - (int64_t)seg * n;
        if (Hout && i >= 0 && i < n) {
            double *out = Hout + (int64_t)seg * 3 * n;
            out[i] = hx;
            out[n + i] = hy;
            out[2 * n + i] = hz;
        }
    }
}

// Independent-wave fused traversal.  Without work counters every wave takes one item: its global wave
// index, or with `order` the item at that place of the order (light items of the previous launch last,
// so the launch does not end on a long item).  With work counters the launch is persistent: each wave
// takes item after item in the order given, until the items run out.  Every wave reaches the exit: the
// counters only grow.
// Waves per SIMD: five for the FP32-mixed walk with the paper's cells (96 VGPRs, a few spilled bytes;
// 3 % faster MD step than at four), four for the others (the FP64 walk fits 128 VGPRs and runs 7 % faster
// than at three, but spills heavily at five).
// Segments of the persistent launch's item order: segment x holds the items i with i * kXcds / nw == x,
// which start at ceil(x nw / kXcds).
constexpr int kXcds = 8;
__host__ __device__ inline uint32_t order_segment_start(int x, int nw)
{
    return (uint32_t)(((int64_t)x * nw + kXcds - 1) / kXcds);
}

template <bool MIXED, bool QUAD, bool SCALED>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MIXED && !QUAD ? 5 : 4))) void k_adjoint(
    FFBH_ADJ_PARAMS, const uint32_t *__restrict__ order, uint32_t *__restrict__ work_ctr)
{
    if (!work_ctr) {
        // one wave per item; with an order, wave lin takes item order[lin] (heavy items of the previous
        // launch first within each XCD's range, light ones last)
        const int wpb = blockDim.x / kWave;
        const int lin = xcd_block(blockIdx.x, gridDim.x) * wpb + (int)(threadIdx.x / kWave);
        if (lin >= num_waves) return;
        int gw = lin;
        if (order) {
            const uint32_t o = order[lin];
            if (o < (uint32_t)num_waves) gw = (int)o;
        }
        adjoint_wave<MIXED, QUAD, SCALED>(gw, FFBH_ADJ_ARGS);
        return;
    }
    // The items are split into kXcds contiguous segments (neighbouring items share tree data).  Workgroups
    // are dispatched to the XCDs round-robin, so workgroup b runs on XCD b mod kXcds: its waves take items
    // of that XCD's segment first, keeping its L2 on one part of the tree, and then help the other
    // segments.  Each segment has its own work counter, which only grows, so every wave reaches the exit.
    const int lane = threadIdx.x & (kWave - 1);
    const int home = (int)(blockIdx.x % kXcds);
    for (int k = 0; k < kXcds; ++k) {
        const int sg = (home + k) % kXcds;
        const uint32_t s0 = order_segment_start(sg, num_waves), len = order_segment_start(sg + 1, num_waves) - s0;
        for (;;) {
            uint32_t v = 0u;
            if (lane == 0) v = atomicAdd(work_ctr + sg, 1u);
            const uint32_t item = __builtin_amdgcn_readfirstlane(v);
            if (item >= len) break;
            const uint32_t gw = order[s0 + item];
            if (gw >= (uint32_t)num_waves) {
                if (lane == 0) set_flag(status, BH_FLAG_TREE);
                return;
            }
            adjoint_wave<MIXED, QUAD, SCALED>((int)gw, FFBH_ADJ_ARGS);
        }
    }
}

// Order of the wave items of the next persistent launch, from the previous launch's costs, within each of
// the kXcds segments of consecutive items: the items outside the lightest ~45 % (of the whole launch)
// first, in index order (neighbouring items share tree data, so the launch keeps its cache locality), then
// the light items, heaviest first (64 buckets of the cost range), so each segment ends on short items.  A
// stable counting sort in one workgroup on the key (segment, class); then the segments' work counters are
// reset.  Costs all zero (first launch) give the index order.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 64;
constexpr int kOrderKeys = kXcds * kOrderBins;
// Share of the items moved to the end of their segment (measured at 2^20: 15 % and 30 % slower, 60 % and
// 75 % slower again; 45 % the fastest in both precisions).
constexpr uint32_t kLightPercent = 45u;

__global__ __launch_bounds__(kOrderThreads) void k_order_waves(const uint32_t *__restrict__ cost, int nw,
                                                               uint32_t *__restrict__ order,
                                                               uint32_t *__restrict__ work_ctr)
{
    constexpr int kWaves = kOrderThreads / kWave;
    __shared__ uint32_t red[kWaves];
    __shared__ uint32_t fine[kOrderBins];  // items per cost bucket, lightest bucket first
    __shared__ uint32_t hist[kOrderKeys];  // items per key, then the start of each key
    __shared__ uint32_t wcnt[kWaves][kOrderKeys];
    __shared__ int split;                  // buckets below it are the light items
    const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    uint32_t mx = 0u;
    for (int i = t; i < nw; i += kOrderThreads) mx = max(mx, cost[i]);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, off, kWave));
    if (lane == 0) red[wave] = mx;
    if (t < kOrderBins) fine[t] = 0u;
    __syncthreads();
    uint32_t cmax = 0u;
    for (int w = 0; w < kWaves; ++w) cmax = max(cmax, red[w]);
    auto bucket = [cmax](uint32_t c) -> int { return (int)((uint64_t)c * kOrderBins / ((uint64_t)cmax + 1u)); };
    for (int i = t; i < nw; i += kOrderThreads) atomicAdd(&fine[bucket(cost[i])], 1u);
    __syncthreads();
    if (t == 0) {
        // the light items: the lowest buckets holding at most kLightPercent % of the items (bucket 63
        // holds the heaviest item, so split <= 63 and the keys below fit in six bits)
        uint32_t acc = 0u;
        int sp = 0;
        while (sp < kOrderBins && (uint64_t)(acc + fine[sp]) * 100u <= (uint64_t)nw * kLightPercent)
            acc += fine[sp++];
        split = sp;
    }
    __syncthreads();
    const int sp = split;
    // key = segment * kOrderBins + class; class 0: heavy items; class k = 1..split: light bucket split - k
    // (heaviest light bucket first)
    auto key_of = [&](int i, uint32_t c) -> int {
        const int q = bucket(c);
        const int seg = (int)(((int64_t)i * kXcds) / nw);
        return seg * kOrderBins + (q >= sp ? 0 : sp - q);
    };
    // exclusive starts of the keys: count, then scan (one thread per key, then a serial scan)
    for (int k = t; k < kOrderKeys; k += kOrderThreads) hist[k] = 0u;
    __syncthreads();
    for (int i = t; i < nw; i += kOrderThreads) atomicAdd(&hist[key_of(i, cost[i])], 1u);
    __syncthreads();
    if (t == 0) {
        uint32_t start = 0u;
        for (int k = 0; k < kOrderKeys; ++k) {
            const uint32_t c = hist[k];
            hist[k] = start;
            start += c;
        }
    }
    __syncthreads();
    for (int c0 = 0; c0 < nw; c0 += kOrderThreads) {
        for (int k = t; k < kWaves * kOrderKeys; k += kOrderThreads) (&wcnt[0][0])[k] = 0u;
        __syncthreads();
        const int i = c0 + t;
        const bool ok = i < nw;
        const int b = ok ? key_of(i, cost[i]) : 0;
        // lanes of this wave with the same key, and this lane's rank among them
        uint64_t m = ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 9; ++bit) {
            const bool set = (b >> bit) & 1;
            const uint64_t v = ballot(set);
            m &= set ? v : ~v;
        }
        const int before = lanes_below(m);
        if (ok && before == 0) wcnt[wave][b] = (uint32_t)__builtin_popcountll(m);
        __syncthreads();
        for (int k = t; k < kOrderKeys; k += kOrderThreads) {
            uint32_t acc = hist[k];
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[w][k];
                wcnt[w][k] = acc;
                acc += c;
            }
            hist[k] = acc;
        }
        __syncthreads();
        if (ok) {
            const uint32_t at = wcnt[wave][b] + (uint32_t)before;
            if (at < (uint32_t)nw) order[at] = (uint32_t)i;
        }
        __syncthreads();
    }
    if (t < kXcds) work_ctr[t] = 0u;
}

// Sum of the parts of a split adjoint walk for every target, in part order (so the result does not depend
// on scheduling): gathered dL/dr, forward field (sorted order and caller order), and per-wave energy
// partials of 64 targets.  Grid: (ceil(n / 256), B) workgroups of 256.
__global__ __launch_bounds__(256) void k_parts_sum(const double *__restrict__ part_buf, int parts,
                                                   const double *__restrict__ smom, const double *__restrict__ hext,
                                                   const uint32_t *__restrict__ perm, double *__restrict__ g_gather,
                                                   double *__restrict__ Hs, double *__restrict__ Hout,
                                                   double *__restrict__ e_part, int64_t n, int64_t ntot)
{
    const int64_t local = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int seg = blockIdx.y;
    const bool valid = local < n;
    const int64_t si = (int64_t)seg * n + (valid ? local : 0);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (valid)
        for (int p = 0; p < parts; ++p)
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] += part_buf[((int64_t)p * 6 + c) * ntot + si];
    double e = 0.0;
    if (valid) {
        const double mx = smom[si], my = smom[ntot + si], mz = smom[2 * ntot + si];
        e = -0.5 * (mx * v[3] + my * v[4] + mz * v[5]);
        if (hext) e -= mx * hext[3 * seg] + my * hext[3 * seg + 1] + mz * hext[3 * seg + 2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            g_gather[c * ntot + si] = v[c];
            Hs[c * ntot + si] = v[3 + c];
        }
        const int64_t i = (int64_t)perm[si] - (int64_t)seg * n;
        if (Hout && i >= 0 && i < n) {
            double *out = Hout + (int64_t)seg * 3 * n;
            out[i] = v[3];
            out[n + i] = v[4];
            out[2 * n + i] = v[5];
        }
    }
    e = wave_sum(e);
    const int64_t wps = (n + kWave - 1) / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0 && local < n) e_part[(int64_t)seg * wps + local / kWave] = e;
}

// Upstream field gradient in sorted order: Hbar = gH - 1/2 gE m.
__global__ __launch_bounds__(256) void k_hbar(const double *__restrict__ gH, const double *__restrict__ gE,
                                              const double *__restrict__ smom, const uint32_t *__restrict__ perm,
                                              int64_t n, int64_t ntot, double *__restrict__ hbar)
{
    int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= ntot) return;
    const int64_t o = perm[s], b = o / n, i = o - b * n;
    if (o >= ntot) return;
    const double ge = gE ? gE[b] : 0.0;
    for (int a = 0; a < 3; ++a) {
        double v = gH ? gH[b * 3 * n + a * n + i] : 0.0;
        v += -0.5 * ge * smom[a * ntot + s];
        hbar[a * ntot + s] = v;
    }
}

__global__ __launch_bounds__(256) void k_zero(double *__restrict__ a, int64_t len)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) a[i] = 0.0;
}

// The node adjoint records of the nodes the last build made (their count is on the device).
__global__ __launch_bounds__(256) void k_zero_nodes(double *__restrict__ a, const uint32_t *__restrict__ nn,
                                                    int64_t max_nodes)
{
    const int64_t len = 8 * ((int64_t)*nn < max_nodes ? (int64_t)*nn : max_nodes);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) a[i] = 0.0;
}

// Downward pass and output: members collect their cells' adjoints along the leaf-to-root path; the
// explicit derivative of E in m (-1/2 H - H_ext, times dL/dE) is added; results go to caller order.
// With order-2 cells (node_adjq not null) a member j of cell C also receives, through
// D_C = sum (r_j - c_C) m_j^T and c_C = the members' mean, dL/dr_j += E_C m_j - E_C M_C / n_C and
// dL/dm_j += E_C (r_j - c_C) (E_C symmetric, stored as xx, yy, zz, xy, xz, yz).
__global__ __launch_bounds__(256) void k_downward(
    const NodeRec *__restrict__ nodes, const int32_t *__restrict__ leaf_of, const double *__restrict__ node_adj,
    const double *__restrict__ g_gather, const double *__restrict__ g_rm, const double *__restrict__ Hs,
    const double *__restrict__ hext, const double *__restrict__ gE,
    const uint32_t *__restrict__ perm, int64_t n, int64_t ntot, double *__restrict__ dpos,
    double *__restrict__ dmom, int64_t max_nodes, const double *__restrict__ node_adjq,
    const double *__restrict__ node_m64, const double *__restrict__ spos, const double *__restrict__ smom)
{
    int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= ntot) return;
    double Ax = 0.0, Ay = 0.0, Az = 0.0, Bx = 0.0, By = 0.0, Bz = 0.0;
    double qr[3] = {0.0, 0.0, 0.0}, qm[3] = {0.0, 0.0, 0.0};
    double rj[3] = {0.0, 0.0, 0.0}, mj[3] = {0.0, 0.0, 0.0};
    if (node_adjq) {
        for (int a = 0; a < 3; ++a) {
            rj[a] = spos[a * ntot + s];
            mj[a] = smom[a * ntot + s];
        }
    }
    int node = leaf_of[s];
    for (int depth = 0; node >= 0 && node < max_nodes && depth < 2 * kMaxLevel + 2; ++depth) {
        const double *a = node_adj + 8 * (int64_t)node;
        const NodeRec nd = nodes[node];
        const double inv = 1.0 / (double)nd.count;
        Ax += a[0]; Ay += a[1]; Az += a[2];
        Bx += a[3] * inv; By += a[4] * inv; Bz += a[5] * inv;
        if (node_adjq) {
            const double *e = node_adjq + 8 * (int64_t)node;
            const double E[3][3] = {{e[0], e[3], e[4]}, {e[3], e[1], e[5]}, {e[4], e[5], e[2]}};
            const double *M = node_m64 + 4 * (int64_t)node;
            const double d[3] = {rj[0] - nd.cx, rj[1] - nd.cy, rj[2] - nd.cz};
            for (int k = 0; k < 3; ++k) {
                qr[k] += E[k][0] * (mj[0] - M[0] * inv) + E[k][1] * (mj[1] - M[1] * inv) +
                         E[k][2] * (mj[2] - M[2] * inv);
                qm[k] += E[k][0] * d[0] + E[k][1] * d[1] + E[k][2] * d[2];
            }
        }
        node = nd.parent;
    }
    const int64_t o = perm[s], b = o / n, i = o - b * n;
    if (o >= ntot) return;
    const double ge = gE ? gE[b] : 0.0;
    const double *he = hext ? hext + 3 * b : nullptr;
    double *dp = dpos + b * 3 * n, *dm = dmom + b * 3 * n;
    const double *q = g_rm + 8 * s;
    dp[i] = g_gather[s] - q[0] - Bx + qr[0];
    dp[n + i] = g_gather[ntot + s] - q[1] - By + qr[1];
    dp[2 * n + i] = g_gather[2 * ntot + s] - q[2] - Bz + qr[2];
    double ex = -0.5 * Hs[s], ey = -0.5 * Hs[ntot + s], ez = -0.5 * Hs[2 * ntot + s];
    if (he) { ex -= he[0]; ey -= he[1]; ez -= he[2]; }
    dm[i] = q[3] + Ax + ge * ex + qm[0];
    dm[n + i] = q[4] + Ay + ge * ey + qm[1];
    dm[2 * n + i] = q[5] + Az + ge * ez + qm[2];
}

// dL/dH_ext = -dL/dE * sum_i m_i, one block per system.
__global__ __launch_bounds__(1024) void k_dhext(const double *__restrict__ mom, const double *__restrict__ gE,
                                                int64_t n, double *__restrict__ dhext)
{
    __shared__ double red[3][1024];
    const int b = blockIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += 1024)
        for (int a = 0; a < 3; ++a) s[a] += mom[(int64_t)b * 3 * n + a * n + i];
    for (int a = 0; a < 3; ++a) red[a][threadIdx.x] = s[a];
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 3; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) dhext[3 * b + threadIdx.x] = gE ? -gE[b] * red[threadIdx.x][0] : 0.0;
}

// Items of the independent-wave fused traversal: (system, target wave, part).
static int adjoint_items(const Handle &h)
{
    const int wps = (int)((h.L.n + h.adj_tpw - 1) / h.adj_tpw);
    return (int)(h.L.B * wps * h.adj_parts);
}

bool uses_wave_order(const Handle &h) { return h.adj_sched && h.adj_parts == 1; }

void launch_order_items(const uint32_t *cost, int nw, uint32_t *order, uint32_t *work_ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_order_waves, dim3(1), dim3(kOrderThreads), 0, s, cost, nw, order, work_ctr);
}

void launch_order_waves(Handle &h, hipStream_t s)
{
    launch_order_items(h.w.wave_cost, adjoint_items(h), h.w.wave_order, h.w.sched_ctr, s);
}

hipError_t launch_backward(Handle &h, const double *d_mom, const double *d_hext, const double *d_gH,
                           const double *d_gE, double *d_dpos, double *d_dmom, double *d_dhext, hipStream_t s,
                           double *d_H, double *d_E, bool moments_done, bool order_done)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    if (!moments_done) {
        hipError_t e = launch_upward_moments(h, d_mom, s);  // pseudo-particle moments
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_hbar, dim3(grid_for(L.ntot, 256)), dim3(256), 0, s, d_gH, d_gE, w.smom, w.perm, L.n,
                       L.ntot, w.hbar);
    hipLaunchKernelGGL(k_zero_nodes, dim3(grid_for(8 * L.max_nodes, 256, 2048)), dim3(256), 0, s, w.node_adj,
                       w.status + 2, L.max_nodes);
    const bool quad = L.expansion == 2;
    if (quad)
        hipLaunchKernelGGL(k_zero_nodes, dim3(grid_for(8 * L.max_nodes, 256, 2048)), dim3(256), 0, s, w.node_adjq,
                           w.status + 2, L.max_nodes);
    hipLaunchKernelGGL(k_zero, dim3(grid_for(8 * L.ntot, 256, 4096)), dim3(256), 0, s, w.g_rm, 8 * L.ntot);
    const int wpb = h.waves_per_block;
    const double theta2 = h.p.theta * h.p.theta;
    if (h.ev[2]) (void)hipEventRecord(h.ev[2], s);
    const bool mixed = h.p.precision == BH_FP32_MIXED;
    {
        const int tpw = h.adj_tpw, parts = h.adj_parts;
        const int wps = (int)((L.n + tpw - 1) / tpw);
        const int nwv = adjoint_items(h);
        const unsigned blk = (unsigned)((nwv + wpb - 1) / wpb);
        // cost-ordered launches: persistent (adj_sched 1: as many workgroups as can be resident at once,
        // items from per-XCD work counters) or one wave per item in that order (adj_sched 2)
        const bool sched = uses_wave_order(h);
        if (sched && !order_done) launch_order_waves(h, s);
        const bool persistent = sched && h.adj_sched == 1;
        const unsigned grid = persistent && (unsigned)h.adj_resident < blk ? (unsigned)h.adj_resident : blk;
        const uint32_t *ord = sched ? w.wave_order : nullptr;
        uint32_t *ctr = persistent ? w.sched_ctr : nullptr;
        uint32_t *cost = parts == 1 ? w.wave_cost : nullptr;
        const void *nq = mixed ? (const void *)w.node_q32 : (const void *)w.node_q64;
        const uint32_t *tgt = uses_target_order(L) ? w.tgt_order : nullptr;
        const int mac = mac_form(theta2);
        const int inside = mac == kMacInside ? 1 : 0;
        const bool scaled = mac == kMacScaled;
#define FFBH_ADJ(MX, QD, SC, T)                                                                                 \
    hipLaunchKernelGGL((k_adjoint<MX, QD, SC>), dim3(grid), dim3(wpb * kWave), wpb * sizeof(AdjLds<T>), s, w.nodes, \
                       w.node_m64, w.spos, w.smom, MX ? w.src32 : w.src64, w.hbar, w.perm, d_hext, w.g_gather,    \
                       w.g_rm, w.node_adj, w.Hs, d_H, w.e_part, w.status, L.n, L.ntot, wps, nwv, theta2,          \
                       (int)L.max_nodes, tpw, parts, w.part_buf, cost, nq, w.node_adjq, tgt, inside, ord, ctr)
        if (scaled) {
            if (mixed && quad) FFBH_ADJ(true, true, true, float);
            else if (mixed) FFBH_ADJ(true, false, true, float);
            else if (quad) FFBH_ADJ(false, true, true, double);
            else FFBH_ADJ(false, false, true, double);
        } else {
            if (mixed && quad) FFBH_ADJ(true, true, false, float);
            else if (mixed) FFBH_ADJ(true, false, false, float);
            else if (quad) FFBH_ADJ(false, true, false, double);
            else FFBH_ADJ(false, false, false, double);
        }
#undef FFBH_ADJ
        if (parts > 1)
            hipLaunchKernelGGL(k_parts_sum, dim3((unsigned)((L.n + 255) / 256), (unsigned)L.B), dim3(256), 0, s,
                               w.part_buf, parts, w.smom, d_hext, w.perm, w.g_gather, w.Hs, d_H, w.e_part, L.n,
                               L.ntot);
    }
    if (h.ev[3]) (void)hipEventRecord(h.ev[3], s);
    if (d_E)
        launch_energy_final(h, d_E, s, h.adj_parts > 1 ? kWave : h.adj_tpw);
    hipLaunchKernelGGL(k_downward, dim3(grid_for(L.ntot, 256)), dim3(256), 0, s, w.nodes, w.leaf_of, w.node_adj,
                       w.g_gather, w.g_rm, w.Hs, d_hext, d_gE, w.perm, L.n, L.ntot, d_dpos, d_dmom,
                       L.max_nodes, quad ? w.node_adjq : nullptr, w.node_m64, w.spos, w.smom);
    if (d_dhext)
        hipLaunchKernelGGL(k_dhext, dim3((unsigned)L.B), dim3(1024), 0, s, d_mom, d_gE, L.n, d_dhext);
    return hipGetLastError();
}

// Workgroups of the independent-wave fused traversal that fit on the device at once (for the persistent
// launch), with this handle's precision and waves per workgroup.
hipError_t adjoint_resident_blocks(Handle &h, int &blocks)
{
    const int wpb = h.waves_per_block;
    int per_cu = 0, cus = 0;
    hipError_t e;
    const bool quad = h.L.expansion == 2;
    const bool sc = mac_form(h.p.theta * h.p.theta) == kMacScaled;
    // the instantiation the handle launches (the occupancy depends on its registers)
    if (h.p.precision == BH_FP32_MIXED) {
        auto k = quad ? (sc ? k_adjoint<true, true, true> : k_adjoint<true, true, false>)
                      : (sc ? k_adjoint<true, false, true> : k_adjoint<true, false, false>);
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, wpb * kWave, wpb * sizeof(AdjLds<float>));
    } else {
        auto k = quad ? (sc ? k_adjoint<false, true, true> : k_adjoint<false, true, false>)
                      : (sc ? k_adjoint<false, false, true> : k_adjoint<false, false, false>);
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, wpb * kWave, wpb * sizeof(AdjLds<double>));
    }
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h.device);
    if (e != hipSuccess) return e;
    blocks = per_cu * cus;
    return blocks > 0 ? hipSuccess : hipErrorInvalidValue;
}

}  // namespace ffbh
