// Forward Barnes-Hut traversal: dipolar field of Eq. (H_dip) on every particle and the energy
// E = -1/2 sum m.H - sum m.H_ext (Sec. 3.2 kernel 5: traversal with spatially close targets sharing a
// wavefront).
//
// One wavefront owns 64 consecutive targets of its system's target order (Hilbert order above 2048
// particles, sorted Morton order below).  The wave walks the union of
// its lanes' traversals depth first, children in octant order: the node on top of the stack is
// fetched once for the whole wave with a scalar load, every lane in the node's lane mask applies its
// own acceptance test (FP64, exactly as the definition states), accepting lanes add the
// pseudo-particle's field, and the lanes that must open the node either sum the leaf directly or
// push the children with their mask.  Each lane therefore visits exactly its own cells in its own
// order, independent of the wave shape.
#include "traverse.h"

namespace ffbh {

// Per-wave LDS of the forward traversal (dynamic shared memory, one record per wave of the block).
template <typename T>
struct FieldLds {
    LdsTarget tgt[kWave];  // the wave's targets
    T acc[kWave][4];       // direct-sum field of the current leaf, by owner lane
    int cnt[kWave];        // direct interactions of the current leaf (counting launches)
    int list[kWave];       // lanes that opened the current leaf
};

// Direct sums of one leaf (first, count) for the c listed lanes, in groups of G lanes (see the compacted
// direct sums in traverse.h): lane b of group g pairs member b with listed target t0 + g; the group's
// field total is added to the target's LDS slot.  Pairs are skipped for the target itself and flagged when
// coincident, as in the definition of the direct sum.
template <bool COUNT, int G, typename T, typename Src>
__device__ inline void field_leaf(FieldLds<T> &W, int lane, const Src *__restrict__ sr, int first, int count, int c,
                                  uint32_t &coincident)
{
    const int grp = lane / G, b = lane % G;
    const int slot = group3_slot<G>(lane);
    const bool wr = group3_writer<G>(lane) && slot < 3;
    for (int c0 = 0; c0 < count; c0 += G) {
        const int cn = min(G, count - c0);
        const bool sok = b < cn;
        const int k = first + c0 + (sok ? b : 0);
        const Src sk = sr[k];
        const T mx = (T)sk.mx, my = (T)sk.my, mz = (T)sk.mz;
        for (int t0 = 0; t0 < c; t0 += kWave / G) {
            const int a = t0 + grp;
            const bool tok = a < c;
            const int tl = W.list[tok ? a : 0];
            const LdsTarget tg = W.tgt[tl];
            const T x = (T)(tg.rx - sk.x), y = (T)(tg.ry - sk.y), z = (T)(tg.rz - sk.z);
            const T r2 = norm2<T>(x, y, z);
            const bool other = tok && sok && k != tg.si;
            const bool use = other && r2 > (T)0;
            coincident |= other && !(r2 > (T)0) ? 1u : 0u;
            T hx = 0, hy = 0, hz = 0;
            dip_acc_r2<T>(use, r2, x, y, z, mx, my, mz, hx, hy, hz);
            const T v = group_sum3<G>(lane, hx, hy, hz);
            if (tok && wr) lds_add(&W.acc[tl][slot], v);
            if constexpr (COUNT) {
                const uint64_t um = ballot(use) >> (grp * G);
                const int nu = __builtin_popcountll(um & ((1ull << G) - 1ull));
                if (tok && b == 0) lds_add(&W.cnt[tl], nu);
            }
        }
    }
}

// QUAD: accepted cells add their first-moment term (order-2 cells; node_q holds D per node, stride 16).
// MAC: the form of the acceptance test (MacForm: with the explicit test for cells holding the target,
// without it, or on squared sides scaled by 1/theta^2); a template argument rather than a kernel argument,
// because this walk is limited by scalar issue as much as by vector issue and a branch per visit costs two
// scalar instructions.
// Eight waves per SIMD (64 VGPRs): the FP64 walk spills a few bytes there and runs as fast as at seven;
// the FP32-mixed walk fits without spilling and runs 2-3 % faster than with the hint at seven.
template <bool MIXED, bool COUNT, bool QUAD, int MAC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8))) void k_field(
    const NodeRec *__restrict__ nodes, const double *__restrict__ node_m64, const double *__restrict__ spos,
    const double *__restrict__ smom, const void *__restrict__ src, const uint32_t *__restrict__ perm,
    const double *__restrict__ hext, double *__restrict__ H, double *__restrict__ Hs,
    double *__restrict__ e_part, int32_t *__restrict__ cnt_far, int32_t *__restrict__ cnt_near,
    uint32_t *__restrict__ status, int64_t n, int64_t ntot, int waves_per_seg, int num_waves,
    double theta2, int max_nodes, const void *__restrict__ node_q, const uint32_t *__restrict__ tgt_order,
    const uint32_t *__restrict__ order, uint32_t *__restrict__ wave_cost)
{
    using T = typename std::conditional<MIXED, float, double>::type;
    using Src = typename std::conditional<MIXED, Src32, Src64>::type;
    const Src *__restrict__ sr = (const Src *)src;
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int lin = xcd_block(blockIdx.x, gridDim.x) * wpb + (int)(threadIdx.x / kWave);
    if (lin >= num_waves) return;  // whole waves only
    // with an order, the wave takes the item at its place in it (heavy items of the previous walk first
    // within each XCD's range, light ones last); an order outside the items is ignored
    int gw = lin;
    if (order) {
        const uint32_t o = order[lin];
        if (o < (uint32_t)num_waves) gw = (int)o;
    }
    const int seg = gw / waves_per_seg;
    const int local = (gw - seg * waves_per_seg) * kWave + lane;
    const bool valid = local < n;
    const int si = target_of(tgt_order, seg, n, local, valid);
    const double rx = spos[si], ry = spos[ntot + si], rz = spos[2 * ntot + si];

    double hx = 0.0, hy = 0.0, hz = 0.0;  // FP64 accumulation
    T px = 0, py = 0, pz = 0;             // partial sums since the last flush (MIXED only)
    int nfar = 0, nnear = 0;
    // a lane value, not a bool: a divergent bool carried around the walk loop costs scalar mask merges at
    // every iteration
    uint32_t coincident = 0u;
    FieldLds<T> &W = ((FieldLds<T> *)ffbh_dyn_lds)[threadIdx.x / kWave];
    W.tgt[lane] = LdsTarget{rx, ry, rz, si, 0};
    W.acc[lane][0] = W.acc[lane][1] = W.acc[lane][2] = (T)0;
    W.cnt[lane] = 0;

    LaneStack st;
    st.init(seg, 1, ballot(valid));
    // Node indices are checked where they enter the stack (child ranges at the push; the root is the
    // system's), so every visited node is in [0, max_nodes); a wave pushes each internal node's children
    // at most once, so at most max_nodes pushes keep the walk finite whatever the tree holds.
    int guard = max_nodes;
    uint32_t rounds = 0;  // leaf pair rounds (wave-uniform)
    while (st.more()) {
        uint64_t mask;
        const int cur = st.pop_settled(mask);
        const NodeRec nd = nodes[cur];
        // masks of the lanes that take part, of the targets inside the node (opened whatever the test
        // says; below kSelfRejectTheta2 the test rejects them itself) and of the acceptance test
        uint64_t insm = 0ull;
        if constexpr (MAC == kMacInside) insm = ballot((unsigned)(si - nd.first) < (unsigned)nd.count);
        // acceptance test in FP64, exactly as defined
        const double dx = rx - nd.cx, dy = ry - nd.cy, dz = rz - nd.cz;
        const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        const uint64_t accm = mask & ~insm & ballot(MAC == kMacScaled ? nd.s2 < d2 : nd.s2 < theta2 * d2);
        const bool acc = lane_in(accm);
        if (accm != 0ull) {
            // the whole wave computes (lanes that do not accept add exact zeros)
            if (MIXED) {
                dip_acc_r2<T>(acc, (T)d2, (T)dx, (T)dy, (T)dz, (T)nd.mx, (T)nd.my, (T)nd.mz, px, py, pz);
            } else {
                const double *m = node_m64 + 4 * (int64_t)cur;
                dip_acc_r2<double>(acc, d2, dx, dy, dz, m[0], m[1], m[2], hx, hy, hz);
            }
            if (QUAD) {
                const T *D = (const T *)node_q + 16 * (int64_t)cur;
                if (MIXED) first_moment_acc_r2<T>(acc, (T)d2, (T)dx, (T)dy, (T)dz, D, px, py, pz);
                else first_moment_acc_r2<double>(acc, d2, dx, dy, dz, (const double *)D, hx, hy, hz);
            }
            if (COUNT) nfar += acc ? 1 : 0;
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
                if (nd.count <= 4) field_leaf<COUNT, 4>(W, lane, sr, nd.first, nd.count, c, coincident);
                else if (nd.count <= 8) field_leaf<COUNT, 8>(W, lane, sr, nd.first, nd.count, c, coincident);
                else field_leaf<COUNT, 16>(W, lane, sr, nd.first, nd.count, c, coincident);
                {
                    const int G = nd.count <= 4 ? 4 : nd.count <= 8 ? 8 : 16;
                    rounds += (uint32_t)(((nd.count + G - 1) / G) * ((c * G + kWave - 1) / kWave + 1));
                }
                wave_lds_sync();
                const T a0 = W.acc[lane][0], a1 = W.acc[lane][1], a2 = W.acc[lane][2];
                W.acc[lane][0] = W.acc[lane][1] = W.acc[lane][2] = (T)0;
                if (COUNT) {
                    nnear += W.cnt[lane];
                    W.cnt[lane] = 0;
                }
                if (MIXED) {
                    hx += (double)(px + a0); hy += (double)(py + a1); hz += (double)(pz + a2);
                    px = py = pz = (T)0;
                } else {
                    hx += (double)a0; hy += (double)a1; hz += (double)a2;
                }
            }
        }
        st.settle();
    }
    if (MIXED) {
        hx += (double)px; hy += (double)py; hz += (double)pz;
    }
    if (ballot(coincident != 0u) != 0ull && lane == 0) set_flag(status, BH_FLAG_COINCIDENT);
    // the item's work (internal nodes opened, times eight, plus leaf pair rounds) orders the next walk
    if (wave_cost && lane == 0) wave_cost[gw] = 8u * (uint32_t)(max_nodes - guard) + rounds;

    // energy contribution of this wave: -1/2 m.H - m.H_ext
    double e = 0.0;
    if (valid) {
        const double mx = smom[si], my = smom[ntot + si], mz = smom[2 * ntot + si];
        e = -0.5 * (mx * hx + my * hy + mz * hz);
        if (hext) e -= mx * hext[3 * seg] + my * hext[3 * seg + 1] + mz * hext[3 * seg + 2];
    }
    e = wave_sum(e);
    if (lane == 0) e_part[gw] = e;

    if (valid) {
        Hs[si] = hx;
        Hs[ntot + si] = hy;
        Hs[2 * ntot + si] = hz;
        const int64_t o = perm[si];
        const int64_t i = o - (int64_t)seg * n;
        if (i >= 0 && i < n) {  // always true for a consistent permutation
            double *out = H + (int64_t)seg * 3 * n;
            out[i] = hx;
            out[n + i] = hy;
            out[2 * n + i] = hz;
            if (COUNT) {
                cnt_far[o] = nfar;
                cnt_near[o] = nnear;
            }
        }
    }
}

// E of every system: sum of its waves' partials in a fixed order (strided per thread, then a fixed
// LDS tree), so repeated runs give the same bits.
__global__ __launch_bounds__(256) void k_energy_final(const double *__restrict__ e_part, int waves_per_seg,
                                                      double *__restrict__ E)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    double s = 0.0;
    for (int w = threadIdx.x; w < waves_per_seg; w += 256) s += e_part[(int64_t)b * waves_per_seg + w];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[b] = red[0];
}

template <bool MIXED, bool COUNT, bool QUAD>
static void launch_k_field(Handle &h, const double *d_hext, double *d_H, hipStream_t s)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    const int wpb = h.waves_per_block;
    const unsigned blocks = (unsigned)((L.num_waves + wpb - 1) / wpb);
    const int waves_per_seg = (int)((L.n + kWave - 1) / kWave);
    const double theta2 = h.p.theta * h.p.theta;
    const void *src = MIXED ? (const void *)w.src32 : (const void *)w.src64;
    using T = typename std::conditional<MIXED, float, double>::type;
    const size_t lds = (size_t)wpb * sizeof(FieldLds<T>);
    const void *q = MIXED ? (const void *)w.node_q32 : (const void *)w.node_q64;
    const uint32_t *tgt = uses_target_order(L) ? w.tgt_order : nullptr;
#define FFBH_FIELD(MAC)                                                                                          \
    hipLaunchKernelGGL((k_field<MIXED, COUNT, QUAD, MAC>), dim3(blocks), dim3(wpb * kWave), lds, s, w.nodes,         \
                       w.node_m64, w.spos, w.smom, src, w.perm, d_hext, d_H, w.Hs, w.e_part, h.cnt_far,          \
                       h.cnt_near, w.status, L.n, L.ntot, waves_per_seg, (int)L.num_waves, theta2,               \
                       (int)L.max_nodes, q, tgt, h.field_sched ? w.field_order : nullptr, w.field_cost)
    const int mac = mac_form(theta2);
    if (mac == kMacInside) FFBH_FIELD(kMacInside);
    else if (mac == kMacScaled) FFBH_FIELD(kMacScaled);
    else FFBH_FIELD(kMacPlain);
#undef FFBH_FIELD
}

hipError_t launch_field(Handle &h, const double *d_mom, const double *d_hext, double *d_H, double *d_E,
                        hipStream_t s)
{
    hipError_t e = launch_upward_moments(h, d_mom, s);
    if (e != hipSuccess) return e;
    const bool mixed = h.p.precision == BH_FP32_MIXED;
    const bool cnt = h.cnt_far != nullptr;
    if (h.ev[0]) (void)hipEventRecord(h.ev[0], s);
    if (h.L.expansion == 2) {
        if (mixed && cnt) launch_k_field<true, true, true>(h, d_hext, d_H, s);
        else if (mixed) launch_k_field<true, false, true>(h, d_hext, d_H, s);
        else if (cnt) launch_k_field<false, true, true>(h, d_hext, d_H, s);
        else launch_k_field<false, false, true>(h, d_hext, d_H, s);
    } else {
        if (mixed && cnt) launch_k_field<true, true, false>(h, d_hext, d_H, s);
        else if (mixed) launch_k_field<true, false, false>(h, d_hext, d_H, s);
        else if (cnt) launch_k_field<false, true, false>(h, d_hext, d_H, s);
        else launch_k_field<false, false, false>(h, d_hext, d_H, s);
    }
    if (h.ev[1]) (void)hipEventRecord(h.ev[1], s);
    if (d_E) launch_energy_final(h, d_E, s, kWave);
    return hipGetLastError();
}

void launch_order_field(Handle &h, hipStream_t s)
{
    launch_order_items(h.w.field_cost, (int)h.L.num_waves, h.w.field_order, h.w.field_ctr, s);
}

void launch_energy_final(Handle &h, double *d_E, hipStream_t s, int targets_per_wave)
{
    const int waves_per_seg = (int)((h.L.n + targets_per_wave - 1) / targets_per_wave);
    hipLaunchKernelGGL(k_energy_final, dim3((unsigned)h.L.B), dim3(256), 0, s, h.w.e_part, waves_per_seg, d_E);
}

}  // namespace ffbh
