// Forward Barnes-Hut traversal: dipolar field of Eq. (H_dip) on every particle and the energy
// E = -1/2 sum m.H - sum m.H_ext (Sec. 3.2 kernel 5: traversal with spatially close targets sharing a
// wavefront).
//
// One wavefront owns 64 consecutive targets in (system, Morton) order.  The wave walks the union of
// its lanes' traversals depth first, children in octant order: the node on top of the stack is
// fetched once for the whole wave with a scalar load, every lane in the node's lane mask applies its
// own acceptance test (FP64, exactly as the definition states), accepting lanes add the
// pseudo-particle's field, and the lanes that must open the node either sum the leaf directly or
// push the children with their mask.  Each lane therefore visits exactly its own cells in its own
// order, independent of the wave shape.
#include "traverse.h"

namespace ffbh {

template <bool MIXED, bool COUNT>
__global__ __launch_bounds__(512) void k_field(
    const NodeRec *__restrict__ nodes, const double *__restrict__ node_m64, const double *__restrict__ spos,
    const double *__restrict__ smom, const float *__restrict__ smom32, const uint32_t *__restrict__ perm,
    const double *__restrict__ hext, double *__restrict__ H, double *__restrict__ Hs,
    double *__restrict__ e_part, int32_t *__restrict__ cnt_far, int32_t *__restrict__ cnt_near,
    uint32_t *__restrict__ status, int64_t n, int64_t ntot, int waves_per_seg, int num_waves,
    double theta2, int max_nodes)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    const int gw = xcd_block(blockIdx.x, gridDim.x) * wpb + (int)(threadIdx.x / kWave);
    if (gw >= num_waves) return;  // whole waves only
    const int seg = gw / waves_per_seg;
    const int local = (gw - seg * waves_per_seg) * kWave + lane;
    const bool valid = local < n;
    const int si = (int)(seg * n) + (valid ? local : 0);
    const double rx = spos[si], ry = spos[ntot + si], rz = spos[2 * ntot + si];

    double hx = 0.0, hy = 0.0, hz = 0.0;
    int nfar = 0, nnear = 0;
    bool coincident = false;

    LaneStack st{0, 0, 0, 0, 0};
    st.push(lane, seg, seg + 1, __ballot(valid));
    int guard = max_nodes;  // a wave visits each node at most once
    while (st.sp > 0) {
        uint64_t mask;
        const int cur = st.pop(lane, mask);
        if (--guard < 0 || (unsigned)cur >= (unsigned)max_nodes) {
            if (lane == 0) set_flag(status, BH_FLAG_TREE);
            break;
        }
        const NodeRec nd = nodes[cur];
        if (nd.first < 0 || nd.count < 1 || (int64_t)nd.first + nd.count > ntot) {
            if (lane == 0) set_flag(status, BH_FLAG_TREE);
            break;
        }
        const bool active = (mask >> lane) & 1ull;
        const bool inside = (unsigned)(si - nd.first) < (unsigned)nd.count;
        bool acc = false;
        if (active && !inside) {
            const double dx = rx - nd.cx, dy = ry - nd.cy, dz = rz - nd.cz;
            const double d2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            acc = nd.s2 < theta2 * d2;
            if (acc) {
                if (MIXED) {
                    float fx = 0.f, fy = 0.f, fz = 0.f;
                    dip_acc<float>((float)dx, (float)dy, (float)dz, nd.mx, nd.my, nd.mz, fx, fy, fz);
                    hx += (double)fx;
                    hy += (double)fy;
                    hz += (double)fz;
                } else {
                    const double *m = node_m64 + 4 * (int64_t)cur;
                    dip_acc<double>(dx, dy, dz, m[0], m[1], m[2], hx, hy, hz);
                }
                if (COUNT) ++nfar;
            }
        }
        const uint64_t open = __ballot(active && !acc);
        if (open == 0ull) continue;
        if (nd.nchild != 0) {
            if (st.sp >= kStackMax) {
                if (lane == 0) set_flag(status, BH_FLAG_STACK);
                break;
            }
            st.push(lane, nd.child, nd.child + nd.nchild, open);
            continue;
        }
        // leaf that this lane must sum directly (members other than the target itself)
        const bool me = (open >> lane) & 1ull;
        const int k1 = nd.first + nd.count;
        if (MIXED) {
            float px = 0.f, py = 0.f, pz = 0.f;
            for (int k = nd.first; k < k1; ++k) {
                const double sx = spos[k], sy = spos[ntot + k], sz = spos[2 * ntot + k];
                const float mx = smom32[k], my = smom32[ntot + k], mz = smom32[2 * ntot + k];
                if (me && k != si) {
                    const float x = (float)(rx - sx), y = (float)(ry - sy), z = (float)(rz - sz);
                    if (x == 0.f && y == 0.f && z == 0.f) {
                        coincident = true;
                    } else {
                        dip_acc<float>(x, y, z, mx, my, mz, px, py, pz);
                        if (COUNT) ++nnear;
                    }
                }
            }
            hx += (double)px;
            hy += (double)py;
            hz += (double)pz;
        } else {
            for (int k = nd.first; k < k1; ++k) {
                const double sx = spos[k], sy = spos[ntot + k], sz = spos[2 * ntot + k];
                const double mx = smom[k], my = smom[ntot + k], mz = smom[2 * ntot + k];
                if (me && k != si) {
                    const double x = rx - sx, y = ry - sy, z = rz - sz;
                    if (x == 0.0 && y == 0.0 && z == 0.0) {
                        coincident = true;
                    } else {
                        dip_acc<double>(x, y, z, mx, my, mz, hx, hy, hz);
                        if (COUNT) ++nnear;
                    }
                }
            }
        }
    }
    if (__ballot(coincident) != 0ull && lane == 0) set_flag(status, BH_FLAG_COINCIDENT);

    // energy contribution of this wave: -1/2 m.H - m.H_ext
    double e = 0.0;
    if (valid) {
        const double mx = smom[si], my = smom[ntot + si], mz = smom[2 * ntot + si];
        const double *he = hext ? hext + 3 * seg : nullptr;
        e = -0.5 * (mx * hx + my * hy + mz * hz);
        if (he) e -= mx * he[0] + my * he[1] + mz * he[2];
    }
    e = wave_sum(e);
    if (lane == 0) e_part[gw] = e;

    if (valid) {
        Hs[si] = hx;
        Hs[ntot + si] = hy;
        Hs[2 * ntot + si] = hz;
        const int64_t o = perm[si];
        const int64_t i = o - (int64_t)seg * n;
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

template <bool MIXED, bool COUNT>
static void launch_k_field(Handle &h, const double *d_hext, double *d_H, hipStream_t s)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    const int wpb = h.waves_per_block;
    const unsigned blocks = (unsigned)((L.num_waves + wpb - 1) / wpb);
    const int waves_per_seg = (int)((L.n + kWave - 1) / kWave);
    const double theta2 = h.p.theta * h.p.theta;
    hipLaunchKernelGGL((k_field<MIXED, COUNT>), dim3(blocks), dim3(wpb * kWave), 0, s, w.nodes,
                       w.node_m64, w.spos, w.smom, w.smom32, w.perm, d_hext, d_H, w.Hs, w.e_part,
                       h.cnt_far, h.cnt_near, w.status, L.n, L.ntot, waves_per_seg, (int)L.num_waves, theta2, (int)L.max_nodes);
}

hipError_t launch_field(Handle &h, const double *d_mom, const double *d_hext, double *d_H, double *d_E,
                        hipStream_t s)
{
    hipError_t e = launch_upward_moments(h, d_mom, s);
    if (e != hipSuccess) return e;
    const bool mixed = h.p.precision == BH_FP32_MIXED;
    const bool cnt = h.cnt_far != nullptr;
    if (h.ev[0]) (void)hipEventRecord(h.ev[0], s);
    if (mixed && cnt) launch_k_field<true, true>(h, d_hext, d_H, s);
    else if (mixed) launch_k_field<true, false>(h, d_hext, d_H, s);
    else if (cnt) launch_k_field<false, true>(h, d_hext, d_H, s);
    else launch_k_field<false, false>(h, d_hext, d_H, s);
    if (h.ev[1]) (void)hipEventRecord(h.ev[1], s);
    if (d_E) launch_energy_final(h, d_E, s);
    return hipGetLastError();
}

void launch_energy_final(Handle &h, double *d_E, hipStream_t s)
{
    const int waves_per_seg = (int)((h.L.n + kWave - 1) / kWave);
    hipLaunchKernelGGL(k_energy_final, dim3((unsigned)h.L.B), dim3(256), 0, s, h.w.e_part, waves_per_seg, d_E);
}

}  // namespace ffbh
