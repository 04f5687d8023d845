// One Langevin MD step (Sec. 2 equations of motion in vector form, integrated with the explicit
// Euler-Maruyama scheme of Sec. 4; Sec. 3.2 kernel 6): tree build, Barnes-Hut field and energy gradient
// (fused forward + adjoint), a WCA short-range repulsion between particles (partners from a cell grid cut
// from the build's Morton codes) and against the container walls, and the update of positions,
// velocities, moments and angular velocities from the state at the start of the step.
//
// Readings: the paper writes the rotation in polar angles (with the theta/phi equations garbled); the
// vector form used here is m' = R(omega dt) m with I domega/dt = m x H_eff - gamma_r omega + noise,
// H_eff = -dE/dm.  Noise per Cartesian component has variance 2 gamma kT dt (fluctuation-dissipation).
// Short range (sr_kind): 0, the purely repulsive WCA potential (cut at 2^(1/6) sigma, shifted to zero
// there); 1, the paper's "Lennard-Jones" law as printed (Eq. LJ).  Walls of the same law act on the
// centre-to-face distance with sigma_w = sigma / 2.
// Thermal noise: Philox4x32-10 (Salmon et al., SC'11) keyed by (seed, system), counter (step, particle,
// draw), mapped to normals by the Box-Muller transform.
#include "traverse.h"

namespace ffbh {

// ---- Philox4x32-10 ----------------------------------------------------------------------------------

struct U4 {
    uint32_t x, y, z, w;
};

__device__ inline U4 philox_round(U4 c, uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 r;
    r.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    r.y = (uint32_t)p1;
    r.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    r.w = (uint32_t)p0;
    return r;
}

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        c = philox_round(c, k0, k1);
    }
    return c;
}

__device__ inline double u01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

// Two standard normals from two 32-bit words (Box-Muller).
__device__ inline void box_muller(uint32_t a, uint32_t b, double &n0, double &n1)
{
    const double r = sqrt(-2.0 * log(u01(a)));
    const double t = 6.283185307179586 * u01(b);
    n0 = r * cos(t);
    n1 = r * sin(t);
}

// ---- short-range forces (partners from a cell grid cut from the Morton codes) -----------------------------

// Force on a particle at offset x = r_i - r_k from a short-range partner, 24 eps [c12 (s/r)^12 - (s/r)^6] x / r^2
// for r < rc: c12 = 2 is the WCA repulsion, c12 = 1 the paper's form (Eq. LJ).
__device__ inline void sr_pair(double x, double y, double z, double s2, double eps, double c12, double rc2,
                               double &fx, double &fy, double &fz)
{
    const double r2 = x * x + y * y + z * z;
    if (r2 >= rc2 || r2 <= 0.0) return;
    const double sr2 = s2 / r2;
    const double sr6 = sr2 * sr2 * sr2;
    const double f = 24.0 * eps * (c12 * sr6 * sr6 - sr6) / r2;
    fx += f * x;
    fy += f * y;
    fz += f * z;
}

// Wall force along one axis for centre-to-face distances dlo (to the lower face) and dhi, the same law with
// sigma_w = sigma / 2 and cut rcw, the distance floored at sigma_w / 10.
__device__ inline double wall_force(double dlo, double dhi, double sw, double eps, double c12, double rcw)
{
    const double dmin = 0.1 * sw;
    double f = 0.0;
    if (dlo < rcw) {
        const double d = dlo > dmin ? dlo : dmin;
        const double s6 = (sw / d) * (sw / d) * (sw / d) * (sw / d) * (sw / d) * (sw / d);
        f += 24.0 * eps * (c12 * s6 * s6 - s6) / d;
    }
    if (dhi < rcw) {
        const double d = dhi > dmin ? dhi : dmin;
        const double s6 = (sw / d) * (sw / d) * (sw / d) * (sw / d) * (sw / d) * (sw / d);
        f -= 24.0 * eps * (c12 * s6 * s6 - s6) / d;
    }
    return f;
}

// Short-range partners are found on a cell grid cut from the Morton codes of the tree build: the level-L
// cell of a particle is the top 3L bits of its code, so the members of a cell are contiguous in the
// sorted order.  L is the finest level (at most the grid's cap) whose cells are at least the cut-off wide
// after allowing one quantisation step, so every partner within the cut-off lies in the 27 cells around a
// particle's own.
__device__ inline int grid_level(double side, double rc, int lcap)
{
    int L = lcap;
    while (L > 0 && side * (__builtin_ldexp(1.0, -L) - __builtin_ldexp(1.0, -kBits)) <= rc) --L;
    return L;
}

// Spread the low 10 bits of v so that bit k moves to bit 3k (grid coordinates have at most 7 bits).
__device__ inline uint32_t spread3_small(uint32_t v)
{
    uint32_t x = v & 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Member range [start, end) of the sorted particles of every occupied cell, written by the cell's first and
// last members; the table is cleared before (k_clear_cells), so an unoccupied cell reads as empty.
__global__ __launch_bounds__(256) void k_clear_cells(uint2 *__restrict__ cells, int64_t len)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256)
        cells[i] = make_uint2(0u, 0u);
}

__global__ __launch_bounds__(256) void k_cell_fill(const uint64_t *__restrict__ codes, const double *__restrict__ bbox,
                                                   int64_t n, int64_t ntot, double rc, int lcap, int64_t T,
                                                   uint2 *__restrict__ cells)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= ntot) return;
    const int64_t b = o / n, s = o - b * n;
    const int shift = 3 * (kBits - grid_level(bbox[8 * b + 3], rc, lcap));
    const uint64_t c = codes[o] >> shift;
    uint2 *e = cells + b * T + (int64_t)c;
    if (s == 0 || (codes[o - 1] >> shift) != c) e->x = (uint32_t)o;
    if (s == n - 1 || (codes[o + 1] >> shift) != c) e->y = (uint32_t)(o + 1);
}

// Short-range forces on every particle (one thread per sorted particle): partners from the 27 surrounding
// cells, then the container walls; written in the caller's order.  c12 selects the law, rc and rcw the cut-offs.
__global__ __launch_bounds__(256) void k_wca(const uint64_t *__restrict__ codes, const double *__restrict__ bbox,
                                             const uint2 *__restrict__ cells, const double *__restrict__ spos,
                                             const uint32_t *__restrict__ perm, double *__restrict__ F, int64_t n,
                                             int64_t ntot, int lcap, int64_t T, double sigma, double eps,
                                             double c12, double rc, double rcw, double3 box_lo, double3 box_hi)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= ntot) return;
    const int64_t b = o / n, lo_i = b * n, hi_i = lo_i + n;
    const double rx = spos[o], ry = spos[ntot + o], rz = spos[2 * ntot + o];
    const double rc2 = rc * rc, s2 = sigma * sigma;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (eps > 0.0) {
        const int L = grid_level(bbox[8 * b + 3], rc, lcap);
        const int shift = 3 * (kBits - L), down = kBits - L;
        const uint64_t code = codes[o];
        const int cx = (int)(compact3(code >> 2) >> down), cy = (int)(compact3(code >> 1) >> down),
                  cz = (int)(compact3(code) >> down);
        const int cmax = (1 << L) - 1;
        const uint2 *tab = cells + b * T;
        // Per slab of nine cells: the member ranges are read before any member, so their loads overlap
        // (all 27 at once takes 152 VGPRs and ran 30 % slower).  The slab's members are then walked as one
        // list (candidate t lies in the last cell whose running count is at most t), so a wave iterates
        // as often as its busiest lane has candidates, not as often as the sum over the cells of the
        // busiest lane per cell, and no load waits for another.
        for (int dz = -1; dz <= 1; ++dz) {
            const int nz = cz + dz;
            if ((unsigned)nz > (unsigned)cmax) continue;
            uint32_t first[9], cnt[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int nx = cx + k % 3 - 1, ny = cy + k / 3 - 1;
                const bool in = (unsigned)nx <= (unsigned)cmax && (unsigned)ny <= (unsigned)cmax;
                const uint2 r = in ? tab[(spread3_small((uint32_t)nx) << 2) | (spread3_small((uint32_t)ny) << 1) |
                                         spread3_small((uint32_t)nz)]
                                   : make_uint2(0u, 0u);
                // a range always lies inside this system's block of sorted particles
                const int64_t j0 = (int64_t)r.x > lo_i ? (int64_t)r.x : lo_i;
                const int64_t j1 = (int64_t)r.y < hi_i ? (int64_t)r.y : hi_i;
                first[k] = (uint32_t)j0;
                cnt[k] = j1 > j0 ? (uint32_t)(j1 - j0) : 0u;
            }
            uint32_t start[9], tot = 0u;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                start[k] = tot;
                tot += cnt[k];
            }
            for (uint32_t t = 0; t < tot; ++t) {
                uint32_t j = first[0] + t;
#pragma unroll
                for (int k = 1; k < 9; ++k)
                    if (t >= start[k]) j = first[k] + (t - start[k]);
                if ((int64_t)j == o) continue;
                sr_pair(rx - spos[j], ry - spos[ntot + j], rz - spos[2 * ntot + j], s2, eps, c12, rc2, fx, fy, fz);
            }
        }
        // container walls
        const double sw = 0.5 * sigma;
        fx += wall_force(rx - box_lo.x, box_hi.x - rx, sw, eps, c12, rcw);
        fy += wall_force(ry - box_lo.y, box_hi.y - ry, sw, eps, c12, rcw);
        fz += wall_force(rz - box_lo.z, box_hi.z - rz, sw, eps, c12, rcw);
    }
    const int64_t i = (int64_t)perm[o] - lo_i;
    if (i < 0 || i >= n) return;
    double *out = F + b * 3 * n;
    out[i] = fx;
    out[n + i] = fy;
    out[2 * n + i] = fz;
}

// ---- integrator ---------------------------------------------------------------------------------------

struct MDConst {
    double dt, kT, gamma_t, gamma_r, mass, inertia;
    uint64_t seed;
};

__global__ __launch_bounds__(256) void k_integrate(double *__restrict__ pos, double *__restrict__ vel,
                                                   double *__restrict__ mom, double *__restrict__ omega,
                                                   const double *__restrict__ dEdr, const double *__restrict__ dEdm,
                                                   const double *__restrict__ Fsr, const uint64_t *__restrict__ d_step,
                                                   int64_t n, int64_t ntot, MDConst c)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= ntot) return;
    const int64_t b = g / n, i = g - b * n;
    const int64_t o = b * 3 * n + i;  // x component; y at +n, z at +2n
    const uint64_t step = *d_step;
    // noise: two Philox blocks -> eight normals, six used
    const uint32_t k0 = (uint32_t)c.seed, k1 = (uint32_t)(c.seed >> 32) ^ (uint32_t)b;
    const U4 q0 = philox4x32_10(U4{(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)i, 0u}, k0, k1);
    const U4 q1 = philox4x32_10(U4{(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)i, 1u}, k0, k1);
    double xi[8];
    box_muller(q0.x, q0.y, xi[0], xi[1]);
    box_muller(q0.z, q0.w, xi[2], xi[3]);
    box_muller(q1.x, q1.y, xi[4], xi[5]);
    box_muller(q1.z, q1.w, xi[6], xi[7]);

    const double r[3] = {pos[o], pos[o + n], pos[o + 2 * n]};
    const double v[3] = {vel[o], vel[o + n], vel[o + 2 * n]};
    const double m[3] = {mom[o], mom[o + n], mom[o + 2 * n]};
    const double w[3] = {omega[o], omega[o + n], omega[o + 2 * n]};
    const double F[3] = {-dEdr[o] + Fsr[o], -dEdr[o + n] + Fsr[o + n], -dEdr[o + 2 * n] + Fsr[o + 2 * n]};
    const double He[3] = {-dEdm[o], -dEdm[o + n], -dEdm[o + 2 * n]};
    const double tq[3] = {m[1] * He[2] - m[2] * He[1], m[2] * He[0] - m[0] * He[2], m[0] * He[1] - m[1] * He[0]};
    const double at = sqrt(2.0 * c.gamma_t * c.kT * c.dt) / c.mass;
    const double ar = sqrt(2.0 * c.gamma_r * c.kT * c.dt) / c.inertia;
    double vn[3], rn[3], wn[3];
    for (int a = 0; a < 3; ++a) {
        vn[a] = v[a] + (c.dt / c.mass) * (F[a] - c.gamma_t * v[a]) + at * xi[a];
        rn[a] = r[a] + c.dt * v[a];
        wn[a] = w[a] + (c.dt / c.inertia) * (tq[a] - c.gamma_r * w[a]) + ar * xi[3 + a];
    }
    // rotate m by the angle |omega| dt about omega (Rodrigues), then renormalise
    double mn[3] = {m[0], m[1], m[2]};
    const double wl = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wl > 0.0) {
        const double u[3] = {w[0] / wl, w[1] / wl, w[2] / wl};
        const double ph = wl * c.dt, cs = cos(ph), sn = sin(ph);
        const double ud = u[0] * m[0] + u[1] * m[1] + u[2] * m[2];
        const double ux[3] = {u[1] * m[2] - u[2] * m[1], u[2] * m[0] - u[0] * m[2], u[0] * m[1] - u[1] * m[0]};
        for (int a = 0; a < 3; ++a) mn[a] = m[a] * cs + ux[a] * sn + u[a] * ud * (1.0 - cs);
    }
    const double ml = sqrt(mn[0] * mn[0] + mn[1] * mn[1] + mn[2] * mn[2]);
    for (int a = 0; a < 3; ++a) {
        pos[o + a * n] = rn[a];
        vel[o + a * n] = vn[a];
        omega[o + a * n] = wn[a];
        mom[o + a * n] = mn[a] / ml;
    }
}

// The step's last kernel: the device step counter, and the call counted out (call_leave).
__global__ void k_step_inc(uint64_t *d_step, uint32_t *status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *d_step += 1ull;
        call_leave(status);
    }
}

hipError_t launch_md(Handle &h, const md_state *st, const md_params *mp, hipStream_t s)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    // Two streams.  The caller's carries build -> fused traversal -> downward pass -> integrator.  The
    // side stream orders the traversal's items (from the costs of the previous step) beside the bounding
    // cube and the sort, and, as soon as the build has sorted the particles, puts the targets in Hilbert
    // order and computes the short-range forces beside the rest of the build (octree, levels, upward pass:
    // short, latency-bound launches).  The side stream rejoins the caller's
    // before the traversal, which therefore has the whole device.  The step starts after everything
    // enqueued on the caller's stream before it and is complete for everything enqueued after it; under
    // graph capture the fork and the join become edges.  Small systems, and handles without a side stream,
    // keep everything on one stream.
    hipError_t e;
    const bool fork = L.ntot >= kForkMinParticles && h.side != nullptr;  // a bh_init handle has no side stream
    const bool order = fork && uses_wave_order(h);  // else launch_backward orders the items itself
    if (order) {
        if ((e = hipEventRecord(h.fork_ev, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(h.side, h.fork_ev, 0)) != hipSuccess) return e;
        launch_order_waves(h, h.side);
    }
    // short-range forces from the sorted particles (on the side stream when forked)
    // sr_kind 0: WCA, pair and wall cut at the potential minimum; 1: the paper's form, walls at half the pair cut
    const double wca_rc = 1.122462048309373;  // 2^(1/6)
    const bool lj = mp->sr_kind == 1;
    const double c12 = lj ? 1.0 : 2.0;
    const double rc = lj ? (mp->sr_cut > 0.0 ? mp->sr_cut : 2.5 * mp->wca_sigma) : wca_rc * mp->wca_sigma;
    const double rcw = lj ? 0.5 * rc : wca_rc * 0.5 * mp->wca_sigma;
    const SortedWork short_range = [&](hipStream_t ss) {
        const int64_t ncell = L.B * L.cell_T;
        hipLaunchKernelGGL(k_clear_cells, dim3(grid_for(ncell, 256, 2048)), dim3(256), 0, ss, w.cells, ncell);
        hipLaunchKernelGGL(k_cell_fill, dim3(grid_for(L.ntot, 256)), dim3(256), 0, ss, w.codes, w.bbox, L.n,
                           L.ntot, rc, L.cell_lcap, L.cell_T, w.cells);
        hipLaunchKernelGGL(k_wca, dim3(grid_for(L.ntot, 256)), dim3(256), 0, ss, w.codes, w.bbox, w.cells, w.spos,
                           w.perm, w.md_force, L.n, L.ntot, L.cell_lcap, L.cell_T, mp->wca_sigma, mp->wca_eps, c12,
                           rc, rcw, make_double3(mp->box_lo[0], mp->box_lo[1], mp->box_lo[2]),
                           make_double3(mp->box_hi[0], mp->box_hi[1], mp->box_hi[2]));
        hipError_t e2 = hipGetLastError();
        if (e2 == hipSuccess && fork) e2 = hipEventRecord(h.join_ev, ss);
        return e2;
    };
    // tree, centroids, moment sums on the caller's stream; the target order and the short-range forces on
    // the side stream, enqueued right after the sort
    e = launch_build(h, st->pos, s, st->mom, fork ? h.side : nullptr, false, true, short_range);
    if (e != hipSuccess) return e;
    if (L.expansion == 2) {
        e = launch_upward_first_moments(h, s);  // order-2 cells
        if (e != hipSuccess) return e;
    }
    if (fork && (e = hipStreamWaitEvent(s, h.join_ev, 0)) != hipSuccess) return e;
    e = launch_backward(h, st->mom, mp->d_hext, nullptr, w.ones, w.md_grad_r, w.md_grad_m, nullptr, s, nullptr,
                        nullptr, true, order);
    if (e != hipSuccess) return e;
    MDConst c{mp->dt, mp->kT, mp->gamma_t, mp->gamma_r, mp->mass, mp->inertia, mp->seed};
    hipLaunchKernelGGL(k_integrate, dim3(grid_for(L.ntot, 256)), dim3(256), 0, s, st->pos, st->vel, st->mom,
                       st->omega, w.md_grad_r, w.md_grad_m, w.md_force, st->d_step, L.n, L.ntot, c);
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, st->d_step, w.status);
    return hipGetLastError();
}

}  // namespace ffbh
