// All-pairs dipolar field and force (the paper's all-pairs GPU step, Sec. 3.1 / Alg. 1): for every particle
// i of a system, H_i = sum_{j != i} T(r_i - r_j) m_j (Eq. H_dip) and, optionally, the all-pairs energy
// gradient dE/dr_i = -sum_{j != i} f_dip(r_i - r_j; m_i, m_j) (the f_dip summand of Sec. 2), with
// E = -1/2 sum m.H - sum m.H_ext.  It is the exact reference the Barnes-Hut path approximates, and the
// paper's AP column of Table 1.
//
// Layout: a workgroup of 256 threads owns 512 targets (two per thread, for two pairs per LDS read);
// sources pass through LDS in tiles of 256 records of 48 bytes (FP64 position, moment in T), read by
// every lane from the same address (broadcast).  Offsets are formed in FP64 and rounded to T, as in the
// tree path; the FP32-mixed mode sums each tile in FP32 and accumulates tiles in FP64.
#include "traverse.h"

namespace ffbh {

constexpr int kApThreads = 256;
constexpr int kApTile = 256;

template <typename T>
struct ApSrc;
template <>
struct ApSrc<float> {
    double x, y, z;
    float mx, my, mz, pad0;
    double pad1;
};
template <>
struct ApSrc<double> {
    double x, y, z, mx, my, mz;
};
static_assert(sizeof(ApSrc<float>) == 48 && sizeof(ApSrc<double>) == 48, "48-byte LDS source records");

template <bool MIXED, bool FORCE>
__global__ __launch_bounds__(kApThreads) void k_ap(const double *__restrict__ pos, const double *__restrict__ mom,
                                                   int64_t n, double *__restrict__ H, double *__restrict__ dEdr)
{
    using T = typename std::conditional<MIXED, float, double>::type;
    __shared__ ApSrc<T> tile[kApTile];
    const int64_t b = blockIdx.y;
    const double *p = pos + b * 3 * n;
    const double *m = mom + b * 3 * n;
    const int64_t i0 = (int64_t)blockIdx.x * 2 * kApThreads + threadIdx.x, i1 = i0 + kApThreads;
    const bool v0 = i0 < n, v1 = i1 < n;
    const int64_t c0 = v0 ? i0 : 0, c1 = v1 ? i1 : 0;
    const double ax = p[c0], ay = p[n + c0], az = p[2 * n + c0];
    const double bx = p[c1], by = p[n + c1], bz = p[2 * n + c1];
    const T am[3] = {(T)m[c0], (T)m[n + c0], (T)m[2 * n + c0]};
    const T bm[3] = {(T)m[c1], (T)m[n + c1], (T)m[2 * n + c1]};
    double ha[3] = {0.0, 0.0, 0.0}, hb[3] = {0.0, 0.0, 0.0};  // FP64 accumulation
    double ga[3] = {0.0, 0.0, 0.0}, gb[3] = {0.0, 0.0, 0.0};

    for (int64_t t0 = 0; t0 < n; t0 += kApTile) {
        const int64_t j = t0 + threadIdx.x;
        if (j < n) {
            ApSrc<T> r;
            r.x = p[j]; r.y = p[n + j]; r.z = p[2 * n + j];
            r.mx = (T)m[j]; r.my = (T)m[n + j]; r.mz = (T)m[2 * n + j];
            tile[threadIdx.x] = r;
        }
        __syncthreads();
        const int cnt = (int)(n - t0 < kApTile ? n - t0 : kApTile);
        T pha[3] = {0, 0, 0}, phb[3] = {0, 0, 0}, pga[3] = {0, 0, 0}, pgb[3] = {0, 0, 0};
        for (int k = 0; k < cnt; ++k) {
            const ApSrc<T> s = tile[k];
            const int64_t jk = t0 + k;
            {
                const T x = (T)(ax - s.x), y = (T)(ay - s.y), z = (T)(az - s.z);
                const bool use = v0 && jk != i0 && x * x + y * y + z * z > (T)0;
                if (FORCE) {
                    T gx, gy, gz, tx, ty, tz;
                    adj_field<T>(use, x, y, z, am[0], am[1], am[2], s.mx, s.my, s.mz, gx, gy, gz, tx, ty, tz,
                                 pha[0], pha[1], pha[2]);
                    pga[0] += gx; pga[1] += gy; pga[2] += gz;
                } else {
                    dip_acc<T>(use, x, y, z, s.mx, s.my, s.mz, pha[0], pha[1], pha[2]);
                }
            }
            {
                const T x = (T)(bx - s.x), y = (T)(by - s.y), z = (T)(bz - s.z);
                const bool use = v1 && jk != i1 && x * x + y * y + z * z > (T)0;
                if (FORCE) {
                    T gx, gy, gz, tx, ty, tz;
                    adj_field<T>(use, x, y, z, bm[0], bm[1], bm[2], s.mx, s.my, s.mz, gx, gy, gz, tx, ty, tz,
                                 phb[0], phb[1], phb[2]);
                    pgb[0] += gx; pgb[1] += gy; pgb[2] += gz;
                } else {
                    dip_acc<T>(use, x, y, z, s.mx, s.my, s.mz, phb[0], phb[1], phb[2]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ha[a] += (double)pha[a];
            hb[a] += (double)phb[a];
            ga[a] += (double)pga[a];
            gb[a] += (double)pgb[a];
        }
        __syncthreads();  // the tile is rewritten next
    }
    double *Ho = H + b * 3 * n;
    double *Go = dEdr ? dEdr + b * 3 * n : nullptr;
    if (v0) {
        Ho[i0] = ha[0]; Ho[n + i0] = ha[1]; Ho[2 * n + i0] = ha[2];
        if (FORCE && Go) {
            Go[i0] = -ga[0]; Go[n + i0] = -ga[1]; Go[2 * n + i0] = -ga[2];
        }
    }
    if (v1) {
        Ho[i1] = hb[0]; Ho[n + i1] = hb[1]; Ho[2 * n + i1] = hb[2];
        if (FORCE && Go) {
            Go[i1] = -gb[0]; Go[n + i1] = -gb[1]; Go[2 * n + i1] = -gb[2];
        }
    }
}

// E_b = -1/2 sum_i m_i.H_i - sum_i m_i.H_ext,b, one workgroup per system, in a fixed order.
__global__ __launch_bounds__(1024) void k_ap_energy(const double *__restrict__ mom, const double *__restrict__ H,
                                                    const double *__restrict__ hext, int64_t n,
                                                    double *__restrict__ E)
{
    __shared__ double red[1024];
    const int64_t b = blockIdx.x;
    const double *m = mom + b * 3 * n, *h = H + b * 3 * n;
    const double *he = hext ? hext + 3 * b : nullptr;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        double e = -0.5 * (m[i] * h[i] + m[n + i] * h[n + i] + m[2 * n + i] * h[2 * n + i]);
        if (he) e -= m[i] * he[0] + m[n + i] * he[1] + m[2 * n + i] * he[2];
        s += e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[b] = red[0];
}

hipError_t launch_ap(int64_t n, int32_t batch, int32_t precision, const double *pos, const double *mom,
                     const double *hext, double *H, double *dEdr, double *E, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 2 * kApThreads - 1) / (2 * kApThreads)), (unsigned)batch);
    const bool mixed = precision == BH_FP32_MIXED;
    if (dEdr) {
        if (mixed)
            hipLaunchKernelGGL((k_ap<true, true>), grid, dim3(kApThreads), 0, s, pos, mom, n, H, dEdr);
        else
            hipLaunchKernelGGL((k_ap<false, true>), grid, dim3(kApThreads), 0, s, pos, mom, n, H, dEdr);
    } else {
        if (mixed)
            hipLaunchKernelGGL((k_ap<true, false>), grid, dim3(kApThreads), 0, s, pos, mom, n, H, nullptr);
        else
            hipLaunchKernelGGL((k_ap<false, false>), grid, dim3(kApThreads), 0, s, pos, mom, n, H, nullptr);
    }
    if (E) hipLaunchKernelGGL(k_ap_energy, dim3((unsigned)batch), dim3(1024), 0, s, mom, H, hext, n, E);
    return hipGetLastError();
}

}  // namespace ffbh
