// Device building blocks shared by the forward and adjoint traversals (gfx950, wave64).
#pragma once

#include "ffbh_internal.h"

namespace ffbh {

// 1/sqrt(a) in FP64: the hardware estimate y (relative error about 2^-23) refined by one third-order
// step of the binomial series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - a y^2:
//   y <- y + y e (1/2 + 3e/8),
// whose truncation error 5e^3/16 (about 2^-70) is far below FP64 rounding; five operations where two
// Newton steps take eight.
__device__ inline double rsqrt64(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    const double t = a * y;
    const double e = __builtin_fma(-t, y, 1.0);
    const double p = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, p, y);
}

template <typename T>
__device__ inline T fmaT(T a, T b, T c);
template <>
__device__ inline double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <>
__device__ inline float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ inline T rsqT(T a);
template <>
__device__ inline double rsqT<double>(double a) { return rsqrt64(a); }
template <>
__device__ inline float rsqT<float>(float a) { return __builtin_amdgcn_rsqf(a); }

// Field of dipole m at offset x (target minus source), Eq. (H_dip) rearranged as
// h += (3 (m.x) x / |x|^2 - m) / |x|^3 when `use`; otherwise the inverse distance is replaced by zero
// and h receives exactly zero, so lanes of a wave that do not take part need no select on the result.
// r2 = |x|^2 comes from the caller (a far cell's is the acceptance test's FP64 distance, rounded once).
template <typename T>
__device__ inline void dip_acc_r2(bool use, T r2, T x, T y, T z, T mx, T my, T mz, T &hx, T &hy, T &hz)
{
    const T ri = use ? rsqT<T>(r2) : (T)0;
    const T ri2 = ri * ri;
    const T ri3 = ri2 * ri;
    const T md = fmaT<T>(mz, z, fmaT<T>(my, y, mx * x));
    const T t = (T)3 * md * ri2;
    hx = fmaT<T>(fmaT<T>(t, x, -mx), ri3, hx);
    hy = fmaT<T>(fmaT<T>(t, y, -my), ri3, hy);
    hz = fmaT<T>(fmaT<T>(t, z, -mz), ri3, hz);
}

template <typename T>
__device__ inline T norm2(T x, T y, T z) { return fmaT<T>(z, z, fmaT<T>(y, y, x * x)); }

template <typename T>
__device__ inline void dip_acc(bool use, T x, T y, T z, T mx, T my, T mz, T &hx, T &hy, T &hz)
{
    dip_acc_r2<T>(use, norm2<T>(x, y, z), x, y, z, mx, my, mz, hx, hy, hz);
}

// Field of a cell's first moment D (row-major, D[3k+b] = sum_j (r_j - c)_k m_j,b) at offset x from the
// cell's centre c: the next term of the Taylor expansion of Eq. H_dip about c,
//   h = -3 (D x + D^T x + x tr D) / |x|^5 + 15 (x.D x) x / |x|^7 .
// When `use` is false the inverse distance is zero and the increment is exactly zero.  r2 = |x|^2 comes
// from the caller (see dip_acc_r2).
template <typename T>
__device__ inline void first_moment_acc_r2(bool use, T r2, T x, T y, T z, const T *D, T &hx, T &hy, T &hz)
{
    const T ri = use ? rsqT<T>(r2) : (T)0;
    const T ri2 = ri * ri;
    const T ri5 = ri2 * ri2 * ri;
    const T u0 = fmaT<T>(D[2], z, fmaT<T>(D[1], y, D[0] * x));
    const T u1 = fmaT<T>(D[5], z, fmaT<T>(D[4], y, D[3] * x));
    const T u2 = fmaT<T>(D[8], z, fmaT<T>(D[7], y, D[6] * x));
    const T w0 = fmaT<T>(D[6], z, fmaT<T>(D[3], y, D[0] * x));
    const T w1 = fmaT<T>(D[7], z, fmaT<T>(D[4], y, D[1] * x));
    const T w2 = fmaT<T>(D[8], z, fmaT<T>(D[5], y, D[2] * x));
    const T tr = D[0] + D[4] + D[8];
    const T qd = fmaT<T>(z, u2, fmaT<T>(y, u1, x * u0));
    const T s = (T)15 * qd * ri2;
    hx = fmaT<T>(fmaT<T>(s, x, (T)-3 * (u0 + w0 + x * tr)), ri5, hx);
    hy = fmaT<T>(fmaT<T>(s, y, (T)-3 * (u1 + w1 + y * tr)), ri5, hy);
    hz = fmaT<T>(fmaT<T>(s, z, (T)-3 * (u2 + w2 + z * tr)), ri5, hz);
}

// Adjoint of the first-moment term for the target's upstream field gradient u: with phi = 1/|x|, the
// term is h_D,a = -sum D_kb d_a d_b d_k phi, and for u . h_D
//   G = d(u.h_D)/dx = -[105 (u.x) q x / r^9 - 15 (x (x.Du + u.Dx + (u.x) tr D) + u q + (u.x)(Dx + D^T x)) / r^7
//                       + 3 (Du + D^T u + u tr D) / r^5]              (q = x.Dx; target gather, centre -G)
//   E = d(u.h_D)/dD = -[3 (x u^T + u x^T + (u.x) I) / r^5 - 15 (u.x) x x^T / r^7]    (symmetric)
// E is returned as (xx, yy, zz, xy, xz, yz).  When `use` is false every output is exactly zero.
template <typename T>
__device__ inline void first_moment_adj_r2(bool use, T r2, T x, T y, T z, const T *D, T ux, T uy, T uz, T &gx,
                                           T &gy, T &gz, T &e0, T &e1, T &e2, T &e3, T &e4, T &e5)
{
    const T ri = use ? rsqT<T>(r2) : (T)0;
    const T ri2 = ri * ri;
    const T ri5 = ri2 * ri2 * ri, ri7 = ri5 * ri2, ri9 = ri7 * ri2;
    const T p0 = fmaT<T>(D[2], z, fmaT<T>(D[1], y, D[0] * x));   // D x
    const T p1 = fmaT<T>(D[5], z, fmaT<T>(D[4], y, D[3] * x));
    const T p2 = fmaT<T>(D[8], z, fmaT<T>(D[7], y, D[6] * x));
    const T w0 = fmaT<T>(D[6], z, fmaT<T>(D[3], y, D[0] * x));   // D^T x
    const T w1 = fmaT<T>(D[7], z, fmaT<T>(D[4], y, D[1] * x));
    const T w2 = fmaT<T>(D[8], z, fmaT<T>(D[5], y, D[2] * x));
    const T d0 = fmaT<T>(D[2], uz, fmaT<T>(D[1], uy, D[0] * ux));  // D u
    const T d1 = fmaT<T>(D[5], uz, fmaT<T>(D[4], uy, D[3] * ux));
    const T d2 = fmaT<T>(D[8], uz, fmaT<T>(D[7], uy, D[6] * ux));
    const T t0 = fmaT<T>(D[6], uz, fmaT<T>(D[3], uy, D[0] * ux));  // D^T u
    const T t1 = fmaT<T>(D[7], uz, fmaT<T>(D[4], uy, D[1] * ux));
    const T t2 = fmaT<T>(D[8], uz, fmaT<T>(D[5], uy, D[2] * ux));
    const T tr = D[0] + D[4] + D[8];
    const T q = fmaT<T>(z, p2, fmaT<T>(y, p1, x * p0));
    const T ud = fmaT<T>(uz, z, fmaT<T>(uy, y, ux * x));            // u.x
    const T uDx = fmaT<T>(uz, p2, fmaT<T>(uy, p1, ux * p0));
    const T xDu = fmaT<T>(z, d2, fmaT<T>(y, d1, x * d0));
    const T c9 = (T)105 * ud * q * ri9, c7 = (T)15 * ri7, c5 = (T)3 * ri5;
    const T sx = xDu + uDx + ud * tr;
    gx = -(c9 * x - c7 * (x * sx + ux * q + ud * (w0 + p0)) + c5 * (d0 + t0 + ux * tr));
    gy = -(c9 * y - c7 * (y * sx + uy * q + ud * (w1 + p1)) + c5 * (d1 + t1 + uy * tr));
    gz = -(c9 * z - c7 * (z * sx + uz * q + ud * (w2 + p2)) + c5 * (d2 + t2 + uz * tr));
    const T f = c7 * ud;
    e0 = -(c5 * ((T)2 * ux * x + ud) - f * x * x);
    e1 = -(c5 * ((T)2 * uy * y + ud) - f * y * y);
    e2 = -(c5 * ((T)2 * uz * z + ud) - f * z * z);
    e3 = -(c5 * (uy * x + ux * y) - f * x * y);
    e4 = -(c5 * (uz * x + ux * z) - f * x * z);
    e5 = -(c5 * (uz * y + uy * z) - f * y * z);
}

// Adjoint pair plus the forward field.  With a = upstream field gradient of the target, b = source
// moment, x = offset (target minus source):
//   g  = 3 [ (a.b) x + (b.x) a + (a.x) b ] / |x|^5 - 15 (a.x)(b.x) x / |x|^7   (f_dip summand, Sec. 2)
//      = 3 |x|^-5 [ (a.b - 5 (a.x)(b.x) / |x|^2) x + (b.x) a + (a.x) b ]
//   t  = T(x) a = (3 (a.x) x / |x|^2 - a) / |x|^3                                (T symmetric)
//   h += T(x) b, the field of dipole b at x (Eq. H_dip),
// sharing the distance powers and dot products.  When `use` is false the inverse distance is zero and
// g, t and the increment of h are exactly zero.
// r2 = |x|^2 comes from the caller (see dip_acc_r2).  With ACC, g is also added to ug[0..2] as s w + ug
// with one FMA per component, where g = s w (g itself is then only read by the caller's wave reduction,
// which may overwrite it in place).
template <typename T, bool ACC = false>
__device__ inline void adj_field_r2(bool use, T r2, T x, T y, T z, T ax, T ay, T az, T bx, T by, T bz, T &gx,
                                    T &gy, T &gz, T &tx, T &ty, T &tz, T &hx, T &hy, T &hz, T *ug = nullptr)
{
    const T ri = use ? rsqT<T>(r2) : (T)0;
    const T ri2 = ri * ri;
    const T ri3 = ri2 * ri;
    const T k3 = (T)3 * ri2;  // shared by 3/|x|^5 and both 3 (.x)/|x|^2 factors
    const T adx = fmaT<T>(az, z, fmaT<T>(ay, y, ax * x));
    const T bdx = fmaT<T>(bz, z, fmaT<T>(by, y, bx * x));
    const T ab = fmaT<T>(az, bz, fmaT<T>(ay, by, ax * bx));
    const T c0 = fmaT<T>((T)-5 * adx * bdx, ri2, ab);
    const T s = k3 * ri3;
    const T wx = fmaT<T>(c0, x, fmaT<T>(bdx, ax, adx * bx));
    const T wy = fmaT<T>(c0, y, fmaT<T>(bdx, ay, adx * by));
    const T wz = fmaT<T>(c0, z, fmaT<T>(bdx, az, adx * bz));
    gx = s * wx;
    gy = s * wy;
    gz = s * wz;
    if constexpr (ACC) {
        ug[0] = fmaT<T>(s, wx, ug[0]);
        ug[1] = fmaT<T>(s, wy, ug[1]);
        ug[2] = fmaT<T>(s, wz, ug[2]);
    }
    const T ta = adx * k3;
    tx = fmaT<T>(ta, x, -ax) * ri3;
    ty = fmaT<T>(ta, y, -ay) * ri3;
    tz = fmaT<T>(ta, z, -az) * ri3;
    const T tb = bdx * k3;
    hx = fmaT<T>(fmaT<T>(tb, x, -bx), ri3, hx);
    hy = fmaT<T>(fmaT<T>(tb, y, -by), ri3, hy);
    hz = fmaT<T>(fmaT<T>(tb, z, -bz), ri3, hz);
}

template <typename T>
__device__ inline void adj_field(bool use, T x, T y, T z, T ax, T ay, T az, T bx, T by, T bz, T &gx, T &gy,
                                 T &gz, T &tx, T &ty, T &tz, T &hx, T &hy, T &hz)
{
    adj_field_r2<T>(use, norm2<T>(x, y, z), x, y, z, ax, ay, az, bx, by, bz, gx, gy, gz, tx, ty, tz, hx, hy, hz);
}

// ---- wave64 reductions (DPP) ---------------------------------------------------------------------

template <int CTRL>
__device__ inline float dpp_f(float v)
{
    // bound_ctrl: lanes whose source is out of range read 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Sum of v over all 64 lanes, returned uniformly (must be called with every lane active).
__device__ inline float wave_sum(float v)
{
    v += dpp_f<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);  // row_half_mirror
    v += dpp_f<0x140>(v);  // row_mirror: every lane of a row now holds the row's sum
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (a + b) + (c + d);
}

// Sum over all 64 lanes, left in lane 63 only (other lanes hold partial sums); every lane active.
// Rows are reduced with quad/half-row/row mirrors, then rows 1 and 3 add the row before them
// (row_bcast:15) and rows 2 and 3 add lane 31 (row_bcast:31).
__device__ inline float wave_sum_to63(float v)
{
    v += dpp_f<0xb1>(v);
    v += dpp_f<0x4e>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));
    return v;
}

template <int CTRL>
__device__ inline double dpp_d(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffff), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

__device__ inline double readlane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

__device__ inline double wave_sum_to63(double v)
{
    v += dpp_d<0xb1>(v);
    v += dpp_d<0x4e>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    const long long bits = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffff), 0x142, 0xa, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), 0x142, 0xa, 0xf, false);
    v += __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
    const long long bits2 = __double_as_longlong(v);
    lo = __builtin_amdgcn_update_dpp(0, (int)(bits2 & 0xffffffff), 0x143, 0xc, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(bits2 >> 32), 0x143, 0xc, 0xf, false);
    v += __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
    return v;
}

__device__ inline float readlane_t(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double readlane_t(double v, int lane) { return readlane_d(v, lane); }

__device__ inline double wave_sum(double v)
{
    v += dpp_d<0xb1>(v);
    v += dpp_d<0x4e>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    const double a = readlane_d(v, 0), b = readlane_d(v, 16), c = readlane_d(v, 32), d = readlane_d(v, 48);
    return (a + b) + (c + d);
}

// Sum over the two lanes l and l ^ 16 (permlane16_swap) or l and l ^ 32 (permlane32_swap): the swap of
// a register with itself hands every lane the value of its partner row in the second result.
__device__ inline float swap16_sum(float v)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float swap32_sum(float v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline double swap16_sum(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}
__device__ inline double swap32_sum(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}
template <int CTRL>
__device__ inline float dpp_t(float v) { return dpp_f<CTRL>(v); }
template <int CTRL>
__device__ inline double dpp_t(double v) { return dpp_d<CTRL>(v); }

// One exchange step of a transposed reduction: the two lanes paired by DPP control CTRL each keep one of
// two values (the lane with `hi` keeps u, its partner l) and add the partner's copy of it.
template <int CTRL, typename T>
__device__ inline T xkeep(bool hi, T l, T u)
{
    const T keep = hi ? u : l, give = hi ? l : u;
    return keep + dpp_t<CTRL>(give);
}

// Row exchanges of two different values in one instruction.  permlane32_swap(a, b) leaves lanes 0..31 of
// one result and of the other holding the two halves of a, and lanes 32..63 the two halves of b, so the
// sum of the results is a + (a from lane l ^ 32) in lanes 0..31 and the same for b in lanes 32..63.
// permlane16_swap(a, b) does the same with rows: rows 0 and 2 sum a with the row above or below (l ^ 16),
// rows 1 and 3 sum b.
__device__ inline float swap32_pair(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float swap16_pair(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline double swap32_pair(double a, double b)
{
    const uint64_t x = (uint64_t)__double_as_longlong(a), y = (uint64_t)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)y, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}
__device__ inline double swap16_pair(double a, double b)
{
    const uint64_t x = (uint64_t)__double_as_longlong(a), y = (uint64_t)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)x, (uint32_t)y, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(x >> 32), (uint32_t)(y >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}

// Wave totals of six per-lane values (all 64 lanes active).  The row exchanges come first and move two
// values each: after the 32-lane swaps lanes 0..31 carry v0, v2, v4 and lanes 32..63 carry v1, v3, v5;
// after the 16-lane swaps rows 0..3 carry v0, v2, v1, v3 in one register and rows 0, 1 / 2, 3 carry v4 / v5
// in another.  Inside each row one exchange step over l ^ 8 keeps the first register in lanes 0..7 and the
// second in lanes 8..15, and three DPP additions finish the eight-lane groups.  The total of value c is
// then held by lane total6_lane(c): 0, 32, 16, 48, 8, 40 for c = 0..5.
template <typename T>
__device__ inline T wave_total6(int lane, T v0, T v1, T v2, T v3, T v4, T v5)
{
    const T w0 = swap32_pair(v0, v1), w1 = swap32_pair(v2, v3), w2 = swap32_pair(v4, v5);
    const T x0 = swap16_pair(w0, w1), x1 = swap16_sum(w2);
    T y = xkeep<0x128>((lane & 8) != 0, x0, x1);  // row_ror 8 pairs l and l ^ 8
    y += dpp_t<0x141>(y);
    y += dpp_t<0x4e>(y);
    return y + dpp_t<0xb1>(y);
}
// Which of the six totals this lane holds for writing (-1: none).
__device__ inline int total6_comp(int lane)
{
    if ((lane & 7) != 0) return -1;
    const int row = lane >> 4;
    if (lane & 8) return (row & 1) ? -1 : 4 + (row >> 1);
    return row == 0 ? 0 : row == 1 ? 2 : row == 2 ? 1 : 3;
}

// ---- compacted direct sums (leaf cells) -----------------------------------------------------------
//
// At a leaf, only the lanes that opened it (typically about a sixth of the wave) have pairs to sum.  The
// opening lanes are listed in LDS and the pairs are packed densely: the wave is cut into groups of G lanes
// (G = 4, 8 or 16, the smallest that holds the leaf's members, larger leaves in chunks of 16), lane b of
// group g takes member b against listed target t0 + g, so one pass covers 64 / G targets.  Per-target sums
// are group reductions added to the target's LDS slot; the owner lane collects them after the leaf.

// Sum of three values over each aligned group of G lanes.  Returns the group total of value
// group3_slot<G>(lane) (3 means none).
template <int G>
__device__ inline int group3_slot(int lane)
{
    return G == 4 ? (lane & 3) : ((lane >> 1) & 3);
}
// The lane that writes the group's total of its slot (one per slot and group).
template <int G>
__device__ inline bool group3_writer(int lane)
{
    return G == 4 ? true : G == 8 ? (lane & 1) == 0 : (lane & 9) == 0;
}
template <int G, typename T>
__device__ inline T group_sum3(int lane, T v0, T v1, T v2)
{
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    if constexpr (G == 4) {
        const T a0 = xkeep<0x4e>(b1, v0, v2), a1 = xkeep<0x4e>(b1, v1, (T)0);  // partner i ^ 2
        return xkeep<0xb1>(b0, a0, a1);                                         // partner i ^ 1
    } else {
        const T a0 = xkeep<0x141>(b2, v0, v2), a1 = xkeep<0x141>(b2, v1, (T)0);  // partner 7 - i
        T r = xkeep<0x4e>(b1, a0, a1);                                           // slot 2 b2 + b1
        r += dpp_t<0xb1>(r);                                                     // i and i ^ 1 hold it
        if constexpr (G == 16) r += dpp_t<0x128>(r);                             // row_ror 8: both halves
        return r;
    }
}

// Sum of six values over each aligned group of G lanes (slots 6, 7 are zero).  G = 8, 16: one value per
// lane, slot (lane & 7).  G = 4: two values per lane, slots 2 (lane & 3) and 2 (lane & 3) + 1.
template <int G, typename T>
__device__ inline void group_sum6(int lane, T v0, T v1, T v2, T v3, T v4, T v5, T &o0, T &o1)
{
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    if constexpr (G == 4) {
        const T k0 = xkeep<0x4e>(b1, v0, v4), k1 = xkeep<0x4e>(b1, v1, v5);
        const T k2 = xkeep<0x4e>(b1, v2, (T)0), k3 = xkeep<0x4e>(b1, v3, (T)0);  // slots 4 b1 + j
        o0 = xkeep<0xb1>(b0, k0, k2);
        o1 = xkeep<0xb1>(b0, k1, k3);
    } else {
        const T k0 = xkeep<0x141>(b2, v0, v4), k1 = xkeep<0x141>(b2, v1, v5);
        const T k2 = xkeep<0x141>(b2, v2, (T)0), k3 = xkeep<0x141>(b2, v3, (T)0);
        const T u0 = xkeep<0x4e>(b1, k0, k2), u1 = xkeep<0x4e>(b1, k1, k3);
        T z = xkeep<0xb1>(b0, u0, u1);
        if constexpr (G == 16) z += dpp_t<0x128>(z);
        o0 = z;
        o1 = (T)0;
    }
}

// Sum over the lanes of a row with equal (lane mod G), returned in every lane of the row: rotations
// inside the row.
template <int G, typename T>
__device__ inline T row_stride_sum(T v)
{
    if constexpr (G == 4) v += dpp_t<0x124>(v);  // row_ror 4
    if constexpr (G <= 8) v += dpp_t<0x128>(v);  // row_ror 8
    return v;
}

// Lane mask of a lane condition (the condition is already a mask; no conversion through an integer).
__device__ inline uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// This lane's bit of a wave-uniform lane mask, as a lane condition (the mask is used as the condition
// directly, without per-lane shifts).
__device__ inline bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Number of set bits of m below this lane.
__device__ inline int lanes_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Orders this wave's LDS accesses around a cross-lane exchange (DS instructions of one wave execute in
// order; this keeps the compiler from moving accesses across the exchange).
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline void lds_add(T *p, T v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Target of a lane, as the compacted direct sums read it.
struct LdsTarget {
    double rx, ry, rz;
    int si, pad;
};

// Sorted position of target `local` of system seg: entry seg n + local of the target order, or seg n + local
// without one.  Lanes past the system's end take its first particle (they only read it).
__device__ inline int target_of(const uint32_t *__restrict__ order, int seg, int64_t n, int local, bool valid)
{
    const int base = (int)(seg * n);
    if (!valid) return base;
    if (!order) return base + local;
    const uint32_t o = order[base + local];
    return (o - (uint32_t)base) < (uint32_t)n ? (int)o : base + local;  // always in range for a consistent order
}

extern __shared__ __align__(16) unsigned char ffbh_dyn_lds[];

// Logical block index, arranged so that each of the 8 XCDs (which receive workgroups round-robin)
// works on one contiguous range of the target order and keeps those nodes in its own L2.
__device__ inline int xcd_block(int bid, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = bid & 7, k = bid >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Depth-first stack of node ranges for one wave.  The range being walked is held in scalar registers (next
// node, nodes left, lane mask), so taking the next node costs no vector instructions; the ranges below it
// are held one per lane (entry e in lane e: first node | (count - 1) << 28 and the 64-bit mask) and are
// read back with v_readlane when the walked range runs out.  A push first parks the rest of the walked
// range in the next lane, so nodes are visited in the same order as with a plain stack of ranges.
struct LaneStack {
    int ent, mlo, mhi;  // parked ranges, entry `lane` in this lane
    int sp;             // number of parked ranges
    int tnode, tleft;   // walked range: next node and nodes left
    uint64_t tmask;     // walked range: lane mask

    // Start with one range; first and count must be wave-uniform (read from lane 0 so that the compiler
    // can keep the walked range, and the node loads that depend on it, scalar).
    __device__ inline void init(int first, int count, uint64_t m)
    {
        ent = mlo = mhi = 0;
        sp = 0;
        tnode = __builtin_amdgcn_readfirstlane(first);
        tleft = __builtin_amdgcn_readfirstlane(count);
        tmask = m;
    }
    // Two ways to walk.  pop: the walked range is refilled from the parked ones when a take finds it
    // empty (loop test more_any).  pop_settled: the caller refills it at the end of each visit (settle),
    // so it is empty only when the walk is over, and the loop test (more) and the take are one compare and
    // three increments; the forward walk, whose scalar issue is as busy as its vector issue, uses this
    // one.  Both visit the nodes in the same order.
    __device__ inline bool more() const { return tleft > 0; }
    __device__ inline bool more_any() const { return tleft > 0 || sp > 0; }
    // Drop every range: the walk ends at the next more() (error exits, without a second loop exit).
    __device__ inline void clear()
    {
        sp = 0;
        tleft = 0;
    }
    __device__ inline void push(int lane, int first, int count, uint64_t m)
    {
        if (tleft > 0) {
            const bool here = lane == sp;
            ent = here ? (tnode | ((tleft - 1) << 28)) : ent;
            mlo = here ? (int)(uint32_t)tmask : mlo;
            mhi = here ? (int)(uint32_t)(tmask >> 32) : mhi;
            ++sp;
        }
        tnode = first;
        tleft = count;
        tmask = m;
    }
    // Next node and its lane mask (call only while more(), with settle() at the end of every visit).
    __device__ inline int pop_settled(uint64_t &m)
    {
        m = tmask;
        --tleft;
        return tnode++;
    }
    // Next node and its lane mask (call only while more_any(), so a range is parked when the walked one
    // is empty).  The refill is written out here and in settle() rather than shared: each walk's register
    // allocation (measured) depends on it.
    __device__ inline int pop(uint64_t &m)
    {
        if (tleft == 0) {
            --sp;
            const uint32_t e = (uint32_t)__builtin_amdgcn_readlane(ent, sp);
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(mlo, sp);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(mhi, sp);
            tnode = (int)(e & 0x0fffffffu);
            tleft = (int)(e >> 28) + 1;
            tmask = ((uint64_t)hi << 32) | lo;
        }
        return pop_settled(m);
    }
    // End of a visit: if the walked range has run out, the top parked range becomes the walked one.
    __device__ inline void settle()
    {
        if (tleft == 0 && sp > 0) {
            --sp;
            const uint32_t e = (uint32_t)__builtin_amdgcn_readlane(ent, sp);
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(mlo, sp);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(mhi, sp);
            tnode = (int)(e & 0x0fffffffu);
            tleft = (int)(e >> 28) + 1;
            tmask = ((uint64_t)hi << 32) | lo;
        }
    }
};

// Sorted source particle for the direct sums: position FP64, moment FP64 (Src64) or FP32 (Src32),
// 48 bytes so that one particle is two scalar loads from one address.
struct Src64 {
    double x, y, z, mx, my, mz;
};
struct Src32 {
    double x, y, z;
    float mx, my, mz, pad;
    double pad2;
};
static_assert(sizeof(Src64) == 48 && sizeof(Src32) == 48, "source records are 48 bytes");

}  // namespace ffbh
