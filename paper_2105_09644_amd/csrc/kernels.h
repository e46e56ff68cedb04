// Device-side pieces of the TreeRay sweep: HEALPix pixelisation, the radial
// kernels and wave-level helpers.  Included by the kernel translation unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tr {

constexpr double kPi = 3.14159265358979323846;

// Fixed shift of the angular sub-point lattice, as fractions of a sub-box
// (breaks exact ties between sub-points and pixel edges on regular grids).
constexpr double kJit0 = 4.1e-4, kJit1 = 7.3e-4, kJit2 = 2.3e-4;

// ---------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum over the 64 lanes with DPP: an inclusive scan inside each row of 16
// lanes (row_shr 1, 2, 4, 8), then row broadcasts of lanes 15 and 31; lane
// 63 ends with the total, which is broadcast.
__device__ inline int dpp_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false); }
__device__ inline int dpp_shr2(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false); }
__device__ inline int dpp_shr4(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false); }
__device__ inline int dpp_shr8(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false); }
__device__ inline int dpp_bc15(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false); }
__device__ inline int dpp_bc31(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false); }

__device__ inline float wave_sum(float v)
{
    v += __int_as_float(dpp_shr1(__float_as_int(v)));
    v += __int_as_float(dpp_shr2(__float_as_int(v)));
    v += __int_as_float(dpp_shr4(__float_as_int(v)));
    v += __int_as_float(dpp_shr8(__float_as_int(v)));
    v += __int_as_float(dpp_bc15(__float_as_int(v)));
    v += __int_as_float(dpp_bc31(__float_as_int(v)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ inline double dpp_d(double v, int which)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int a, b;
    switch (which) {
        case 1: a = dpp_shr1(lo); b = dpp_shr1(hi); break;
        case 2: a = dpp_shr2(lo); b = dpp_shr2(hi); break;
        case 4: a = dpp_shr4(lo); b = dpp_shr4(hi); break;
        case 8: a = dpp_shr8(lo); b = dpp_shr8(hi); break;
        case 15: a = dpp_bc15(lo); b = dpp_bc15(hi); break;
        default: a = dpp_bc31(lo); b = dpp_bc31(hi); break;
    }
    return __hiloint2double(b, a);
}

__device__ inline double wave_sum(double v)
{
    v += dpp_d(v, 1);
    v += dpp_d(v, 2);
    v += dpp_d(v, 4);
    v += dpp_d(v, 8);
    v += dpp_d(v, 15);
    v += dpp_d(v, 31);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G lanes (G = 4, 8, 16, 32 or 64, uniform) with
// every lane of a group ending with the same bits: lane swaps inside quads
// ([1,0,3,2], [2,3,0,1]), then the mirror inside 8 and inside 16 lanes; each
// step adds two partial sums in either order, and addition commutes.  Groups
// of 32 or 64 lanes then add the sums of their rows of 16, read from the
// rows' first lanes into scalars.  Call with every lane active.
template <int CTRL>
__device__ inline double dpp_swap_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double read_lane_d(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ inline double group_sum(double v, int G)
{
    v += dpp_swap_d<0xB1>(v);
    v += dpp_swap_d<0x4E>(v);
    if (G >= 8) v += dpp_swap_d<0x141>(v);
    if (G >= 16) v += dpp_swap_d<0x140>(v);
    if (G >= 32) {
        const double h0 = read_lane_d(v, 0) + read_lane_d(v, 16);
        const double h1 = read_lane_d(v, 32) + read_lane_d(v, 48);
        v = G == 64 ? h0 + h1 : (lane_id() < 32 ? h0 : h1);
    }
    return v;
}

// The same in FP32 (one DPP move per step).
template <int CTRL>
__device__ inline float dpp_swap_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ inline float read_lane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ inline float group_sum(float v, int G)
{
    v += dpp_swap_f<0xB1>(v);
    v += dpp_swap_f<0x4E>(v);
    if (G >= 8) v += dpp_swap_f<0x141>(v);
    if (G >= 16) v += dpp_swap_f<0x140>(v);
    if (G >= 32) {
        const float h0 = read_lane_f(v, 0) + read_lane_f(v, 16);
        const float h1 = read_lane_f(v, 32) + read_lane_f(v, 48);
        v = G == 64 ? h0 + h1 : (lane_id() < 32 ? h0 : h1);
    }
    return v;
}

// s + e = a + b exactly (Knuth's TwoSum, round to nearest)
__device__ inline void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bv = s - a;
    e = (a - (s - bv)) + (b - bv);
}

// Compensated group sum of (hi, lo) pairs: at each butterfly step the two
// partial sums are added with their rounding error carried in lo; every
// lane of a group ends with the same bits (each step adds the same two
// values in either order, and both TwoSum and addition are commutative).
template <int CTRL>
__device__ inline void csum_step(float &hi, float &lo)
{
    const float oh = dpp_swap_f<CTRL>(hi), ol = dpp_swap_f<CTRL>(lo);
    float s, e;
    two_sum(hi, oh, s, e);
    hi = s;
    lo = (lo + ol) + e;
}

__device__ inline void group_csum(float &hi, float &lo, int G)
{
    csum_step<0xB1>(hi, lo);
    csum_step<0x4E>(hi, lo);
    if (G >= 8) csum_step<0x141>(hi, lo);
    if (G >= 16) csum_step<0x140>(hi, lo);
    if (G >= 32) {
        // the rows' pairs, added pairwise with the same compensation
        float h[2], l[2];
        for (int q = 0; q < 2; ++q) {
            float s, e;
            two_sum(read_lane_f(hi, 32 * q), read_lane_f(hi, 32 * q + 16), s, e);
            h[q] = s;
            l[q] = (read_lane_f(lo, 32 * q) + read_lane_f(lo, 32 * q + 16)) + e;
        }
        if (G == 64) {
            float s, e;
            two_sum(h[0], h[1], s, e);
            hi = s;
            lo = (l[0] + l[1]) + e;
        } else {
            const bool first = lane_id() < 32;
            hi = first ? h[0] : h[1];
            lo = first ? l[0] : l[1];
        }
    }
}

// Position of the n-th (from 0) set bit of m; n < popcount(m).  A binary
// search on the popcounts of the low halves.
__device__ inline int nth_set_bit(uint64_t m, int n)
{
    uint32_t w = (uint32_t)m;
    int pos = 0, c = __popc(w);
    if (n >= c) {
        n -= c;
        w = (uint32_t)(m >> 32);
        pos = 32;
    }
#pragma unroll
    for (int b = 16; b >= 1; b >>= 1) {
        c = __popc(w & ((1u << b) - 1u));
        if (n >= c) {
            n -= c;
            w >>= b;
            pos += b;
        }
    }
    return pos;
}

// Largest value over the 64 lanes (values >= 0), the same on every lane.
__device__ inline int wave_max_nonneg(int v)
{
    v = max(v, dpp_shr1(v));
    v = max(v, dpp_shr2(v));
    v = max(v, dpp_shr4(v));
    v = max(v, dpp_shr8(v));
    v = max(v, dpp_bc15(v));
    v = max(v, dpp_bc31(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Exclusive prefix sum over the 64 lanes with DPP (no LDS): an inclusive
// scan inside each row of 16 (row_shr 1, 2, 4, 8 with zeros shifted in), then
// the row totals carried by the row broadcasts of lanes 15 and 31.
__device__ inline int wave_excl_scan_dpp(int v, int &total)
{
    int x = v;
    x += dpp_shr1(x);
    x += dpp_shr2(x);
    x += dpp_shr4(x);
    x += dpp_shr8(x);
    x += dpp_bc15(x);
    x += dpp_bc31(x);
    total = __builtin_amdgcn_readlane(x, 63);
    return x - v;
}

// ---------------------------------------------------------------------------
// HEALPix RING pixel of a direction (Gorski et al. 2005).  Equatorial zone
// |z| <= 2/3: the pixel edges are the lines of constant
// a = N(1/2 + t - 3z/4) and b = N(1/2 + t + 3z/4), t = phi/(pi/2).  Polar
// caps: edges of constant t' sig and (1 - t') sig, t' = frac(t),
// sig = N sqrt(3 (1 - |z|)), with 1 - |z| = rho^2 / (r (r + |z|)).
// ---------------------------------------------------------------------------
__device__ inline int pix_equatorial(int ns, int jp, int jm)
{
    int ir = ns + 1 + jp - jm;                  // ring counted from z = 2/3
    // rounding at |z| = 2/3 can put the edge indices one ring outside the zone
    ir = ir < 1 ? 1 : (ir > 2 * ns + 1 ? 2 * ns + 1 : ir);
    const int kshift = 1 - (ir & 1);
    // floor division by 2; jp, jm lie in [0, 5 ns], so ip is in
    // [-ns/2, 4.5 ns + 1] and wraps at most once
    int ip = (jp + jm - ns + kshift + 1) >> 1;
    const int m = 4 * ns;
    ip = ip >= m ? ip - m : (ip < 0 ? ip + m : ip);
    return 2 * ns * (ns - 1) + (ir - 1) * m + ip;
}

__device__ inline int pix_polar(int ns, int ir, int ipf, bool north)
{
    // ipf = floor(t ir) with t in [0, 4]: wraps at most once
    const int m = 4 * ir;
    const int ip = ipf >= m ? ipf - m : (ipf < 0 ? ipf + m : ipf);
    return north ? 2 * ir * (ir - 1) + ip : 12 * ns * ns - 2 * ir * (ir + 1) + ip;
}

// FP64 form with correctly rounded operations and no contraction, so that a
// direction gives the same pixel as any other FP64 evaluation of the same
// formulas (the only inexact library call is atan2).
__device__ __attribute__((noinline)) int ang2pix_d(int ns, double x, double y, double z)
{
#pragma clang fp contract(off)
    const double rho2 = x * x + y * y;
    const double r = __dsqrt_rn(rho2 + z * z);
    const double zc = z / r;
    const double za = fabs(zc);
    double phi = atan2(y, x);
    if (phi < 0) phi = phi + 2.0 * kPi;
    const double t = phi / (0.5 * kPi);
    if (za <= 2.0 / 3.0) {
        const double a = (double)ns * ((0.5 + t) - 0.75 * zc);
        const double b = (double)ns * ((0.5 + t) + 0.75 * zc);
        return pix_equatorial(ns, (int)floor(a), (int)floor(b));
    }
    const double tp = t - floor(t);
    const double omz = rho2 / (r * (r + fabs(z)));
    const double sig = (double)ns * __dsqrt_rn(3.0 * omz);
    const int jp = (int)floor(tp * sig);
    const int jm = (int)floor((1.0 - tp) * sig);
    const int ir = jp + jm + 1;
    return pix_polar(ns, ir, (int)floor(t * (double)ir), zc > 0);
}

// FP64 position of sub-point (ia, ib, ic) relative to the target: the box's
// lower corner relative to the target centre, an exact half-integer
// (2 corner - 2 centre is an integer), plus (index + 1/2 + jitter) * box
// extent / s, without contraction (the same operation sequence in every FP64
// evaluation).  It depends on the offset alone, not on where the target lies,
// and scales exactly with the cell size.
__device__ __attribute__((noinline)) int subpoint_pix_d(int ns, int s, int bx, int by, int bz, int ex, int ey, int ez,
                                                        int tx2, int ty2, int tz2, int ia, int ib, int ic)
{
#pragma clang fp contract(off)
    const double ds = (double)s;
    const double vx = 0.5 * (double)(2 * bx - tx2) + (((double)ia + 0.5) + kJit0) * ((double)ex / ds);
    const double vy = 0.5 * (double)(2 * by - ty2) + (((double)ib + 0.5) + kJit1) * ((double)ey / ds);
    const double vz = 0.5 * (double)(2 * bz - tz2) + (((double)ic + 0.5) + kJit2) * ((double)ez / ds);
    return ang2pix_d(ns, vx, vy, vz);
}

// t = atan2(y, x) / (pi/2) in [0, 4].  atan(q) (2/pi) on [0, 1] is the odd
// polynomial q P(q^2), P of degree 7 fitted here (max error 2.4e-8); the
// octant symmetries give the rest.
__device__ inline float quarter_turns(float x, float y)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const float q = mn * __builtin_amdgcn_rcpf(mx);
    const float s = q * q;
    float p = -2.581218548e-03f;
    p = fmaf(p, s, 1.391839830e-02f);
    p = fmaf(p, s, -3.559490869e-02f);
    p = fmaf(p, s, 6.138415100e-02f);
    p = fmaf(p, s, -8.854509426e-02f);
    p = fmaf(p, s, 1.269837831e-01f);
    p = fmaf(p, s, -2.121844841e-01f);
    p = fmaf(p, s, 6.366193494e-01f);
    p *= q;
    if (ay > ax) p = 1.0f - p;
    if (x < 0.f) p = 2.0f - p;
    if (y < 0.f) p = 4.0f - p;
    return p;
}

// reciprocal and square root: hardware approximations (1 ulp) in FP32,
// correctly rounded in FP64
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double frcp(double x) { return 1.0 / x; }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double fsqrt(double x) { return __dsqrt_rn(x); }

// |v - round(v)| < tol, from the floor fl = floor(v) already taken for an index
__device__ inline bool near_edge(float v, float fl, float tol) { return fabsf((v - fl) - 0.5f) > 0.5f - tol; }

// FP32 form.  Every edge decision (|z| against 2/3, the edge indices, the
// pixel inside the ring) is checked against a guard band tol larger than the
// worst-case FP32 error of the decided quantity; unsure is set when any lies
// inside it, and the caller then re-evaluates that sub-point in FP64.
__device__ inline int ang2pix_f(int ns, float x, float y, float z, float tol, bool &unsure)
{
    const float rho2 = fmaf(x, x, y * y);
    const float rinv = __builtin_amdgcn_rsqf(fmaf(z, z, rho2));
    const float zc = z * rinv;
    const float za = fabsf(zc);
    const float t = quarter_turns(x, y);
    unsure |= fabsf(za - (2.f / 3.f)) < tol;
    const float fns = (float)ns;
    if (za <= 2.f / 3.f) {
        const float a = fns * (0.5f + t - 0.75f * zc);
        const float b = fns * (0.5f + t + 0.75f * zc);
        const float fa = floorf(a), fb = floorf(b);
        unsure |= near_edge(a, fa, tol) | near_edge(b, fb, tol);
        return pix_equatorial(ns, (int)fa, (int)fb);
    }
    const float ft = floorf(t);
    const float tp = t - ft;
    unsure |= fabsf(tp - 0.5f) > 0.5f - tol;
    // 1 - |z| = rho^2 / (r (r + |z|)) = rho^2 rinv^2 / (1 + |zc|)
    const float omz = rho2 * rinv * rinv * __builtin_amdgcn_rcpf(1.0f + za);
    const float sig = fns * __builtin_amdgcn_sqrtf(3.f * omz);
    const float A = tp * sig, B = (1.f - tp) * sig;
    const float fA = floorf(A), fB = floorf(B);
    unsure |= near_edge(A, fA, tol) | near_edge(B, fB, tol);
    const int ir = (int)fA + (int)fB + 1;
    const float C = t * (float)ir;
    const float fC = floorf(C);
    unsure |= near_edge(C, fC, tol);
    return pix_polar(ns, ir, (int)fC, zc > 0.f);
}

// ---------------------------------------------------------------------------
// Radial kernels (App. A)
// W_p: piece-wise cubic, a1 = 1.21, a2 = -6.35, A = 0.408, M = 1.184; the
// outer branch is the cubic with a double root at sqrt(3)/2 that equals A
// at 1/2 and has leading coefficient a2.
// ---------------------------------------------------------------------------
template <typename Real>
__device__ inline Real wp_kernel(Real x)
{
    const Real a1 = (Real)1.21, a2 = (Real)-6.35, A = (Real)0.408, M = (Real)1.184;
    const Real xe = (Real)0.86602540378443864676;
    const Real q = (Real)(2.0 * 0.408 * (2.0 + 1.73205080756887729353) + 0.5 * 6.35);
    x = x < (Real)0 ? -x : x;
    if (x < (Real)0.5) return (a1 * x - ((Real)0.5 * a1 + (Real)4 * (M - A))) * x * x + M;
    if (x < xe) {
        const Real u = x - xe;
        return u * u * (a2 * x + q);
    }
    return (Real)0;
}

}  // namespace tr
