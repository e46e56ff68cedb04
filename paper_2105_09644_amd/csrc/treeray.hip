// TreeRay/OnTheSpot on MI355X (gfx950): device kernels and the C ABI.
//
// Steps of one outer iteration (paper Sec. 2):
//   k_fill / k_deposit     point sources onto the leaf cells (Sec. 2.1, 2.7)
//   k_cell_quantities      eps, alpha, e of every cell (eqs. os:ems, os:abs, os:erd)
//   k_reduce_level         FP64 bottom-up node moments, one launch per tree level
//   k_pack                 node records for the sweep (FP64 or FP32, SoA)
//   k_sweep                per target: walk + node->ray mapping + per-ray
//                          On-the-Spot integration + sum over rays (Sec. 2.3-2.5)
//   k_hist / k_select / k_delta   delta_cell with an exact radix-select median
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "tr_internal.h"

namespace tr {

// moment rows of the FP64 node arrays
enum { MO_EPS = 0, MO_ALPHA, MO_E, MO_V, MO_MASS, MO_MX, MO_MY, MO_MZ, MO_VX, MO_VY, MO_VZ, MO_MION, MO_COUNT };

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// a1. Point sources onto leaf cells.  A source coordinate within 1e-9 finest
// cells of a cell face is moved onto it; the rate is split equally over every
// leaf cell whose closed cube contains the point.  One thread per source
// descends the tree from its domain's root.
// ---------------------------------------------------------------------------
__global__ void k_deposit(const double *__restrict__ xyz, const double *__restrict__ q,
                          const int32_t *__restrict__ sdom, int32_t n_src, const DomDev *__restrict__ doms,
                          const int4 *__restrict__ geo, const int2 *__restrict__ topo, double *ndot,
                          int32_t *err)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    const DomDev D = doms[sdom[s]];
    double u[3];
    for (int a = 0; a < 3; ++a) {
        double v = xyz[3 * s + a] / D.dx_cm;
        const double rn = floor(v + 0.5);
        if (fabs(v - rn) <= 1e-9) v = rn;
        u[a] = v;
    }
    int stack[160];
    int sp = 0;
    stack[sp++] = D.root;
    int cells[8];
    int nc = 0;
    while (sp > 0) {
        const int n = stack[--sp];
        const int4 g = geo[n];
        const double sz = (double)(g.w & kSizeMask);
        if (!(u[0] >= g.x && u[0] <= g.x + sz && u[1] >= g.y && u[1] <= g.y + sz && u[2] >= g.z &&
              u[2] <= g.z + sz))
            continue;
        const int2 tp = topo[n];
        if (tp.y == 0) {
            if (nc < 8) cells[nc] = tp.x;
            ++nc;
        } else {
            if (sp + tp.y > 160) { atomicOr(err, 4); return; }
            for (int c = 0; c < tp.y; ++c) stack[sp++] = tp.x + c;
        }
    }
    if (nc == 0 || nc > 8 || !(q[s] >= 0.0) || !isfinite(q[s])) {
        atomicOr(err, 1);
        return;
    }
    const double share = q[s] / (double)nc;
    for (int c = 0; c < nc; ++c) atomicAdd(&ndot[cells[c]], share);
}

// Sources as uniform spheres (Sec. 2.7): each leaf cell receives the rate
// times the fraction of the sphere's in-domain volume that lies inside it.
// Volume of a ball cut by a box = integral over z of the area of a disk cut
// by a rectangle; that area is exact, and the integral is split where the
// circle meets an edge line or a corner of the rectangle (the area's
// derivatives jump there) and taken on each piece after the substitution
// z = p + (q - p)(1 - cos(pi t))/2 with Gauss-Legendre nodes in t.
__constant__ double c_gl_t[kGlNodes], c_gl_w[kGlNodes];

// area of {x >= u, y >= v} inside the disk of radius r, for u, v >= 0
__device__ double disk_corner(double r, double u, double v)
{
    if (u * u + v * v >= r * r) return 0.0;
    const double r2 = r * r, x1 = sqrt(r2 - v * v);
    const double gu = u * sqrt(fmax(r2 - u * u, 0.0)) + r2 * asin(fmin(u / r, 1.0));
    const double g1 = x1 * v + r2 * asin(fmin(x1 / r, 1.0));
    return 0.5 * (g1 - gu) - v * (x1 - u);
}

// the same for any signs: a negative bound is reflected (the half-plane
// x >= u < 0 is twice x >= 0 less x >= -u)
__device__ double disk_quadrant(double r, double u, double v)
{
    if (u >= 0.0 && v >= 0.0) return disk_corner(r, u, v);
    if (v >= 0.0) return 2.0 * disk_corner(r, 0.0, v) - disk_corner(r, -u, v);
    if (u >= 0.0) return 2.0 * disk_corner(r, u, 0.0) - disk_corner(r, u, -v);
    return 2.0 * (2.0 * disk_corner(r, 0.0, 0.0) - disk_corner(r, 0.0, -v)) -
           (2.0 * disk_corner(r, -u, 0.0) - disk_corner(r, -u, -v));
}

__device__ double disk_rect(double r, double x0, double x1, double y0, double y1)
{
    return disk_quadrant(r, x0, y0) - disk_quadrant(r, x1, y0) - disk_quadrant(r, x0, y1) + disk_quadrant(r, x1, y1);
}

// volume of the ball (centre c, radius R) inside the box [lo, hi]
__device__ double ball_box(const double c[3], double R, const double lo[3], const double hi[3])
{
    const double za = fmax(lo[2], c[2] - R), zb = fmin(hi[2], c[2] + R);
    if (za >= zb || lo[0] >= c[0] + R || hi[0] <= c[0] - R || lo[1] >= c[1] + R || hi[1] <= c[1] - R) return 0.0;
    const double x0 = lo[0] - c[0], x1 = hi[0] - c[0], y0 = lo[1] - c[1], y1 = hi[1] - c[1];
    const double dist[8] = {fabs(x0), fabs(x1), fabs(y0), fabs(y1), sqrt(x0 * x0 + y0 * y0), sqrt(x1 * x1 + y0 * y0),
                            sqrt(x0 * x0 + y1 * y1), sqrt(x1 * x1 + y1 * y1)};
    double cut[18];
    int nc = 0;
    cut[nc++] = za;
    cut[nc++] = zb;
    for (int k = 0; k < 8; ++k) {
        if (dist[k] >= R) continue;
        const double h = sqrt(R * R - dist[k] * dist[k]);
        if (c[2] - h > za && c[2] - h < zb) cut[nc++] = c[2] - h;
        if (c[2] + h > za && c[2] + h < zb) cut[nc++] = c[2] + h;
    }
    for (int i = 1; i < nc; ++i)   // insertion sort of at most 18 heights
        for (int j = i; j > 0 && cut[j] < cut[j - 1]; --j) {
            const double t = cut[j];
            cut[j] = cut[j - 1];
            cut[j - 1] = t;
        }
    double v = 0.0;
    for (int k = 0; k + 1 < nc; ++k) {
        const double p = cut[k], q = cut[k + 1];
        if (!(q > p)) continue;
        double sum = 0.0;
        for (int i = 0; i < kGlNodes; ++i) {
            const double t = c_gl_t[i];
            const double z = p + (q - p) * 0.5 * (1.0 - cospi(t));
            const double h = z - c[2];
            const double r2 = R * R - h * h;
            if (r2 > 0.0) sum += c_gl_w[i] * disk_rect(sqrt(r2), x0, x1, y0, y1) * sinpi(t);
        }
        v += sum * (q - p) * 0.5 * kPi;
    }
    return v;
}

// One thread per source; pass 0 sums the in-domain volume, pass 1 deposits.
__global__ void k_deposit_spheres(const double *__restrict__ xyz, const double *__restrict__ q,
                                  const int32_t *__restrict__ sdom, int32_t n_src, const DomDev *__restrict__ doms,
                                  const int4 *__restrict__ geo, const int2 *__restrict__ topo, double radius_cm,
                                  double *ndot, int32_t *err)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_src) return;
    const DomDev D = doms[sdom[s]];
    const double R = radius_cm / D.dx_cm;
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = xyz[3 * s + a] / D.dx_cm;
    if (!(q[s] >= 0.0) || !isfinite(q[s])) {
        atomicOr(err, 1);
        return;
    }
    double total = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        int stack[160];
        int sp = 0;
        stack[sp++] = D.root;
        while (sp > 0) {
            const int n = stack[--sp];
            const int4 g = geo[n];
            const int sz = g.w & kSizeMask;
            const double lo[3] = {(double)g.x, (double)g.y, (double)g.z};
            const double hi[3] = {lo[0] + sz, lo[1] + sz, lo[2] + sz};
            bool touch = true;
            for (int a = 0; a < 3; ++a) touch &= lo[a] < u[a] + R && hi[a] > u[a] - R;
            if (!touch) continue;
            const int2 tp = topo[n];
            if (tp.y == 0) {
                const double v = ball_box(u, R, lo, hi);
                if (v > 0.0) {
                    if (pass == 0) total += v;
                    else atomicAdd(&ndot[tp.x], q[s] * (v / total));
                }
            } else {
                if (sp + tp.y > 160) {
                    atomicOr(err, 4);
                    return;
                }
                for (int c = 0; c < tp.y; ++c) stack[sp++] = tp.x + c;
            }
        }
        if (pass == 0 && !(total > 0.0)) {
            atomicOr(err, 1);
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// a2. Cell quantities in internal units (length: finest cell of the domain;
// rate: rate_unit, a power of two).  s = ndot - alpha_B n^2 dV is netted
// inside the cell: eps = max(s, 0), alpha = max(-s, 0).  E = F_prev dV.
// ---------------------------------------------------------------------------
__global__ void k_cell_quantities(int64_t n_cells, const double *__restrict__ n_h,
                                  const double *__restrict__ ndot, const double *__restrict__ f_prev,
                                  const int32_t *__restrict__ cell_node, const int32_t *__restrict__ cell_dom,
                                  const DomDev *__restrict__ doms, const int4 *__restrict__ geo, int32_t thin,
                                  double *__restrict__ M, int64_t nn, int32_t *err)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int node = cell_node[c];
    const DomDev D = doms[cell_dom[c]];
    const int4 g = geo[node];
    const int sz = g.w & kSizeMask;
    const double dv = (double)sz * (double)sz * (double)sz;
    const double nh = n_h[c];
    double fp = f_prev ? f_prev[c] : 0.0;
    if (!(nh >= 0.0) || !isfinite(nh) || !(fp >= 0.0) || !isfinite(fp)) {
        atomicOr(err, 2);
    }
    const double s = ndot[c] / D.rate_unit - (thin ? 0.0 : D.alpha_int * nh * nh * dv);
    const double mass = nh * dv;
    M[MO_EPS * nn + node] = s > 0.0 ? s : 0.0;
    M[MO_ALPHA * nn + node] = s < 0.0 ? -s : 0.0;
    M[MO_E * nn + node] = (fp / D.flux_unit) * dv;
    M[MO_V * nn + node] = dv;
    M[MO_MASS * nn + node] = mass;
    const double cx = g.x + 0.5 * sz, cy = g.y + 0.5 * sz, cz = g.z + 0.5 * sz;
    M[MO_MX * nn + node] = mass * cx;
    M[MO_MY * nn + node] = mass * cy;
    M[MO_MZ * nn + node] = mass * cz;
    M[MO_VX * nn + node] = dv * cx;
    M[MO_VY * nn + node] = dv * cy;
    M[MO_VZ * nn + node] = dv * cz;
    // ionised gas: cells with a positive previous flux (the IF MAC's ionised mass)
    M[MO_MION * nn + node] = fp > 0.0 ? mass : 0.0;
}

// ---------------------------------------------------------------------------
// a3. Node moments: plain FP64 sums over the children (contiguous), one
// launch per level, deepest first.
// ---------------------------------------------------------------------------
__global__ void k_reduce_level(int64_t b, int64_t e, const int2 *__restrict__ topo, double *__restrict__ M,
                               int64_t nn)
{
    const int64_t n = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= e) return;
    const int2 tp = topo[n];
    if (tp.y == 0) return;
    for (int m = 0; m < MO_COUNT; ++m) {
        double s = 0.0;
        const double *row = M + m * nn + tp.x;
        for (int c = 0; c < tp.y; ++c) s += row[c];
        M[m * nn + n] = s;
    }
}

// Node records for the sweep, and the node flags of the IF and Src MACs
// (Sec. 2.4): an ionisation front when the ionised mass lies strictly between
// 1e-8 and 1 - 1e-8 of the mass, emission when eps_n > 0.
template <typename R, typename R4>
__global__ void k_pack(int64_t nn, const double *__restrict__ M, R4 *__restrict__ A, R4 *__restrict__ B,
                       int4 *__restrict__ geo)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double m = M[MO_MASS * nn + n], v = M[MO_V * nn + n];
    {
        const double mi = M[MO_MION * nn + n], dif = 1e-8;
        int w = geo[n].w & ~(kIfBit | kSrcBit);
        if (dif * m < mi && mi < (1.0 - dif) * m) w |= kIfBit;
        if (M[MO_EPS * nn + n] > 0.0) w |= kSrcBit;
        geo[n].w = w;
    }
    double cx, cy, cz;
    if (m > 0.0) {
        cx = M[MO_MX * nn + n] / m;
        cy = M[MO_MY * nn + n] / m;
        cz = M[MO_MZ * nn + n] / m;
    } else {
        cx = M[MO_VX * nn + n] / v;
        cy = M[MO_VY * nn + n] / v;
        cz = M[MO_VZ * nn + n] / v;
    }
    R4 a, b;
    a.x = (R)cx; a.y = (R)cy; a.z = (R)cz; a.w = (R)M[MO_EPS * nn + n];
    b.x = (R)M[MO_ALPHA * nn + n]; b.y = (R)M[MO_E * nn + n]; b.z = (R)v; b.w = (R)0;
    A[n] = a;
    B[n] = b;
}

// ---------------------------------------------------------------------------
// The sweep
// ---------------------------------------------------------------------------
template <typename Real> struct R4T;
template <> struct R4T<float> { using T = float4; };
template <> struct R4T<double> { using T = double4; };

struct SweepArgs {
    const int4 *geo;
    const int4 *olo;
    const int4 *oext;
    const int2 *topo;
    const void *pA;          // Real4 (com.x, com.y, com.z, eps)
    const void *pB;          // Real4 (alpha, E, V, 0)
    const int32_t *cell_node;
    const int32_t *cell_dom;
    const DomDev *doms;
    const double *r64;       // evaluation points, finest-cell units, per domain
    const float *r32;
    const int64_t *targets;  // explicit target list, or NULL
    const int32_t *order;    // all cells in (domain, Morton) order
    int64_t n_items;
    int64_t n_cells;
    double *f_out;
    uint8_t *ion_out;
    int32_t *queue;          // [0] next item, [1] overflow flag
    unsigned long long *stats;  // [0] accepted, [1] tested, [2] guard recomputes, [3] rays marched in
                                // FP32, [4] of those marched again in FP64, [5] nodes from the table
    void *gbuf;              // ray buffers in global memory (when they do not fit in LDS)
    void *ebuf;              // split LDS buffers: the emission rows, npix x nr_max per workgroup
    int32_t split;           // 1: A, E, V rows in LDS (stride_k = 3 nr_max + 1), emission rows in ebuf
    double theta2, theta_if2, theta_src2;   // squared opening angles (0: criterion off)
    float guard_tol;
    int32_t nside, npix, subsample, fmax, amax, nr_max, stride_k, zeta_g;
    int32_t int_wave;        // 1: a wave per ray (lanes = points); 0: a lane per ray
    int32_t int_group;       // > 0: a group of this many lanes per ray (slots = emitting points)
    int32_t int_fp32;        // 1 (FP32 buffers, groups): the FP32 march, FP64 again near a front
    float front_ratio;       // Phi / Phi_jj below which the FP32 march defers a ray to FP64
    int32_t eps_kernel;      // emission kernel (K_F1 .. K_G; 0 or K_F3: two-point W_f,3)
    int32_t periodic;        // 1: every node through its periodic copy closest to the target
    int32_t mass_gauss;      // 1: W_g for A, E, V and the self term; 0: W_p
    // walk lists too long for LDS: the item is queued in ovf and a second
    // launch (k_sweep_fallback) walks it with per-workgroup lists of gfmax /
    // gamax entries in device memory
    int32_t *ovf;
    int64_t ovf_cap;
    int32_t *glist;
    int32_t gfmax, gamax;
    int32_t pass_rays;   // > 0: the LDS ray buffers hold this many rays; a target's rays are mapped
                         // and integrated in passes over consecutive pixel ranges
    // angular-weight table (NULL: none): for a node of 1, 2, 4 or 8 times the
    // target's size (ri = 0 .. 3) at offset o in target sizes from the
    // target's lower corner, |o_a| <= atab_w[ri], the entry
    // atab_idx[atab_base[ri] + ((o_x + w)(2w + 1) + o_y + w)(2w + 1) + o_z + w]
    // = (first pair << 7) | pairs, each pair in atab_pool = pixel | count << 16
    const int32_t *atab_idx;
    const int32_t *atab_pool;
    int32_t atab_w[kAtabRatios], atab_base[kAtabRatios];
};

// ray buffer rows: eps, A (recombinations), E (previous flux x volume), V
enum { Q_EPS = 0, Q_A = 1, Q_E = 2, Q_V = 3 };

// Where ray k's rows live: A, E and V of point i at b[k stride + oa + (0, 1, 2) nrm + i],
// the emission at e[k estride + i].  Either one buffer with four rows per ray
// (e = b, estride = stride, oa = nrm), or, when four rows do not fit in LDS,
// the A, E, V rows in LDS and the emission rows (written by emitting nodes
// only) in a per-workgroup plane in device memory.
template <typename Real>
struct RayRows {
    Real *b, *e;
    int stride, estride, oa, nrm;
    __device__ Real &A(int k, int i) const { return b[(size_t)k * stride + oa + i]; }
    __device__ Real &E(int k, int i) const { return b[(size_t)k * stride + oa + nrm + i]; }
    __device__ Real &V(int k, int i) const { return b[(size_t)k * stride + oa + 2 * nrm + i]; }
    __device__ Real &eps(int k, int i) const { return e[(size_t)k * estride + i]; }
};

// Accumulation into a ray buffer shared by the waves of a workgroup.  AM: 0 a
// plain add (one wave), 1 a hardware atomic add, 2 (FP32 in LDS) an add by
// compare-and-swap on the value's bits: the same correctly rounded FP32 sum
// in some order, through integer LDS atomics, which this chip runs at a
// higher rate than FP32 ones when many waves deposit at once.
template <typename Real, int AM>
__device__ inline void buf_add(Real *p, Real v)
{
    if constexpr (AM == 2 && sizeof(Real) == 4) {
        unsigned *q = (unsigned *)p;
        unsigned old = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        for (;;) {
            unsigned seen = old;
            const unsigned nv = __float_as_uint(__uint_as_float(old) + v);
            if (__hip_atomic_compare_exchange_strong(q, &seen, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP))
                break;
            old = seen;
        }
    } else if constexpr (AM != 0) {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        *p += v;
    }
}

// Three adds at once (A, E, V of one ray point): in the compare-and-swap form
// the three reads and then the three swaps are in flight together, and only a
// swap that lost a race (another wave changed the value) is repeated.
template <typename Real, int AM>
__device__ inline void buf_add3(Real *p0, Real v0, Real *p1, Real v1, Real *p2, Real v2)
{
    if constexpr (AM == 2 && sizeof(Real) == 4) {
        unsigned *q0 = (unsigned *)p0, *q1 = (unsigned *)p1, *q2 = (unsigned *)p2;
        unsigned o0 = __hip_atomic_load(q0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        unsigned o1 = __hip_atomic_load(q1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        unsigned o2 = __hip_atomic_load(q2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        unsigned r0 = atomicCAS(q0, o0, __float_as_uint(__uint_as_float(o0) + v0));
        unsigned r1 = atomicCAS(q1, o1, __float_as_uint(__uint_as_float(o1) + v1));
        unsigned r2 = atomicCAS(q2, o2, __float_as_uint(__uint_as_float(o2) + v2));
        while (r0 != o0) {
            o0 = r0;
            r0 = atomicCAS(q0, o0, __float_as_uint(__uint_as_float(o0) + v0));
        }
        while (r1 != o1) {
            o1 = r1;
            r1 = atomicCAS(q1, o1, __float_as_uint(__uint_as_float(o1) + v1));
        }
        while (r2 != o2) {
            o2 = r2;
            r2 = atomicCAS(q2, o2, __float_as_uint(__uint_as_float(o2) + v2));
        }
    } else {
        buf_add<Real, AM>(p0, v0);
        buf_add<Real, AM>(p1, v1);
        buf_add<Real, AM>(p2, v2);
    }
}

// Periodic boundaries (Sec. 2.8): v is twice a node centre's offset from the
// target along an axis with period L finest cells; returns the multiple of L
// (in finest cells) that moves the offset into (-L/2, L/2], the closest copy.
__device__ inline int nearest_copy_shift(int v, int L)
{
    const int num = L - v, den = 2 * L;
    const int k = num >= 0 ? num / den : -((-num + den - 1) / den);   // floor(num / den)
    return k * L;
}

// outermost emitting point of a ray
// Per ray, a mask of the points 1 .. N_R - 1 that received emission: ew words
// (1 for N_R <= 64, else 2) of 64 bits, bit i of word w for point 64 w + i.
template <bool ATOMIC>
__device__ inline void mask_or(unsigned long long *p, unsigned long long bits)
{
    if constexpr (ATOMIC)
        __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        *p |= bits;
}

// marks points i0 (if e0) and i0 + 1 (if e1) of the ray whose mask starts at m
template <bool ATOMIC>
__device__ inline void mark_points(unsigned long long *m, int i0, bool e0, bool e1)
{
    const int i1 = i0 + 1;
    const unsigned long long b0 = e0 && i0 >= 1 ? 1ull << (i0 & 63) : 0ull;
    const unsigned long long b1 = e1 ? 1ull << (i1 & 63) : 0ull;
    if ((i0 >> 6) == (i1 >> 6)) {
        if (b0 | b1) mask_or<ATOMIC>(m + (i0 >> 6), b0 | b1);
    } else {
        if (b0) mask_or<ATOMIC>(m + (i0 >> 6), b0);
        if (b1) mask_or<ATOMIC>(m + (i1 >> 6), b1);
    }
}

// outermost marked point (0: none)
__device__ inline int mask_top(unsigned long long w0, unsigned long long w1)
{
    return w1 ? 127 - __clzll((long long)w1) : (w0 ? 63 - __clzll((long long)w0) : 0);
}

// radial kernels by kind: 5 W_p, 6 W_g (App. A.1, A.2)
enum { K_F1 = 1, K_F2 = 2, K_F3 = 3, K_F3N = 4, K_P = 5, K_G = 6 };
template <typename Real>
__device__ inline Real smooth_kernel(bool gauss, Real x)
{
    if (!gauss) return wp_kernel<Real>(x);
    x = x < (Real)0 ? -x : x;
    return x < (Real)0.86602540378443864676 ? (Real)exp((double)(-x * x)) : (Real)0;
}

// Phi (photon rate per steradian) lives in the eps slot of a point once the
// march has passed it; FP32 buffers keep it as a split double in the
// (eps, A) slots, both consumed by then.
__device__ inline double phi_load(const RayRows<double> &R, int k, int j) { return R.eps(k, j); }
__device__ inline void phi_store(const RayRows<double> &R, int k, int j, double v) { R.eps(k, j) = v; }
__device__ inline double phi_load(const RayRows<float> &R, int k, int j)
{
    const uint32_t lo = __float_as_uint(R.eps(k, j));
    const uint32_t hi = __float_as_uint(R.A(k, j));
    return __hiloint2double((int)hi, (int)lo);
}
__device__ inline void phi_store(const RayRows<float> &R, int k, int j, double v)
{
    R.eps(k, j) = __uint_as_float((uint32_t)__double2loint(v));
    R.A(k, j) = __uint_as_float((uint32_t)__double2hiint(v));
}

// 1/x in FP64 for the ray march (x > 0, finite): the hardware estimate (relative
// error below 2^-24 on this chip, measured) refined by one Newton step, which
// squares the error: a few 1e-15, far inside the FP64 form's 1e-10 bound, with
// two fewer dependent FMAs on the march's critical path
__device__ inline double drcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// One ray (Sec. 2.5), one lane: march inwards from the outermost point that
// holds emission (top; nothing reaches the target from beyond it), all
// sources together.
// Per segment [r_i, r_{i+1}] and source j beyond it:
//   R = (alpha_i + alpha_{i+1})/2 dV_{i,j} zeta_s zeta_d zeta_g,
//   zeta_s zeta_d = F_{i+1,j} min(2/F_{i+1}, 1/Fbar_{i+1})   (zeta_d = 2 where Fbar = 0),
//   dV_{i,j} = (r_{i+1} - r_i)(A^2 + A B + B^2)/3, A = r_j - r_i, B = r_j - r_{i+1},
// and the source at r_{i+1} itself takes zeta_s = zeta_d = 1.
// Returns F_{0,k} in internal flux units.
template <typename Real>
__device__ double integrate_ray(const RayRows<Real> &R, int k, const double *r, const double *inv2r, int nr, int top,
                                int nside, int zeta_g, bool clear_eps)
{
    const double inv4pi = 1.0 / (4.0 * kPi);
    const double ns = (double)nside;
    uint64_t m0 = 0, m1 = 0;     // points j holding a live Phi_j
    double a1 = 0.0, fb1 = 0.0;  // alpha and previous flux at r_{i+1}
    // the point's buffer entries are fetched one step ahead
    Real nV = R.V(k, top), nA = R.A(k, top), nE = R.E(k, top), nEps = R.eps(k, top);
    for (int i = top; i >= 0; --i) {
        const double Vi = (double)nV, Ai = (double)nA, Ei = (double)nE, ei = (double)nEps;
        if (i > 0) {
            nV = R.V(k, i - 1);
            nA = R.A(k, i - 1);
            nE = R.E(k, i - 1);
            nEps = R.eps(k, i - 1);
        }
        double ai = 0.0, fbi = 0.0;
        if (Vi > 0.0) {
            const double rv = drcp(Vi);
            ai = Ai * rv;
            fbi = Ei * rv;
        }
        if (i <= nr - 2 && (m0 | m1)) {
            const double ri = r[i], ri1 = r[i + 1], seg = ri1 - ri;
            // F_{i+1}: flux at r_{i+1} from the sources beyond it
            double ftot = 0.0;
            for (int h = 0; h < 2; ++h) {
                uint64_t m = h ? m1 : m0;
                while (m) {
                    const int j = (h << 6) + __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    if (j >= i + 2) {
                        const double dd = r[j] - ri1;
                        ftot += phi_load(R, k, j) * drcp(dd * dd);
                    }
                }
            }
            double g = 0.0;
            if (ftot > 0.0) {
                g = 2.0 * drcp(ftot);
                if (fb1 > 0.0) g = fmin(g, drcp(fb1));
            }
            const double aseg = 0.5 * (ai + a1) * seg * (1.0 / 3.0);
            for (int h = 0; h < 2; ++h) {
                uint64_t m = h ? m1 : m0;
                while (m) {
                    const int j = (h << 6) + __ffsll((unsigned long long)m) - 1;
                    m &= m - 1;
                    double ph = phi_load(R, k, j);
                    const double rj = r[j];
                    const double A = rj - ri, B = rj - ri1;
                    double z = 1.0;
                    if (j >= i + 2) z = ph * drcp(B * B) * g;
                    if (zeta_g) z *= fmin(1.0, ns * A * inv2r[j]);
                    ph = fmax(0.0, ph - aseg * (A * A + A * B + B * B) * z);
                    phi_store(R, k, j, ph);
                    if (!(ph > 0.0)) {
                        if (j < 64) m0 &= ~(1ull << j);
                        else m1 &= ~(1ull << (j - 64));
                    }
                }
            }
        }
        if (i >= 1 && ei > 0.0) {
            phi_store(R, k, i, ei * inv4pi);
            if (i < 64) m0 |= 1ull << i;
            else m1 |= 1ull << (i - 64);
        }
        a1 = ai;
        fb1 = fbi;
    }
    double f0 = 0.0;
    for (int h = 0; h < 2; ++h) {
        uint64_t m = h ? m1 : m0;
        while (m) {
            const int j = (h << 6) + __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const double rj = r[j];
            f0 += phi_load(R, k, j) * drcp(rj * rj);
        }
    }
    // emission rows kept in device memory are left zero for the next target
    // (the march reused them for Phi)
    if (clear_eps)
        for (int i = 1; i <= top; ++i) R.eps(k, i) = (Real)0;
    return f0;
}

template <typename T>
__device__ inline T rdlane(T v, int l);

// value of point i held by lane i % 64 of the pair (v[0], v[1]); i uniform
__device__ inline double point_value(const double v[2], int i)
{
    return i < 64 ? rdlane(v[0], i) : rdlane(v[1], i - 64);
}

// The same march with a whole wave on one ray: lane p holds point p (and
// p + 64), so every source on the ray advances in the same step and the
// total flux F_{i+1} is a wave reduction.  Phi stays in registers.  Returns
// F_{0,k} (uniform) in internal flux units.
template <typename Real, int NH>
__device__ double integrate_ray_wave(const RayRows<Real> &R, int k, const double *r, const double *inv2r, int nr,
                                     int top, int nside, int zeta_g, bool clear_eps)
{
    const int lane = lane_id();
    const double inv4pi = 1.0 / (4.0 * kPi);
    const double ns = (double)nside;
    double al[2], fb[2], ph[2], rp[2], i2r[2], ep[2];
    bool live[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int p = lane + 64 * h;
        al[h] = fb[h] = ph[h] = ep[h] = rp[h] = i2r[h] = 0.0;
        live[h] = false;
        if (p < nr) {
            const double V = (double)R.V(k, p);
            if (V > 0.0) {
                const double rv = drcp(V);
                al[h] = (double)R.A(k, p) * rv;
                fb[h] = (double)R.E(k, p) * rv;
            }
            ep[h] = (double)R.eps(k, p);
            rp[h] = r[p];
            i2r[h] = inv2r[p];
        }
    }
    bool any = false;   // uniform: some source on the ray is still live
    for (int i = top; i >= 0; --i) {
        if (i <= nr - 2 && any) {
            const double ri = r[i], ri1 = r[i + 1];
            const double ai = point_value(al, i), ai1 = point_value(al, i + 1), fb1 = point_value(fb, i + 1);
            double f[2], fs = 0.0;
            f[1] = 0.0;
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                f[h] = 0.0;
                if (live[h] && lane + 64 * h >= i + 2) {
                    const double B = rp[h] - ri1;
                    f[h] = ph[h] * drcp(B * B);
                }
                fs += f[h];
            }
            const double ftot = wave_sum(fs);
            double g = 0.0;
            if (ftot > 0.0) {
                g = 2.0 * drcp(ftot);
                if (fb1 > 0.0) g = fmin(g, drcp(fb1));
            }
            const double aseg = 0.5 * (ai + ai1) * (ri1 - ri) * (1.0 / 3.0);
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                if (live[h]) {
                    const double A = rp[h] - ri, B = rp[h] - ri1;
                    double z = lane + 64 * h >= i + 2 ? f[h] * g : 1.0;
                    if (zeta_g) z *= fmin(1.0, ns * A * i2r[h]);
                    ph[h] = fmax(0.0, ph[h] - aseg * (A * A + A * B + B * B) * z);
                    live[h] = ph[h] > 0.0;
                }
            }
            any = __ballot(live[0] || live[1]) != 0ull;
        }
        if (i >= 1 && point_value(ep, i) > 0.0) {
            const int h = i >> 6;
            if (lane == (i & 63)) {
                ph[h] = ep[h] * inv4pi;
                live[h] = true;
            }
            any = true;
        }
    }
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        if (live[h]) s += ph[h] * drcp(rp[h] * rp[h]);
        // emission rows kept in device memory are left zero for the next target
        if (clear_eps && ep[h] > 0.0) R.eps(k, lane + 64 * h) = (Real)0;
    }
    return wave_sum(s);
}

// Slot sl of a group of G lanes gets the sl-th emitting point of its ray
// (from the ray's mask (w0, w1) of points 1 .. N_R - 1; -1: none); cnt
// returns the ray's number of emitting points.
template <int G>
__device__ inline int group_emitter(unsigned long long w0, unsigned long long w1, int sl, bool has_ray, int &cnt)
{
    const int c0 = (int)__popcll(w0);
    cnt = has_ray ? c0 + (int)__popcll(w1) : 0;
    if (sl >= cnt) return -1;
    return sl < c0 ? nth_set_bit(w0, sl) : 64 + nth_set_bit(w1, sl - c0);
}

// The same march with a group of G lanes per ray (G = 4 .. 64), so that a
// wave integrates 64/G rays at once: slot s of the group holds the ray's s-th
// emitting point j (in pixel-row order) with its Phi_j in a register, and
// F_{i+1} is a group sum.  Every lane of a group reads the same point's
// moments.  k / (w0, w1): this lane's ray (has_ray false: none) and its
// mask of emitting points; tmax: the largest outermost emitting point of the
// wave's rays (uniform).  A
// ray with more than G emitting points is left alone (n_over returns their
// number on its lanes, else 0; the caller integrates it with more lanes).
// Returns F_{0,k} in internal flux units on every lane of the group.  Call
// with every lane active.
template <typename Real, int G>
__device__ double integrate_rays_group(const RayRows<Real> &R, int k, unsigned long long w0, unsigned long long w1,
                                       bool has_ray, int tmax,
                                       const double *r, const double *inv2r, int nr, int nside, int zeta_g,
                                       int &n_over, bool clear_eps)
{
    const int lane = lane_id();
    const int sl = lane & (G - 1);
    const int g0 = lane - sl;   // first lane of the group
    const double inv4pi = 1.0 / (4.0 * kPi);
    const double ns = (double)nside;
    int cnt;
    const int j = group_emitter<G>(w0, w1, sl, has_ray, cnt);
    n_over = has_ray && cnt > G ? cnt : 0;
    const bool act = has_ray && cnt <= G;
    double rj = 0.0, i2rj = 0.0, epsj = 0.0;
    if (act && j > 0) {
        rj = r[j];
        i2rj = inv2r[j];
        epsj = (double)R.eps(k, j);
    }
    const double phjj = epsj * inv4pi;   // Phi_jj, emitted at r_j
    double ph = 0.0, a1 = 0.0, fb1 = 0.0;   // alpha and previous flux at r_{i+1}
    bool live = false;
    // every step is predicated (selects, no branches on lane values); the
    // moments are read one point ahead, beyond the ray's outermost emitting
    // point too (they meet no live source); r_{i+1} and B = r_j - r_{i+1} are
    // the previous step's r_i and A
    double ri1 = tmax + 1 < nr ? r[tmax + 1] : 0.0;
    double Bv = rj - ri1, B2 = Bv * Bv;
    Real nV = R.V(k, tmax), nA = R.A(k, tmax), nE = R.E(k, tmax);
    for (int i = tmax; i >= 0; --i) {
        const double Vi = (double)nV, Ai = (double)nA, Ei = (double)nE;
        if (i >= 1) {
            nV = R.V(k, i - 1);
            nA = R.A(k, i - 1);
            nE = R.E(k, i - 1);
        }
        const double rv = drcp(Vi);
        const double ai = Vi > 0.0 ? Ai * rv : 0.0;
        const double fbi = Vi > 0.0 ? Ei * rv : 0.0;
        const double ri = r[i];
        const double A = rj - ri, A2 = A * A;
        if (i <= nr - 2) {
            const bool far = live && j >= i + 2;
            const double f = far ? ph * drcp(B2) : 0.0;
            const double ftot = group_sum(f, G);   // F_{i+1} of the group's ray
            // min(2 / F_{i+1}, 1 / Fbar_{i+1}), used where f > 0 (so F_{i+1} > 0)
            const double g2 = 2.0 * drcp(ftot);
            const double g = fb1 > 0.0 ? fmin(g2, drcp(fb1)) : g2;
            const double aseg = 0.5 * (ai + a1) * (ri1 - ri) * (1.0 / 3.0);
            double z = far ? f * g : 1.0;
            if (zeta_g) z *= fmin(1.0, ns * A * i2rj);
            const double nph = ph - aseg * (A2 + A * Bv + B2) * z;
            const bool alive = live && nph > 0.0;
            ph = alive ? nph : 0.0;
            live = alive;
        }
        const bool born = act && i >= 1 && j == i;
        ph = born ? phjj : ph;
        live = live || born;
        a1 = ai;
        fb1 = fbi;
        ri1 = ri;
        Bv = A;
        B2 = A2;
    }
    // emission rows kept in device memory are left zero for the next target
    if (clear_eps && act && j > 0) R.eps(k, j) = (Real)0;
    return group_sum(live ? ph * drcp(rj * rj) : 0.0, G);
}

// The same march in FP32 (FP32C integration, Sec. 2.5), a group of G lanes
// per ray as above, for FP32 ray buffers:
//  - radial differences from exact integers: r_j - r_i = c (j^2 - i^2), so a
//    segment's volume dV_{i,j} carries no cancellation error;
//  - Phi_j is kept as an unevaluated FP32 pair (hi + lo): each loss R is
//    subtracted with its rounding error kept (Fast2Sum, exact while R <= Phi),
//    so Phi's error is only that of the R's themselves (a few ulp of each, at
//    most a few 1e-7 of the emitted Phi_jj in all);
//  - F_{0,k} = sum_j Phi_{0,j} / r_j^2 as a compensated group sum.
// Where the FP32 result is not safe to 1e-4 -- a live source whose Phi falls
// below front_ratio of its emitted Phi_jj, or dies in a step whose loss is
// within 1e-3 of what it had (a close call between dying and surviving), the
// regime of an ionisation front -- near is set on the group and the caller
// integrates that ray again in FP64.  Returns F_{0,k} as (hi, lo) on every
// lane of the group.  Call with every lane active.
template <int G>
__device__ void integrate_rays_group_f32(const RayRows<float> &R, int k, unsigned long long w0, unsigned long long w1,
                                         bool has_ray, int tmax,
                                         float rcoef, const double *inv2r, int nr, int nside, int zeta_g,
                                         float front_ratio, int &n_over, bool &near, float &f_hi, float &f_lo,
                                         bool clear_eps)
{
    const int lane = lane_id();
    const int sl = lane & (G - 1);
    const int g0 = lane - sl;
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    const float inv4pi = (float)(1.0 / (4.0 * kPi));
    const float ns = (float)nside;
    const float third = 1.0f / 3.0f;
    int cnt;
    const int j = group_emitter<G>(w0, w1, sl, has_ray, cnt);
    n_over = has_ray && cnt > G ? cnt : 0;
    const bool act = has_ray && cnt <= G;
    float i2rj = 0.0f, epsj = 0.0f, rj = 0.0f;
    const int j2 = j > 0 ? j * j : 0;
    if (act && j > 0) {
        i2rj = (float)inv2r[j];
        epsj = R.eps(k, j);
        rj = rcoef * (float)j2;
    }
    const float phjj = epsj * inv4pi;   // Phi_jj, emitted at r_j
    const float gz = ns * i2rj;         // zeta_g = min(1, gz (r_j - r_i))
    float ph = 0.0f, pl = 0.0f, a1 = 0.0f, fb1 = 0.0f;
    bool live = false, died = false;
    float bd = 0.0f, ld = 0.0f;   // at the source's death: its Phi before the step and the step's loss
    // every step is predicated (selects, no branches on lane values); the
    // moments are read one point ahead, beyond the ray's outermost emitting
    // point too (they meet no live source).  q = j^2 - i^2 exactly, so
    // A = r_j - r_i = c q, and B = r_j - r_{i+1} is the previous step's A.
    float q = (float)(j2 - (tmax + 1) * (tmax + 1));
    float Bv = rcoef * q, B2 = Bv * Bv;
    float nV = R.V(k, tmax), nA = R.A(k, tmax), nE = R.E(k, tmax);
    for (int i = tmax; i >= 0; --i) {
        const float Vi = nV, Ai = nA, Ei = nE;
        if (i >= 1) {
            nV = R.V(k, i - 1);
            nA = R.A(k, i - 1);
            nE = R.E(k, i - 1);
        }
        const float rv = __builtin_amdgcn_rcpf(Vi);
        const float ai = Vi > 0.0f ? Ai * rv : 0.0f;
        const float fbi = Vi > 0.0f ? Ei * rv : 0.0f;
        const float odd = (float)(2 * i + 1);
        q += odd;
        const float A = rcoef * q, A2 = A * A;
        if (i <= nr - 2) {
            const bool far = live && j >= i + 2;
            const float f = far ? (ph + pl) * __builtin_amdgcn_rcpf(B2) : 0.0f;
            const float ftot = group_sum(f, G);   // F_{i+1} of the group's ray
            // min(2 / F_{i+1}, 1 / Fbar_{i+1}); used where f > 0 (so F_{i+1} > 0), and
            // Fbar_{i+1} = 0 gives 1 / Fbar = +inf
            const float g = fminf(2.0f * __builtin_amdgcn_rcpf(ftot), __builtin_amdgcn_rcpf(fb1));
            const float aseg = 0.5f * (ai + a1) * (rcoef * odd) * third;
            float z = far ? f * g : 1.0f;
            if (zeta_g) z *= fminf(1.0f, A * gz);
            const float loss = aseg * (A2 + A * Bv + B2) * z;
            const float before = ph + pl;
            // ph - loss as sh + se, exactly while the source lives (|loss| <= ph:
            // Fast2Sum); a larger loss kills it whatever the rounding, and a near
            // tie is the close call marched again in FP64
            const float sh = ph - loss;
            const float se = -loss - (sh - ph);
            const float npl = pl + se;
            const bool alive = live && sh + npl > 0.0f;
            const bool dies = live && !alive;
            bd = dies ? before : bd;
            ld = dies ? loss : ld;
            died = died || dies;
            ph = alive ? sh : 0.0f;
            pl = alive ? npl : 0.0f;
            live = alive;
        }
        const bool born = act && i >= 1 && j == i;
        ph = born ? phjj : ph;
        live = live || born;
        a1 = ai;
        fb1 = fbi;
        Bv = A;
        B2 = A2;
    }
    // Phi only falls: a live source ended below front_ratio of Phi_jj, or a
    // source died from below that or in a close call between dying and
    // surviving (the step's loss within 1e-3 of what it had)
    const float frp = front_ratio * phjj;
    const bool flag = (live && ph + pl < frp) || (died && (bd < frp || ld < 1.001f * bd));
    float th = 0.0f, tl = 0.0f;
    if (live) {
        const float rr = __builtin_amdgcn_rcpf(rj * rj);
        th = ph * rr;
        tl = pl * rr;
    }
    group_csum(th, tl, G);
    f_hi = th;
    f_lo = tl;
    near = ((__ballot(flag) >> g0) & gmask) != 0ull;
    // emission rows kept in device memory are left zero for the next target
    // (a ray marched again in FP64 is cleared there)
    if (clear_eps && act && j > 0 && !near) R.eps(k, j) = 0.0f;
}

// The class of ray k (k >= np: none) from its mask of emitting points: 0 no
// emission, else ceil(log2) of its number of emitting points, at least lg0, 7
// beyond 64; tp returns its outermost emitting point.
__device__ inline int ray_class(const unsigned long long *emask, int ew, int np, int lg0, int k, int &tp)
{
    unsigned long long w0 = 0ull, w1 = 0ull;
    if (k < np) {
        w0 = emask[(size_t)k * ew];
        if (ew > 1) w1 = emask[(size_t)k * ew + 1];
    }
    tp = mask_top(w0, w1);
    const int cnt = (int)(__popcll(w0) + __popcll(w1));
    return cnt == 0 ? 0 : cnt > 64 ? 7 : max(lg0, 32 - __clz(cnt - 1));
}

// One batch of the group integration: 64 / G rays of G lanes each (myk < 0:
// no ray on this group; (m0, m1) the ray's mask of emitting points).  Adds the
// rays' F_{0,k} on their groups' first lanes: FP64 results into fsum, FP32
// marched ones (FP32 buffers with the FP32 march) into the compensated pair
// (cs_hi, cs_lo), a ray near an ionisation front marched again in FP64.
template <typename Real, int G>
__device__ __forceinline__ void march_batch(const SweepArgs &a, const RayRows<Real> &R, int myk, unsigned long long m0,
                                            unsigned long long m1, Real rcoef,
                                            const double *rd, const double *rd2, int nr, bool split, double &fsum,
                                            float &cs_hi, float &cs_lo, double &n_f32, double &n_f64)
{
    const int lane = lane_id();
    const bool has = myk >= 0;
    const int tmax = wave_max_nonneg(mask_top(m0, m1));
    const bool head = (lane & (G - 1)) == 0;
    int over = 0;   // zero: the ray's class holds its emitting points
    if constexpr (sizeof(Real) == 4) {
        if (a.int_fp32) {
            bool near = false;
            float fh = 0.0f, fl = 0.0f;
            integrate_rays_group_f32<G>(R, has ? myk : 0, m0, m1, has, tmax, rcoef, rd2, nr, a.nside, a.zeta_g,
                                        a.front_ratio, over, near, fh, fl, split);
            const bool ok = head && has;
            if (ok && !near) {
                float sh, se;
                two_sum(cs_hi, fh, sh, se);
                cs_hi = sh;
                cs_lo += se + fl;
            }
            n_f32 += ok ? 1.0 : 0.0;
            // the rays near an ionisation front, again in FP64
            const bool redo = has && near;
            if (__ballot(head && redo)) {
                const double f = integrate_rays_group<Real, G>(R, redo ? myk : 0, m0, m1, redo, tmax, rd, rd2, nr,
                                                               a.nside, a.zeta_g, over, split);
                if (head && redo) fsum += f;
                n_f64 += head && redo ? 1.0 : 0.0;
            }
            return;
        }
    }
    const double f = integrate_rays_group<Real, G>(R, has ? myk : 0, m0, m1, has, tmax, rd, rd2, nr, a.nside, a.zeta_g,
                                                   over, split);
    if (head && has) fsum += f;
}

template <typename T>
__device__ inline T rdlane(T v, int l)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    } else {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
        return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
}

// W_f,1 and W_f,2 (App. A.3) on the bracket r_i <= d < r_{i+1}: both keep the
// flux at the target exact; W_f,1 takes u_{i+1}/u_i = (d - r_i)/(r_{i+1} - d),
// W_f,2 also makes the flux exact at r_{i-1} (i >= 2; it keeps W_f,3 when a
// weight would be negative).  Solved in FP64.
template <typename Real>
__device__ void two_point_variant(int ek, const Real *rt, int i, double d, Real &u0, Real &u1)
{
    const double ri = (double)rt[i], rn = (double)rt[i + 1];
    if (ek == K_F1) {
        const double rho = (d - ri) / (rn - d);
        const double ui = 1.0 / (d * d * (1.0 / (ri * ri) + rho / (rn * rn)));
        u0 = (Real)ui;
        u1 = (Real)(rho * ui);
        return;
    }
    if (i < 2) return;
    const double p = (double)rt[i - 1];
    const double a11 = 1.0 / (ri * ri), a12 = 1.0 / (rn * rn), b1 = 1.0 / (d * d);
    const double a21 = 1.0 / ((ri - p) * (ri - p)), a22 = 1.0 / ((rn - p) * (rn - p)), b2 = 1.0 / ((d - p) * (d - p));
    const double det = a11 * a22 - a12 * a21;
    const double ui = (b1 * a22 - a12 * b2) / det, un = (a11 * b2 - a21 * b1) / det;
    if (ui >= 0.0 && un >= 0.0) {
        u0 = (Real)ui;
        u1 = (Real)un;
    }
}

// N-point W_f,3 (App. A.3, eqs. eKernFC1, eKernFC2): over the points k >= 1
// inside the node's extent, |r_k - d| < sqrt(3)/2 h, weights a + b (k - le)
// with sum 1 and sum 1/r_k^2 = 1/d^2.  Leaves mode 0 (two-point) when fewer
// than two points qualify or a weight would be negative.  Solved in FP64.
template <typename Real>
__device__ void n_point_f3(const Real *rt, int l0, int h0, double d, double h, int &mode, int &le, int &ne, Real &ea,
                           Real &eb)
{
    const double half = 0.86602540378443864676 * h;
    int first = -1, n = 0;
    double s1 = 0, t0 = 0, t1 = 0;
    for (int k = l0 > 1 ? l0 : 1; k <= h0; ++k) {
        const double rk = (double)rt[k];
        if (fabs(rk - d) >= half) continue;
        if (first < 0) first = k;
        const double m = (double)(k - first), w = 1.0 / (rk * rk);
        s1 += m;
        t0 += w;
        t1 += m * w;
        ++n;
    }
    if (n < 2) return;
    const double det = (double)n * t1 - s1 * t0;
    const double av = (t1 - s1 / (d * d)) / det, bv = ((double)n / (d * d) - t0) / det;
    if (av < 0.0 || av + bv * (double)(n - 1) < 0.0) return;
    mode = 1;
    le = first;
    ne = n;
    ea = (Real)av;
    eb = (Real)bv;
}

// Weight of support point i (offset io from the support's first point) in the
// spread emission forms: 1 linear N-point W_f,3, 2 a smoothing kernel scaled by
// ea, 3 the mass fall-back split (fb on the first point, 1 - fb on the next).
template <typename Real>
__device__ inline Real emission_weight(int mode, int i, int io, int le, int ne, Real ea, Real eb, Real fb, Real rcoef,
                                       Real d, Real hinv, bool gauss)
{
    if (mode == 1) return (i >= le && i < le + ne) ? ea + eb * (Real)(i - le) : (Real)0;
    if (mode == 2) return smooth_kernel<Real>(gauss, (rcoef * (Real)(i * i) - d) * hinv) * ea;
    return io == 0 ? fb : (Real)1 - fb;
}

// Maps the accepted nodes acc[0..cnt) (cnt <= 64) onto the target's rays;
// executed by a whole wave in two phases.
//  Phase 1, lane = node: loads the node, its mass-centre distance d, the
//   W_p normalisation over the evaluation points in its support and the W_f,3
//   bracket of its emission (App. A).
//  Phase 2, lane = angular sub-point, node by node: the pixel of each of the
//   s^3 sub-box midpoints of the node's box (the share of pixel k is the count
//   in k over s^3), then the scatter, with lanes covering (pixel, point) pairs.
// The evaluation points are r_i = c i^2; the per-node loop recomputes them
// in registers, so it makes no memory round trip besides its atomics.
// KV: the radial-kernel variants of App. A (otherwise two-point W_f,3 and W_p)
// This lane's (pixel, count) pair of the angular-table entry t ((first << 7) |
// pairs; t < 0: none), 0 beyond the entry's pairs
__device__ inline int table_pairs(const int32_t *pool, int t, int lane)
{
    return t >= 0 && lane < (t & 127) ? pool[(t >> 7) + lane] : 0;
}

template <typename Real, int ATOMIC, bool KV, bool PASS>
__device__ void map_nodes(const SweepArgs &a, const RayRows<Real> &R, unsigned long long *emask, int ew, const int *per,
                          const Real *rt, int nr,
                          Real rc_inv,
                          Real rcoef, const int *acc, int cnt, int tx, int ty, int tz, int tsize, int k0, int np,
                          double &guard_count, double &tab_count)
{
    using R4 = typename R4T<Real>::T;
    // emission rows (few writes; in device memory when the A, E, V rows alone fill LDS): hardware atomics
    constexpr int EATOMIC = ATOMIC != 0 ? 1 : 0;
    const int lane = lane_id();
    const Real xe = (Real)0.86602540378443864676;
    // ---------------- phase 1 ----------------
    int bx = 0, by = 0, bz = 0, ex = 1, ey = 1, ez = 1, lo = 0, nsup = 0, ie = 1;
    Real d = 1, hinv = 1, wscale = 0, fb0 = 1, qa = 0, qe = 0, qv = 0, e0 = 0, e1 = 0;
    // emission spread over several points: mode 1 linear (a + b (i - le) on [le, le + ne)),
    // 2 a smoothing kernel scaled by ea, 3 the mass fall-back weights; etop: outermost point
    int emode = 0, le = 0, ne = 0, etop = 1;
    Real ea = 0, eb = 0, qeps = 0;
    int tab = -1;   // the node's angular-table entry (-1: classify its sub-points)
    const bool mg = KV && a.mass_gauss != 0;
    if (lane < cnt) {
        const int n = acc[lane];
        const int4 g = a.geo[n];
        const int size = g.w & kSizeMask;
        bx = g.x; by = g.y; bz = g.z;
        ex = ey = ez = size;
        if (g.w & kPartialBit) {
            const int4 o = a.olo[n], e = a.oext[n];
            bx = o.x; by = o.y; bz = o.z;
            ex = e.x; ey = e.y; ez = e.z;
        }
        const R4 A = ((const R4 *)a.pA)[n];
        const R4 B = ((const R4 *)a.pB)[n];
        qa = B.x; qe = B.y; qv = B.z;
        int shx = 0, shy = 0, shz = 0;   // periodic copy closest to the target (by the cube's centre)
        if (per) {
            shx = nearest_copy_shift(2 * g.x + size - tx, per[0]);
            shy = nearest_copy_shift(2 * g.y + size - ty, per[1]);
            shz = nearest_copy_shift(2 * g.z + size - tz, per[2]);
            bx += shx;
            by += shy;
            bz += shz;
        }
        if (a.atab_idx && !(g.w & kPartialBit)) {
            // a cube of 1, 2, 4 or 8 target sizes: offsets of its corner in target sizes (exact)
            const int ri = size == tsize ? 0 : size == 2 * tsize ? 1 : size == 4 * tsize ? 2 : size == 8 * tsize ? 3 : -1;
            if (ri >= 0) {
                const int sh = __builtin_ctz((unsigned)tsize);
                const int kx = (bx - ((tx - tsize) >> 1)) >> sh, ky = (by - ((ty - tsize) >> 1)) >> sh,
                          kz = (bz - ((tz - tsize) >> 1)) >> sh;
                const int w = a.atab_w[ri], nw = 2 * w + 1;
                if (abs(kx) <= w && abs(ky) <= w && abs(kz) <= w)
                    tab = a.atab_idx[a.atab_base[ri] + ((kx + w) * nw + (ky + w)) * nw + (kz + w)];
            }
        }
        const Real dxc = (A.x + (Real)shx) - (Real)0.5 * (Real)tx, dyc = (A.y + (Real)shy) - (Real)0.5 * (Real)ty,
                   dzc = (A.z + (Real)shz) - (Real)0.5 * (Real)tz;
        d = fsqrt(dxc * dxc + dyc * dyc + dzc * dzc);
        const Real h = (Real)size;
        hinv = frcp(h);   // a power of two: exact
        const Real rl = d - xe * h, rh = d + xe * h;
        int l0 = rl > (Real)0 ? (int)fsqrt(rl * rc_inv) - 1 : 0;
        int h0 = (int)fsqrt(rh * rc_inv) + 2;
        l0 = l0 < 0 ? 0 : l0;
        h0 = h0 > nr - 1 ? nr - 1 : h0;
        Real sum = 0;
        for (int i = l0; i <= h0; ++i) sum += smooth_kernel<Real>(mg, (rcoef * (Real)(i * i) - d) * hinv);
        if (sum > (Real)0) {
            wscale = frcp(sum);
            lo = l0;
            nsup = h0 - l0 + 1;
        } else if (d >= rt[nr - 1]) {   // no point in the support: linear split over the bracket
            lo = nr - 1;
            nsup = 1;
            fb0 = 1;
        } else {
            int ib = (int)fsqrt(d * rc_inv);
            ib = ib > nr - 2 ? nr - 2 : ib;
            while (ib > 0 && rt[ib] > d) --ib;
            while (ib < nr - 2 && rt[ib + 1] <= d) ++ib;
            lo = ib;
            nsup = 2;
            fb0 = (rt[ib + 1] - d) * frcp(rt[ib + 1] - rt[ib]);
        }
        qeps = A.w;
        const int ek = KV ? a.eps_kernel : 0;
        if (A.w > (Real)0 && (ek == K_P || ek == K_G)) {   // a smoothing kernel for the emission too
            if (sum > (Real)0) {
                Real es = 0;
                for (int i = l0; i <= h0; ++i) {
                    const Real v = smooth_kernel<Real>(ek == K_G, (rcoef * (Real)(i * i) - d) * hinv);
                    es += v;
                    if (v > (Real)0) etop = i;
                }
                emode = 2;
                ea = frcp(es);
            } else {
                emode = 3;
                etop = lo + nsup - 1;
            }
        } else if (A.w > (Real)0) {   // W_f,3 bracket r_i <= d < r_{i+1}, i >= 1
            Real u0 = 1, u1 = 0;
            if (d >= rt[nr - 1]) {
                ie = nr - 1;
            } else if (d >= rt[1]) {
                int k = (int)fsqrt(d * rc_inv);
                k = k < 1 ? 1 : (k > nr - 2 ? nr - 2 : k);
                while (k > 1 && rt[k] > d) --k;
                while (k < nr - 2 && rt[k + 1] <= d) ++k;
                ie = k;
                const Real ai = frcp(rt[ie] * rt[ie]), an = frcp(rt[ie + 1] * rt[ie + 1]), ad = frcp(d * d);
                u0 = (ad - an) * frcp(ai - an);
                u1 = (Real)1 - u0;
                if (ek == K_F1 || ek == K_F2)
                    two_point_variant(ek, rt, ie, (double)d, u0, u1);
            }
            if (ek == K_F3N && sum > (Real)0)
                n_point_f3(rt, l0, h0, (double)d, (double)h, emode, le, ne, ea, eb);
            if (emode == 1) {
                etop = le + ne - 1;
            } else {
                e0 = A.w * u0;
                e1 = A.w * u1;
                etop = u1 != (Real)0 ? ie + 1 : ie;
            }
        }
    }

    // ---------------- phase 2 ----------------
    const int s = a.subsample, s3 = s * s * s;
    const int ns = a.nside;
    const int nrm = a.nr_max;
    const bool active = lane < s3;
    const int ia = lane / (s * s), ib = (lane / s) % s, ic = lane % s;
    const float ca = ((float)ia + 0.5f) + (float)kJit0, cb = ((float)ib + 0.5f) + (float)kJit1,
                cc = ((float)ic + 0.5f) + (float)kJit2;
    const float inv_s = 1.0f / (float)s;
    const Real inv_s3 = (Real)1 / (Real)s3;
    const uint64_t act_mask = __ballot(active);
    // each below 256; bit 24: the node emits (two-point emission weights e0, e1)
    const int packed = lo | (nsup << 8) | (ie << 16) | ((e0 != (Real)0 || e1 != (Real)0) ? 1 << 24 : 0);
    const int epacked = emode | (le << 2) | (ne << 10) | (etop << 18);   // 2 + 8 + 8 + 8 bits
    // lanes of phase 2 cover (pixel slot, support point) pairs, span points per
    // slot: slot of a lane = (lane mx) >> 16 with mx = ceil(2^16 / span) (exact
    // for lanes below 64 and span <= 64), G = 64 / span slots per batch
    int divp;
    {
        const int span1 = nsup < 1 ? 1 : (nsup < 64 ? nsup : 64);
        divp = ((65536 + span1 - 1) / span1) | ((64 / span1) << 17);
    }
    // the W_p normalisation, or (no support point: linear split) minus the
    // bracket weight of the lower point
    const Real wsf = wscale > (Real)0 ? wscale : -fb0;
    // per node (lane = node): sub-box origin relative to the target and sub-box steps, FP32
    const float ox = 0.5f * (float)(2 * bx - tx), oy = 0.5f * (float)(2 * by - ty), oz = 0.5f * (float)(2 * bz - tz);
    const float sx = (float)ex * inv_s, sy = (float)ey * inv_s, sz = (float)ez * inv_s;
    // the table entries of the next node are fetched while one is mapped
    int next_kc = table_pairs(a.atab_pool, cnt > 0 ? rdlane(tab, 0) : -1, lane);
    for (int j = 0; j < cnt; ++j) {
        // --- angular: slot q (lane q of slot_kc) holds the q-th distinct pixel
        // and its sub-point count (pixel < 2^16, count <= 64), packed so that one
        // shuffle hands a slot to the lanes that scatter it; from the table, or
        // by classifying the node's sub-points ---
        int nd = 0, slot_kc = 0;
        const int jt = rdlane(tab, j);
        const int this_kc = next_kc;
        next_kc = table_pairs(a.atab_pool, j + 1 < cnt ? rdlane(tab, j + 1) : -1, lane);
        if (jt >= 0) {
            if (!PASS) {
                nd = jt & 127;
                if (lane < nd) slot_kc = this_kc;
            } else {
                // the pass's pixels only, as local ray indices
                const int nall = jt & 127;
                for (int q = 0; q < nall; ++q) {
                    const int kc = __builtin_amdgcn_readlane(this_kc, q);
                    const int kl = (kc & 0xffff) - k0;
                    if ((unsigned)kl < (unsigned)np) {
                        slot_kc = lane == nd ? (kl | (kc & ~0xffff)) : slot_kc;
                        ++nd;
                    }
                }
            }
            tab_count += lane == 0 ? 1.0 : 0.0;
        } else {
            // FP32 with a guard band, FP64 inside it: the FP64 classifier's pixel
            // for every sub-point, in both precisions
            const float vx = fmaf(ca, rdlane(sx, j), rdlane(ox, j));
            const float vy = fmaf(cb, rdlane(sy, j), rdlane(oy, j));
            const float vz = fmaf(cc, rdlane(sz, j), rdlane(oz, j));
            bool unsure = false;
            int pix = ang2pix_f(ns, vx, vy, vz, a.guard_tol, unsure);
            unsure &= active;
            if (__ballot(unsure)) {
                const int jbx = rdlane(bx, j), jby = rdlane(by, j), jbz = rdlane(bz, j);
                const int jex = rdlane(ex, j), jey = rdlane(ey, j), jez = rdlane(ez, j);
                if (unsure) {
                    pix = subpoint_pix_d(ns, s, jbx, jby, jbz, jex, jey, jez, tx, ty, tz, ia, ib, ic);
                    guard_count += 1.0;
                }
            }
            if ((unsigned)pix >= (unsigned)a.npix) {
                // cannot happen for a finite direction: reported, never written out of bounds
                atomicOr(&a.queue[1], 4);
                pix = 0;
            }
            // the distinct pixels
            uint64_t rem = act_mask;
            while (rem) {
                const int first = __ffsll((unsigned long long)rem) - 1;
                const int k = __builtin_amdgcn_readlane(pix, first);
                const uint64_t m = __ballot(pix == k) & rem;
                rem &= ~m;
                // (a pass keeps its own pixels, as local ray indices)
                if (!PASS || (unsigned)(k - k0) < (unsigned)np) {
                    const int kc = (k - k0) | ((int)__popcll(m) << 16);   // uniform
                    slot_kc = lane == nd ? kc : slot_kc;
                    ++nd;
                }
            }
        }
        // --- radial weights: this lane serves support point lo + io of batch slot po ---
        const int jpk = rdlane(packed, j);
        const int jlo = jpk & 255, jn = (jpk >> 8) & 255, jie = (jpk >> 16) & 255;
        const Real jd = rdlane(d, j), jhinv = rdlane(hinv, j), jwf = rdlane(wsf, j);
        const Real ja = rdlane(qa, j), je = rdlane(qe, j), jv = rdlane(qv, j);
        Real je0 = 0, je1 = 0;
        if ((jpk >> 24) & 1) {
            je0 = rdlane(e0, j);
            je1 = rdlane(e1, j);
        }
        const int jep = KV ? rdlane(epacked, j) : 0;
        const int jemode = jep & 3, jle = (jep >> 2) & 255, jne = (jep >> 10) & 255;
        const bool has_eps = je0 != (Real)0 || je1 != (Real)0 || jemode != 0;
        const int span = jn < 64 ? jn : 64;                         // points per batch slot
        const int jdv = rdlane(divp, j);
        const int G = jdv >> 17;                                    // pixels per batch
        const int po = (lane * (jdv & 0x1ffff)) >> 16;              // lane / span
        const int io = lane - po * span;
        const bool lane_ok = po < G;
        Real wa = 0, we = 0, wv = 0, wq = 0;   // wq: emission spread over the support (modes 1-3)
        const Real jfb = -jwf;                  // the bracket weight when there is no W_p support
        if (lane_ok) {
            Real w;
            if (jwf > (Real)0) {
                const int i = jlo + io;
                w = smooth_kernel<Real>(mg, (rcoef * (Real)(i * i) - jd) * jhinv) * jwf;
            } else {
                w = io == 0 ? jfb : (Real)1 - jfb;
            }
            wa = w * ja;
            we = w * je;
            wv = w * jv;
            if (KV && jemode != 0) wq = emission_weight<Real>(jemode, jlo + io, io, jle, jne, rdlane(ea, j), rdlane(eb, j),
                                                       jfb, rcoef, jd, jhinv, a.eps_kernel == K_G) *
                                  rdlane(qeps, j);
        }
        const int slot_k = slot_kc & 0xffff, slot_c = slot_kc >> 16;
        // emission: lane q deposits pixel q's share on the two bracket points and
        // marks them in the ray's mask (the spread forms go with A, E, V below)
        if (has_eps && lane < nd && jemode == 0) {
            const Real wk = (Real)slot_c * inv_s3;
            Real *row = &R.eps(slot_k, jie);
            if (je0 != (Real)0) buf_add<Real, EATOMIC>(row, wk * je0);
            if (je1 != (Real)0) buf_add<Real, EATOMIC>(row + 1, wk * je1);
            mark_points<ATOMIC != 0>(emask + (size_t)slot_k * ew, jie, je0 != (Real)0, je1 != (Real)0);
        }
        // A, E, V: lanes cover (pixel slot, point) pairs, G slots at a time
        for (int b0 = 0; b0 < nd; b0 += G) {
            const int q = b0 + po;
            const int kc = __shfl(slot_kc, q & 63, 64);
            const int kq = kc & 0xffff, cq = kc >> 16;
            if (lane_ok && q < nd) {
                const Real wk = (Real)cq * inv_s3;
                Real *row = &R.A(kq, jlo + io);
                buf_add3<Real, ATOMIC>(row, wk * wa, row + nrm, wk * we, row + 2 * nrm, wk * wv);
                if (KV && wq != (Real)0) {   // the emission row
                    buf_add<Real, EATOMIC>(&R.eps(kq, jlo + io), wk * wq);
                    mark_points<ATOMIC != 0>(emask + (size_t)kq * ew, jlo + io, true, false);
                }
            }
        }
        if (jn > 64) {
            // support wider than a wave (N_R > 64): the remaining points, pixel by pixel
            for (int q = 0; q < nd; ++q) {
                const int k = __builtin_amdgcn_readlane(slot_k, q);
                const Real wk = (Real)__builtin_amdgcn_readlane(slot_c, q) * inv_s3;
                Real *row = &R.A(k, jlo);
                for (int i2 = 64 + lane; i2 < jn; i2 += 64) {
                    const int i = jlo + i2;
                    const Real w2 =
                        jwf > (Real)0 ? smooth_kernel<Real>(mg, (rcoef * (Real)(i * i) - jd) * jhinv) * jwf : (Real)0;
                    buf_add<Real, ATOMIC>(row + i2, wk * w2 * ja);
                    buf_add<Real, ATOMIC>(row + nrm + i2, wk * w2 * je);
                    buf_add<Real, ATOMIC>(row + 2 * nrm + i2, wk * w2 * jv);
                    if (KV && jemode != 0) {
                        const Real q2 = emission_weight<Real>(jemode, i, i2, jle, jne, rdlane(ea, j), rdlane(eb, j), jfb,
                                                              rcoef, jd, jhinv, a.eps_kernel == K_G) *
                                        rdlane(qeps, j);
                        if (q2 != (Real)0) {
                            buf_add<Real, EATOMIC>(&R.eps(k, jlo + i2), wk * q2);
                            mark_points<ATOMIC != 0>(emask + (size_t)k * ew, jlo + i2, true, false);
                        }
                    }
                }
            }
        }
    }
}

// LDS flags of the per-target walk (acquire/release inside the workgroup)
__device__ inline int lds_load(const int *p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void lds_store(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP); }

// Breadth-first walk of one target by a single wave (Sec. 2.3, 2.4): a node
// containing the target is opened, every other leaf is accepted, other nodes
// are accepted when size^2 < theta^2 d^2 (geometric centre, doubled integer
// coordinates, the product taken in FP64).  Accepted nodes are appended to
// acc and published through sc[S_AVAIL] as each batch of tests completes, so
// the other waves map them while the walk goes on.
// S_PRE: the bank's item was claimed (and possibly walked, S_WALKED) ahead,
// during the previous target's integration
enum { S_ITEM = 0, S_AVAIL, S_CLAIM, S_DONE, S_OVF, S_TOTAL, S_PRE, S_WALKED,
       // a walk by several waves: the claim's generation, their meetings, the next
       // frontier's length (three by level), the accepted count, an overflow
       S_PGEN, S_PMEET, S_PNEXT, S_PACC = S_PNEXT + 3, S_POVF, S_COUNT = 16 };

// Waits until this wave's device-memory stores have completed (vmcnt 0), so
// that an LDS flag written next publishes them to the workgroup's other waves
// (a workgroup-scope release does not wait for them).
__device__ inline void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// dev_lists: acc is in device memory (the mappers read it after the LDS counts)
__device__ void walk_target(const SweepArgs &a, int root, const int *per, int tx, int ty, int tz, int *fr0, int *fr1,
                            int *acc, int *sc, int fmax, int amax, double &n_test, bool dev_lists)
{
    const int lane = lane_id();
    int *cur = fr0, *nxt = fr1;
    if (lane == 0) cur[0] = root;
    int nfr = 1, nacc = 0;
    bool ovf = false;
    while (nfr > 0 && !ovf) {
        int nn = 0;
        for (int base = 0; base < nfr; base += 64) {
            const int idx = base + lane;
            const bool valid = idx < nfr;
            int n = 0, nch = 0, fc = 0;
            bool acc_it = false;
            if (valid) {
                n = cur[idx];
                const int4 g = a.geo[n];
                const int2 tp = a.topo[n];
                const int sz = g.w & kSizeMask;
                const bool leaf = tp.y == 0;
                const bool inside = (2 * g.x <= tx && tx < 2 * (g.x + sz)) && (2 * g.y <= ty && ty < 2 * (g.y + sz)) &&
                                    (2 * g.z <= tz && tz < 2 * (g.z + sz));
                bool open_it = false;
                if (inside) {
                    open_it = !leaf;
                } else if (leaf) {
                    acc_it = true;
                } else {
                    int vx = 2 * g.x + sz - tx, vy = 2 * g.y + sz - ty, vz = 2 * g.z + sz - tz;
                    if (per) {
                        vx += 2 * nearest_copy_shift(vx, per[0]);
                        vy += 2 * nearest_copy_shift(vy, per[1]);
                        vz += 2 * nearest_copy_shift(vz, per[2]);
                    }
                    const double ddx = (double)vx, ddy = (double)vy, ddz = (double)vz;
                    const double D2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    double th2 = a.theta2;   // lowered by the IF and Src MACs (Sec. 2.4)
                    if ((g.w & kIfBit) && a.theta_if2 > 0.0) th2 = fmin(th2, a.theta_if2);
                    if ((g.w & kSrcBit) && a.theta_src2 > 0.0) th2 = fmin(th2, a.theta_src2);
                    acc_it = th2 * D2 > 4.0 * (double)sz * (double)sz;
                    open_it = !acc_it;
                }
                nch = open_it ? tp.y : 0;
                fc = tp.x;
            }
            n_test += valid ? 1.0 : 0.0;
            const uint64_t macc = __ballot(acc_it);
            const int cacc = __popcll(macc);
            int tot = 0;
            const int off = wave_excl_scan_dpp(nch, tot);
            if (nacc + cacc > amax || nn + tot > fmax) {
                ovf = true;
                break;
            }
            if (acc_it) acc[nacc + __popcll(macc & ((1ull << lane) - 1ull))] = n;
            for (int c = 0; c < nch; ++c) nxt[nn + off + c] = fc + c;
            nacc += cacc;
            nn += tot;
            if (cacc) {
                if (dev_lists) wait_stores();
                if (lane == 0) lds_store(&sc[S_AVAIL], nacc);
            }
        }
        int *t = cur;
        cur = nxt;
        nxt = t;
        nfr = nn;
    }
    if (dev_lists) wait_stores();
    if (lane == 0) {
        sc[S_TOTAL] = nacc;
        if (ovf) sc[S_OVF] = 1;
        lds_store(&sc[S_AVAIL], nacc);
        lds_store(&sc[S_DONE], 1);
    }
}

// The same walk by K waves (half 0 to K - 1) of one workgroup, into a list
// that is read only once the walk is done: the batches of 64 nodes of a level
// go round the waves, their appends to the next frontier and to the accepted
// list are reserved by LDS atomics, and the waves meet at an LDS counter after
// every level (all leave the loop at the same level).  sc[S_PMEET],
// sc[S_PNEXT], sc[S_PACC], sc[S_POVF] and cur[0] = root are set by half 0
// before any starts.  Half 0 publishes the list.
template <int K>
__device__ void walk_target_pair(const SweepArgs &a, int half, const int *per, int tx, int ty, int tz, int *fr0,
                                 int *fr1, int *acc, int *sc, int fmax, int amax, double &n_test, bool dev_lists)
{
    const int lane = lane_id();
    int *cur = fr0, *nxt = fr1;
    int nfr = 1;
    for (int lev = 0;; ++lev) {
        int *const next_count = &sc[S_PNEXT + lev % 3];
        // the counter of the level after next is free (read before the last meeting)
        if (half == 0 && lane == 0) sc[S_PNEXT + (lev + 1) % 3] = 0;
        for (int base = 64 * half; base < nfr; base += 64 * K) {
            const int idx = base + lane;
            const bool valid = idx < nfr;
            int n = 0, nch = 0, fc = 0;
            bool acc_it = false;
            if (valid) {
                n = cur[idx];
                const int4 g = a.geo[n];
                const int2 tp = a.topo[n];
                const int sz = g.w & kSizeMask;
                const bool leaf = tp.y == 0;
                const bool inside = (2 * g.x <= tx && tx < 2 * (g.x + sz)) && (2 * g.y <= ty && ty < 2 * (g.y + sz)) &&
                                    (2 * g.z <= tz && tz < 2 * (g.z + sz));
                bool open_it = false;
                if (inside) {
                    open_it = !leaf;
                } else if (leaf) {
                    acc_it = true;
                } else {
                    int vx = 2 * g.x + sz - tx, vy = 2 * g.y + sz - ty, vz = 2 * g.z + sz - tz;
                    if (per) {
                        vx += 2 * nearest_copy_shift(vx, per[0]);
                        vy += 2 * nearest_copy_shift(vy, per[1]);
                        vz += 2 * nearest_copy_shift(vz, per[2]);
                    }
                    const double ddx = (double)vx, ddy = (double)vy, ddz = (double)vz;
                    const double D2 = ddx * ddx + ddy * ddy + ddz * ddz;
                    double th2 = a.theta2;   // lowered by the IF and Src MACs (Sec. 2.4)
                    if ((g.w & kIfBit) && a.theta_if2 > 0.0) th2 = fmin(th2, a.theta_if2);
                    if ((g.w & kSrcBit) && a.theta_src2 > 0.0) th2 = fmin(th2, a.theta_src2);
                    acc_it = th2 * D2 > 4.0 * (double)sz * (double)sz;
                    open_it = !acc_it;
                }
                nch = open_it ? tp.y : 0;
                fc = tp.x;
            }
            n_test += valid ? 1.0 : 0.0;
            const uint64_t macc = __ballot(acc_it);
            const int cacc = __popcll(macc);
            int tot = 0;
            const int off = wave_excl_scan_dpp(nch, tot);
            int oa = 0, on = 0;
            if (lane == 0) {
                oa = cacc ? atomicAdd(&sc[S_PACC], cacc) : 0;
                on = tot ? atomicAdd(next_count, tot) : 0;
            }
            oa = __shfl(oa, 0, 64);
            on = __shfl(on, 0, 64);
            if (oa + cacc > amax || on + tot > fmax) {
                // nothing is written; all waves stop after this level's meeting
                if (lane == 0) sc[S_POVF] = lev + 1;
                continue;
            }
            if (acc_it) acc[oa + __popcll(macc & ((1ull << lane) - 1ull))] = n;
            for (int c = 0; c < nch; ++c) nxt[on + off + c] = fc + c;
        }
        // meet the other waves: the level's appends are all written
        if (dev_lists) wait_stores();
        if (lane == 0) atomicAdd(&sc[S_PMEET], 1);
        while (lds_load(&sc[S_PMEET]) < K * (lev + 1)) __builtin_amdgcn_s_sleep(1);
        nfr = uniform(lds_load(next_count));
        // (an overflow of the other wave's next level is not this level's)
        const int ov = uniform(lds_load(&sc[S_POVF]));
        if (nfr == 0 || (ov != 0 && ov <= lev + 1)) break;
        int *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (half == 0 && lane == 0) {
        // after an overflow the list has gaps: nothing is mapped (the target
        // goes to the second pass)
        const bool ovf = lds_load(&sc[S_POVF]) != 0;
        sc[S_TOTAL] = ovf ? 0 : lds_load(&sc[S_PACC]);
        if (ovf) sc[S_OVF] = 1;
        lds_store(&sc[S_AVAIL], sc[S_TOTAL]);
        lds_store(&sc[S_DONE], 1);
        sc[S_WALKED] = 1;
    }
}

// The sweep of one launch.  FALLBACK: the second pass over the items whose
// walk lists did not fit in LDS, with the lists in device memory.
template <typename Real, int WAVES, bool LDSBUF, bool FALLBACK, bool KV, bool CAS = false, bool PASS = false>
__device__ __forceinline__ void sweep_body(const SweepArgs &a)
{
    using R4 = typename R4T<Real>::T;
    constexpr int ATOMIC = WAVES == 1 ? 0 : (CAS ? 2 : 1);
    constexpr int CHUNK = 64;   // nodes claimed at a time by a mapping wave (one per lane in phase 1)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar loops over waves' work
    const int nrm = a.nr_max, npix = a.npix;
    // rays held at once (all of them, or a.pass_rays per pass)
    const int prays = PASS && a.pass_rays > 0 ? a.pass_rays : npix;
    const int npass = PASS ? (npix + prays - 1) / prays : 1;
    const size_t buf_elems = (size_t)prays * a.stride_k;
    char *p = smem;
    Real *buf;
    if constexpr (LDSBUF) {
        buf = (Real *)p;
        p += ((buf_elems * sizeof(Real) + 15) / 16) * 16;
    } else {
        buf = (Real *)a.gbuf + (size_t)blockIdx.x * buf_elems;
    }
    // split: three rows (A, E, V) per ray in buf, the emission rows in device memory
    const bool split = LDSBUF && a.split != 0;
    Real *const eplane = split ? (Real *)a.ebuf + (size_t)blockIdx.x * npix * nrm : buf;
    const RayRows<Real> R{buf, eplane, a.stride_k, split ? nrm : a.stride_k, split ? 0 : nrm, nrm};
    Real *rt = (Real *)p;
    p += ((nrm * sizeof(Real) + 15) / 16) * 16;
    Real *wself = (Real *)p;
    p += ((nrm * sizeof(Real) + 15) / 16) * 16;
    double *rd = (double *)p;   // the evaluation points in FP64 for the integration
    p += nrm * sizeof(double);
    double *rd2 = (double *)p;  // 1 / (2 r_i)
    p += nrm * sizeof(double);
    int *fr0, *fr1, *acc;
    int fmax, amax;
    if (FALLBACK) {
        int *gl = a.glist + (size_t)blockIdx.x * (2 * (size_t)a.gfmax + a.gamax);
        fmax = a.gfmax;
        amax = a.gamax;
        fr0 = gl;
        fr1 = gl + fmax;
        acc = gl + 2 * (size_t)fmax;
    } else {
        fmax = a.fmax;
        amax = a.amax;
        fr0 = (int *)p;
        p += fmax * sizeof(int);
        fr1 = (int *)p;
        p += fmax * sizeof(int);
        acc = (int *)p;
        p += amax * sizeof(int);
    }
    int *sc = (int *)p;   // two banks of S_COUNT: the current target's and the next one's
    p += 2 * S_COUNT * sizeof(int);
    double *red = (double *)p;
    p += WAVES * sizeof(double);
    // per ray: the mask of its points that hold emission (ew words)
    const int ew = nrm > 64 ? 2 : 1;
    unsigned long long *const emask = (unsigned long long *)p;

    double n_acc = 0, n_test = 0, n_guard = 0, n_f32 = 0, n_f64 = 0, n_tab = 0, n_re = 0;
    const int64_t n_items =
        FALLBACK ? min((int64_t)__hip_atomic_load(&a.queue[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), a.ovf_cap)
                   : a.n_items;

    // a bank takes the next work item with its walk counters reset
    auto claim = [&](int *b) {
        b[S_ITEM] = atomicAdd(&a.queue[FALLBACK ? 2 : 0], 1);
        b[S_AVAIL] = 0;
        b[S_CLAIM] = 0;
        b[S_DONE] = 0;
        b[S_OVF] = 0;
        b[S_TOTAL] = 0;
        b[S_WALKED] = 0;
    };
    if (tid == 0) {
        sc[S_PRE] = sc[S_COUNT + S_PRE] = 0;
        sc[S_PGEN] = sc[S_COUNT + S_PGEN] = 0;   // (generations start at 1)
    }
    int bank = 0;
    int titer = 0;   // targets begun by this workgroup (the generation of a shared walk's claim)
    int cached_dom = -1, cached_tsize = -1;   // whose radial tables the LDS holds
    for (;;) {
        int *const scb = sc + bank * S_COUNT;
        ++titer;
        __syncthreads();
        if (tid == 0) {
            if (!scb[S_PRE]) claim(scb);
            scb[S_PRE] = 0;
        }
        __syncthreads();
        const int64_t item = uniform(scb[S_ITEM]);   // the same on every lane: scalar loads below
        if (item >= n_items) break;
        const int64_t it = FALLBACK ? (int64_t)a.ovf[item] : item;
        const int64_t cell = a.targets ? a.targets[it] : (int64_t)a.order[it];
        const int64_t o = a.targets ? it : cell;   // output index
        if (cell < 0 || cell >= a.n_cells) {
            if (tid == 0) {
                a.f_out[o] = __longlong_as_double(0x7ff8000000000000ll);
                if (a.ion_out) a.ion_out[o] = 0;
                atomicOr(&a.queue[1], 2);
            }
            continue;
        }
        const int dom = a.cell_dom[cell];
        const DomDev D = a.doms[dom];
        const int nr = D.nr;
        const int tnode = a.cell_node[cell];
        const int4 tg = a.geo[tnode];
        const int tsize = tg.w & kSizeMask;
        // doubled target centre: exact integers
        const int tx = 2 * tg.x + tsize, ty = 2 * tg.y + tsize, tz = 2 * tg.z + tsize;
        const R4 tA = ((const R4 *)a.pA)[tnode];
        const R4 tB = ((const R4 *)a.pB)[tnode];
        const Real rc_inv = (Real)D.rc_inv;
        const Real rcoef = (Real)(1.0 / D.rc_inv);

        // evaluation points and the self-term weights (W_p at d = 0, h = cell size):
        // kept in LDS while consecutive targets share the domain and cell size
        if (dom != cached_dom) {
            for (int i = tid; i < nr; i += WAVES * 64) {
                const double rv = a.r64[D.r_off + i];
                rd[i] = rv;
                rd2[i] = i > 0 ? 1.0 / (2.0 * rv) : 0.0;
                if constexpr (sizeof(Real) == 4) rt[i] = a.r32[D.r_off + i];
                else rt[i] = (Real)rv;
            }
            __syncthreads();
        }
        if (dom != cached_dom || tsize != cached_tsize) {
            if (wave == 0) {
                Real w0 = 0, w1 = 0;
                if (lane < nr) w0 = smooth_kernel<Real>(KV && a.mass_gauss != 0, rt[lane] / (Real)tsize);
                if (lane + 64 < nr) w1 = smooth_kernel<Real>(KV && a.mass_gauss != 0, rt[lane + 64] / (Real)tsize);
                const Real sum = wave_sum(w0 + w1);
                if (lane < nr) wself[lane] = w0 / sum;
                if (lane + 64 < nr) wself[lane + 64] = w1 / sum;
            }
            __syncthreads();
            cached_dom = dom;
            cached_tsize = tsize;
        }
        double ftarget = 0.0;   // this lane's share of the target's flux over the passes
        // The rays k0 .. k0 + np - 1: all of them, or (PASS) one pass of prays
        // consecutive pixels at a time, the passes looping back here (a target
        // whose walk overflows leaves with continue).  Without passes there is
        // no loop, so the body compiles as straight-line code.
        int pass = 0;
    next_pass:
        {
            const int k0 = pass * prays, np = PASS ? min(prays, npix - k0) : npix;
            // ray buffer: zero emission, the target's own share of A, E, V
            {
                // every ray starts from the same 4 (split: 3) N_R values: lane l holds entries l + 64 m
                const Real inv_npix = (Real)1 / (Real)npix;
                const int per_ray = (split ? 3 : 4) * nrm;
                Real val[4 * kMaxRadial / 64];
#pragma unroll
                for (int m = 0; m < 4 * kMaxRadial / 64; ++m) {
                    const int e = lane + 64 * m;
                    const int row = e / nrm + (split ? 1 : 0), i = e - (e / nrm) * nrm;
                    Real v = (Real)0;
                    if (e < per_ray && row != Q_EPS && i < nr) {
                        const Real mom = row == Q_A ? tB.x : row == Q_E ? tB.y : tB.z;
                        v = mom * (wself[i] * inv_npix);
                    }
                    val[m] = v;
                }
                for (int k = wave; k < np; k += WAVES) {
                    Real *dst = buf + (size_t)k * a.stride_k;
#pragma unroll
                    for (int m = 0; m < 4 * kMaxRadial / 64; ++m)
                        if (64 * m < per_ray && lane + 64 * m < per_ray) dst[lane + 64 * m] = val[m];
                }
                for (int e = tid; e < np * ew; e += WAVES * 64) emask[e] = 0ull;
                // a later pass maps the same accepted nodes again
                if (pass > 0 && tid == 0) scb[S_CLAIM] = 0;
                // (the emission plane of split buffers is zero here: cleared when
                // allocated and, entry by entry, by the march that reads it)
            }
            __syncthreads();

            // --- wave 0 walks (unless the target was walked ahead); every wave maps ---
            const int *per = a.periodic ? D.ext : nullptr;
            if (pass == 0 && wave == 0 && !scb[S_WALKED])
                walk_target(a, D.root, per, tx, ty, tz, fr0, fr1, acc, scb, fmax, amax, n_test, FALLBACK);
            for (;;) {
                // claims of CHUNK nodes; once the walk is done, smaller ones near the
                // end of the list (a share of what is left), so the waves finish together
                int start = 0, size = CHUNK;
                if (lane == 0) {
                    if (lds_load(&scb[S_DONE])) {
                        const int left = lds_load(&scb[S_TOTAL]) - lds_load(&scb[S_CLAIM]);
                        size = min(CHUNK, max(4, left / (2 * WAVES)));
                    }
                    start = atomicAdd(&scb[S_CLAIM], size);
                }
                start = __shfl(start, 0, 64);
                size = __shfl(size, 0, 64);
                int end = 0;
                for (;;) {
                    const int avail = lds_load(&scb[S_AVAIL]);
                    if (avail >= start + size) {
                        end = start + size;
                        break;
                    }
                    if (lds_load(&scb[S_DONE])) {
                        const int total = lds_load(&scb[S_TOTAL]);
                        end = min(start + size, total);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                end = uniform(end);
                if (end <= start) break;
                map_nodes<Real, ATOMIC, KV, PASS>(a, R, emask, ew, per, rt, nr, rc_inv, rcoef, acc + start, end - start, tx, ty, tz,
                                            tsize, k0, np, n_guard, n_tab);
            }
            __syncthreads();
            if (scb[S_OVF]) {
                // the partly mapped emission is not integrated: clear the plane
                if (split)
                    for (int e = tid; e < npix * nrm; e += WAVES * 64) eplane[e] = (Real)0;
                if (tid == 0) {
                    bool queued = false;
                    if (!FALLBACK && a.ovf) {
                        const int q = atomicAdd(&a.queue[3], 1);
                        if (q < a.ovf_cap) {
                            a.ovf[q] = (int32_t)item;
                            queued = true;
                        }
                    }
                    if (!queued) {
                        a.f_out[o] = __longlong_as_double(0x7ff8000000000000ll);
                        if (a.ion_out) a.ion_out[o] = 0;
                        atomicOr(&a.queue[1], 1);
                    }
                }
                continue;
            }
            if (pass == 0) n_acc += (wave == 0 && lane == 0) ? (double)scb[S_TOTAL] : 0.0;

            // --- per-ray integration and the sum over rays (rays without emission give 0),
            // by waves 0 .. IW - 1; the others meanwhile walk the next target ---
            // (at 16 waves the last four walk it, else the last one: with fewer waves
            // one more integrating wave is worth more than a faster walk; at 16 the
            // walk on fewer waves outlasts the integration, on more it slows it)
            constexpr int kWalk = WAVES >= 16 ? 4 : 1;   // waves that walk the next target
            constexpr bool kPair = kWalk > 1;
            constexpr int IW = kPair ? WAVES - kWalk : (WAVES > 1 ? WAVES - 1 : 1);
            double fsum = 0.0;
            float cs_hi = 0.0f, cs_lo = 0.0f;   // compensated FP32 sum of this lane's FP32-marched rays
            if (wave >= IW) {
                // no rays here
            } else if (a.int_group > 0) {
                // Every emitting ray gets a group of lanes sized by its number of
                // emitting points: a power of two from the launch's group up to 64
                // (its class), more than 64 points a wave (class 7).  Rays of one
                // class share a batch of 64 / g rays of g lanes; the batches, widest
                // class first and pixel order within a class, are dealt round robin
                // over the waves.
                const int lg0 = 31 - __clz(a.int_group);
                int nb[6];   // batches of classes 2 .. 7 (class 7: a ray each)
                {
                    int n[6] = {0, 0, 0, 0, 0, 0};
                    for (int base = 0; base < np; base += 64) {
                        int tp;
                        const int c = ray_class(emask, ew, np, lg0, base + lane, tp);
#pragma unroll
                        for (int q = 0; q < 6; ++q) n[q] += (int)__popcll(__ballot(c == q + 2));
                    }
                    int re = 0;
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        nb[q] = q == 5 ? n[q] : (n[q] + (64 >> (q + 2)) - 1) >> (4 - q);
                        if (q + 2 > lg0) re += n[q];
                    }
                    n_re += (wave == 0 && lane == 0) ? (double)re : 0.0;
                }
                const int n_batch = nb[0] + nb[1] + nb[2] + nb[3] + nb[4] + nb[5];
                for (int b = wave; b < n_batch; b += IW) {
                    int cls = -1, bi = b;
#pragma unroll
                    for (int q = 5; q >= 0; --q)
                        if (cls < 0) {
                            if (bi < nb[q]) cls = q + 2;
                            else bi -= nb[q];
                        }
                    const int ng = cls == 7 ? 1 : 64 >> cls;
                    // this lane's ray: the (bi ng + lane / g)-th of the class
                    const int want = bi * ng + (cls == 7 ? 0 : lane >> cls);
                    int myk = -1, mytp = 0, run = 0;
                    for (int base = 0; base < np && run < bi * ng + ng; base += 64) {
                        int tp;
                        const int c = ray_class(emask, ew, np, lg0, base + lane, tp);
                        const uint64_t m = __ballot(c == cls);
                        const int n = (int)__popcll(m), w = want - run;
                        const bool mine = w >= 0 && w < n;
                        const int pos = mine ? nth_set_bit(m, w) : 0;
                        const int tv = __shfl(tp, pos, 64);
                        if (mine) {
                            myk = base + pos;
                            mytp = tv;
                        }
                        run += n;
                    }
                    if (cls == 7) {
                        const double fw = integrate_ray_wave<Real, 2>(R, myk, rd, rd2, nr, mytp, a.nside, a.zeta_g, split);
                        if (lane == 0) fsum += fw;
                        continue;
                    }
                    // the ray's mask, for its group's lanes to find their emitting points
                    unsigned long long m0 = 0ull, m1 = 0ull;
                    if (myk >= 0) {
                        m0 = emask[(size_t)myk * ew];
                        if (ew > 1) m1 = emask[(size_t)myk * ew + 1];
                    }
                    switch (cls) {
                        case 2: march_batch<Real, 4>(a, R, myk, m0, m1, rcoef, rd, rd2, nr, split, fsum, cs_hi, cs_lo, n_f32, n_f64); break;
                        case 3: march_batch<Real, 8>(a, R, myk, m0, m1, rcoef, rd, rd2, nr, split, fsum, cs_hi, cs_lo, n_f32, n_f64); break;
                        case 4: march_batch<Real, 16>(a, R, myk, m0, m1, rcoef, rd, rd2, nr, split, fsum, cs_hi, cs_lo, n_f32, n_f64); break;
                        case 5: march_batch<Real, 32>(a, R, myk, m0, m1, rcoef, rd, rd2, nr, split, fsum, cs_hi, cs_lo, n_f32, n_f64); break;
                        default: march_batch<Real, 64>(a, R, myk, m0, m1, rcoef, rd, rd2, nr, split, fsum, cs_hi, cs_lo, n_f32, n_f64); break;
                    }
                }
            } else if (a.int_wave) {
                // a wave per ray, the emitting rays dealt round robin over the waves
                int seen = 0;
                for (int base = 0; base < np; base += 64) {
                    int t = 0;
                    if (base + lane < np)
                        t = mask_top(emask[(size_t)(base + lane) * ew], ew > 1 ? emask[(size_t)(base + lane) * ew + 1] : 0ull);
                    uint64_t m = __ballot(t > 0);
                    while (m) {
                        const int l = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        if (seen % IW == wave) {
                            const int tk = __builtin_amdgcn_readlane(t, l);
                            const double f =
                                nr > 64 ? integrate_ray_wave<Real, 2>(R, base + l, rd, rd2, nr, tk, a.nside, a.zeta_g, split)
                                        : integrate_ray_wave<Real, 1>(R, base + l, rd, rd2, nr, tk, a.nside, a.zeta_g, split);
                            if (lane == 0) fsum += f;
                        }
                        ++seen;
                    }
                }
            } else {
                // a lane per ray: ray k on lane k % 64 of wave (k / 64) % IW
                for (int k = wave * 64 + lane; k < np; k += 64 * IW) {
                    const int t = mask_top(emask[(size_t)k * ew], ew > 1 ? emask[(size_t)k * ew + 1] : 0ull);
                    if (t > 0) fsum += integrate_ray<Real>(R, k, rd, rd2, nr, t, a.nside, a.zeta_g, split);
                }
            }
            // the next target: claimed and walked into the other bank by the last
            // wave, or the last four (the node lists and that bank are not in use
            // until the next barrier)
            if ((kPair ? wave >= WAVES - kWalk : wave == WAVES - 1) && pass == npass - 1) {
                int *const nsc = sc + (bank ^ 1) * S_COUNT;
                const int half = WAVES - 1 - wave;
                if (half == 0) {
                    if (lane == 0) {
                        claim(nsc);
                        nsc[S_PRE] = 1;
                    }
                } else {
                    // half 0's claim of this generation
                    while (lds_load(&nsc[S_PGEN]) != titer) __builtin_amdgcn_s_sleep(1);
                }
                const int64_t nitem = uniform(lds_load(&nsc[S_ITEM]));
                bool walk = false;
                int ndom = 0, ntx = 0, nty = 0, ntz = 0;
                if (nitem < n_items) {
                    const int64_t nit = FALLBACK ? (int64_t)a.ovf[nitem] : nitem;
                    const int64_t ncell = a.targets ? a.targets[nit] : (int64_t)a.order[nit];
                    if (ncell >= 0 && ncell < a.n_cells) {
                        walk = true;
                        ndom = a.cell_dom[ncell];
                        const int4 ng = a.geo[a.cell_node[ncell]];
                        const int nsz = ng.w & kSizeMask;
                        ntx = 2 * ng.x + nsz;
                        nty = 2 * ng.y + nsz;
                        ntz = 2 * ng.z + nsz;
                    }
                }
                const int *nper = a.periodic ? a.doms[ndom].ext : nullptr;
                if (!kPair) {
                    if (walk) {
                        walk_target(a, a.doms[ndom].root, nper, ntx, nty, ntz, fr0, fr1, acc, nsc, fmax, amax, n_test,
                                    FALLBACK);
                        if (lane == 0) nsc[S_WALKED] = 1;
                    }
                } else {
                    if (half == 0) {
                        if (lane == 0) {
                            nsc[S_PMEET] = 0;
                            nsc[S_PNEXT] = 0;
                            nsc[S_PACC] = 0;
                            nsc[S_POVF] = 0;
                            if (walk) fr0[0] = a.doms[ndom].root;
                        }
                        if (FALLBACK) wait_stores();   // (fr0 in device memory)
                        if (lane == 0) lds_store(&nsc[S_PGEN], titer);
                    }
                    if (walk)
                        walk_target_pair<kWalk>(a, half, nper, ntx, nty, ntz, fr0, fr1, acc, nsc, fmax, amax, n_test,
                                                FALLBACK);
                }
            }
            ftarget += fsum + ((double)cs_hi + (double)cs_lo);
        }
        if (PASS && ++pass < npass) {
            __syncthreads();   // the next pass re-initialises the buffers
            goto next_pass;
        }
        const double fsum = wave_sum(ftarget);
        if (lane == 0) red[wave] = fsum;
        __syncthreads();
        if (tid == 0) {
            double f = 0.0;
            for (int w = 0; w < WAVES; ++w) f += red[w];
            const double rtp = 0.5 * (double)tsize;
            f += 3.0 * (double)tA.w / (4.0 * kPi * rtp * rtp);
            a.f_out[o] = f * D.flux_unit;
            if (a.ion_out) a.ion_out[o] = f > 0.0 ? 1 : 0;
        }
        bank ^= 1;
    }
    // statistics
    n_test = wave_sum(n_test);
    n_guard = wave_sum(n_guard);
    n_f32 = wave_sum(n_f32);
    n_f64 = wave_sum(n_f64);
    n_tab = wave_sum(n_tab);
    n_re = wave_sum(n_re);
    if (lane == 0) {
        if (wave == 0 && n_acc > 0) atomicAdd(&a.stats[0], (unsigned long long)n_acc);
        if (n_test > 0) atomicAdd(&a.stats[1], (unsigned long long)n_test);
        if (n_guard > 0) atomicAdd(&a.stats[2], (unsigned long long)n_guard);
        if (n_f32 > 0) atomicAdd(&a.stats[3], (unsigned long long)n_f32);
        if (n_f64 > 0) atomicAdd(&a.stats[4], (unsigned long long)n_f64);
        if (n_tab > 0) atomicAdd(&a.stats[5], (unsigned long long)n_tab);
        if (n_re > 0) atomicAdd(&a.stats[6], (unsigned long long)n_re);
    }
}

template <typename Real, int WAVES, bool LDSBUF>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep(SweepArgs a)
{
    sweep_body<Real, WAVES, LDSBUF, false, false>(a);
}

template <typename Real, int WAVES, bool LDSBUF>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_fallback(SweepArgs a)
{
    sweep_body<Real, WAVES, LDSBUF, true, false>(a);
}

// the same with the radial-kernel variants (fewer launch shapes)
template <typename Real, int WAVES, bool LDSBUF>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_kv(SweepArgs a)
{
    sweep_body<Real, WAVES, LDSBUF, false, true>(a);
}

template <typename Real, int WAVES, bool LDSBUF>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_kv_fallback(SweepArgs a)
{
    sweep_body<Real, WAVES, LDSBUF, true, true>(a);
}

// FP32 ray buffers in LDS accumulated by compare-and-swap (8 and 16 waves)
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_cas(SweepArgs a)
{
    sweep_body<float, WAVES, true, false, false, true>(a);
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_cas_fallback(SweepArgs a)
{
    sweep_body<float, WAVES, true, true, false, true>(a);
}

// LDS ray buffers for part of a target's rays at a time (passes)
template <typename Real, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_pass(SweepArgs a)
{
    sweep_body<Real, WAVES, true, false, false, false, true>(a);
}
template <typename Real, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 4) void k_sweep_pass_fallback(SweepArgs a)
{
    sweep_body<Real, WAVES, true, true, false, false, true>(a);
}

// ---------------------------------------------------------------------------
// a9. delta_cell per domain.  The median is the lower median of the domain's
// previous flux, found exactly by an 8-pass radix select over the IEEE bit
// patterns (non-negative doubles order like their bits).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Angular-weight table (Sec. 2.3 "Mapping nodes onto rays").  A node's
// angular weights depend only on its box relative to the target; for nodes of
// 1, 2 or 4 times the target's size they are tabulated once per context by
// offset, in units of the target's size, with the FP64 classifier the sweep
// itself uses: relative sub-point positions scale exactly with the size, so a
// table entry holds exactly what the sweep would compute for that node.  One
// thread per offset; first the number of distinct pixels, then (after a
// prefix sum on the host) the pairs themselves, in the order of first
// appearance over the sub-points.
// ---------------------------------------------------------------------------
struct AtabGeom {
    int32_t w[kAtabRatios], base[kAtabRatios], nkeys;
};

__device__ inline void atab_key(const AtabGeom &G, int key, int &r, int &ox, int &oy, int &oz)
{
    int ri = 0;
    while (ri + 1 < kAtabRatios && key >= G.base[ri + 1]) ++ri;
    int k = key - G.base[ri];
    const int w = G.w[ri], n = 2 * w + 1;
    oz = k % n - w;
    k /= n;
    oy = k % n - w;
    ox = k / n - w;
    r = 1 << ri;
}

__device__ int atab_pairs(const AtabGeom &G, int key, int ns, int s, int *pix, int *cnt)
{
    int r, ox, oy, oz;
    atab_key(G, key, r, ox, oy, oz);
    int npl = 0;
    for (int ia = 0; ia < s; ++ia)
        for (int ib = 0; ib < s; ++ib)
            for (int ic = 0; ic < s; ++ic) {
                // a unit target with its lower corner at the origin: twice its centre is (1, 1, 1)
                const int p = subpoint_pix_d(ns, s, ox, oy, oz, r, r, r, 1, 1, 1, ia, ib, ic);
                int q = 0;
                while (q < npl && pix[q] != p) ++q;
                if (q == npl) {
                    pix[npl] = p;
                    cnt[npl] = 0;
                    ++npl;
                }
                ++cnt[q];
            }
    return npl;
}

__global__ void k_atab_count(AtabGeom G, int ns, int s, int32_t *npairs)
{
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= G.nkeys) return;
    int pix[64], cnt[64];
    npairs[key] = atab_pairs(G, key, ns, s, pix, cnt);
}

__global__ void k_atab_fill(AtabGeom G, int ns, int s, const int32_t *__restrict__ first, int32_t *idx,
                            int32_t *pool)
{
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= G.nkeys) return;
    int pix[64], cnt[64];
    const int n = atab_pairs(G, key, ns, s, pix, cnt);
    const int f = first[key];
    for (int q = 0; q < n; ++q) pool[f + q] = pix[q] | (cnt[q] << 16);
    idx[key] = (f << 7) | n;
}

// The domain of a cell: from the per-cell array of a context, or from the
// cell ranges of at most kStaticDomains domains (the entry point without a
// context), found by bisection.
constexpr int kStaticDomains = 64;
struct DomByArray {
    const int32_t *cell_dom;
    __device__ int operator()(int64_t c) const { return cell_dom[c]; }
};
struct DomByRanges {
    int32_t n;
    int64_t off[kStaticDomains + 1];   // domain d holds cells [off[d], off[d+1])
    __device__ int operator()(int64_t c) const
    {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
};

template <typename DomOf>
__global__ void k_hist(int64_t n_cells, const double *__restrict__ f, DomOf dom_of,
                       const unsigned long long *__restrict__ prefix, int shift, unsigned int *__restrict__ hist)
{
    __shared__ unsigned int h[256];
    const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t c = b0 + threadIdx.x;
    const int64_t last = (b0 + blockDim.x - 1 < n_cells ? b0 + blockDim.x - 1 : n_cells - 1);
    const int dom0 = dom_of(b0), dom1 = dom_of(last);
    const bool one = dom0 == dom1;   // whole block in one domain: count in LDS first
    for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    if (c < n_cells) {
        const int dom = dom_of(c);
        const unsigned long long key = (unsigned long long)__double_as_longlong(f[c]);
        const unsigned long long mask = (shift >= 56) ? 0ull : (~0ull << (shift + 8));
        if ((key & mask) == prefix[dom]) {
            const unsigned int digit = (unsigned int)((key >> shift) & 255ull);
            if (one) atomicAdd(&h[digit], 1u);
            else atomicAdd(&hist[dom * 256 + digit], 1u);
        }
    }
    __syncthreads();
    if (one)
        for (int i = threadIdx.x; i < 256; i += blockDim.x)
            if (h[i]) atomicAdd(&hist[dom0 * 256 + i], h[i]);
}

__global__ void k_select(int n_dom, int shift, unsigned int *hist, unsigned long long *prefix,
                         unsigned long long *rank)
{
    const int dom = blockIdx.x * blockDim.x + threadIdx.x;
    if (dom >= n_dom) return;
    unsigned long long k = rank[dom];
    unsigned long long cum = 0;
    int b = 0;
    for (; b < 256; ++b) {
        const unsigned int h = hist[dom * 256 + b];
        if (cum + h > k) break;
        cum += h;
    }
    if (b > 255) b = 255;
    rank[dom] = k - cum;
    prefix[dom] |= ((unsigned long long)b) << shift;
    for (int q = 0; q < 256; ++q) hist[dom * 256 + q] = 0;
}

__global__ void k_rank_init(int n_dom, const DomDev *__restrict__ doms, unsigned long long *rank,
                            unsigned long long *prefix, unsigned long long *dmax)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_dom) return;
    rank[d] = (unsigned long long)((doms[d].n_cells - 1) / 2);   // lower median
    prefix[d] = 0ull;
    dmax[d] = 0ull;
}

__global__ void k_rank_init_ranges(DomByRanges R, unsigned long long *rank, unsigned long long *prefix,
                                   unsigned long long *dmax)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= R.n) return;
    rank[d] = (unsigned long long)((R.off[d + 1] - R.off[d] - 1) / 2);   // lower median
    prefix[d] = 0ull;
    dmax[d] = 0ull;
}

template <typename DomOf>
__global__ void k_delta(int64_t n_cells, const double *__restrict__ fn, const double *__restrict__ fo,
                        DomOf dom_of, const unsigned long long *__restrict__ med,
                        unsigned long long *__restrict__ dmax)
{
    __shared__ unsigned long long wmax[16];
    const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t c = b0 + threadIdx.x;
    const int64_t last = (b0 + blockDim.x - 1 < n_cells ? b0 + blockDim.x - 1 : n_cells - 1);
    const int dom0 = dom_of(b0);
    const bool one = dom0 == dom_of(last);
    unsigned long long key = 0;   // bits of a non-negative double order like the value
    int dom = dom0;
    if (c < n_cells) {
        dom = dom_of(c);
        const double m = __longlong_as_double((long long)med[dom]);
        const double old = fo[c];
        const double norm = old > m ? old : m;
        const double diff = fabs(fn[c] - old);
        double dl;
        if (norm > 0.0) dl = diff / norm;
        else dl = diff > 0.0 ? INFINITY : 0.0;
        if (!(dl == dl)) dl = INFINITY;
        key = (unsigned long long)__double_as_longlong(dl);
    }
    if (!one) {
        if (c < n_cells) atomicMax(&dmax[dom], key);
        return;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(key, o, 64);
        key = y > key ? y : key;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long mx = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = wmax[w] > mx ? wmax[w] : mx;
        atomicMax(&dmax[dom0], mx);
    }
}

// the per-domain maxima (bit patterns of non-negative doubles) as doubles
__global__ void k_store_delta(int n_dom, const unsigned long long *__restrict__ dmax, double *__restrict__ out)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < n_dom) out[d] = __longlong_as_double((long long)dmax[d]);
}

// Scratch of the entry point without allocation (tr_delta_noalloc): per
// domain a 256-bin histogram, the median's bit prefix, the rank still to
// skip and the running maximum.  One copy per device, held until the
// process ends; every call on a device shares it.
constexpr size_t kStaticScratchWords = (size_t)kStaticDomains * 128 + 3 * kStaticDomains;
static __device__ __align__(256) unsigned long long scratch[kStaticScratchWords];

}  // namespace tr

// ===========================================================================
// Host side: the context and the C ABI
// ===========================================================================
using namespace tr;

struct tr_ctx {
    tr_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 0;
    std::string err;
    // domains
    std::vector<DomTopo> topo;
    std::vector<DomDev> domh;
    int32_t n_dom = 0;
    int64_t n_cells = 0, n_nodes = 0;
    int32_t depth_max = 0, nr_max = 0;
    std::vector<int64_t> level_begin;   // global level ranges [L, L+1)
    // device arrays
    int4 *geo = nullptr, *olo = nullptr, *oext = nullptr;
    int2 *topo_d = nullptr;
    int32_t *cell_node = nullptr, *cell_dom = nullptr, *order = nullptr;
    DomDev *doms = nullptr;
    double *r64 = nullptr;
    float *r32 = nullptr;
    double *mom = nullptr;
    void *packA = nullptr, *packB = nullptr;
    double *ndot = nullptr;
    // sources
    std::vector<std::vector<double>> sxyz, sq;
    double *d_sxyz = nullptr, *d_sq = nullptr;
    int32_t *d_sdom = nullptr;
    int32_t n_src_dev = 0;
    bool src_dirty = true;
    double rate_unit = 1.0;
    // sweep state
    int32_t *queue = nullptr;
    unsigned long long *stats = nullptr;
    int32_t *err_flags = nullptr;
    void *gbuf = nullptr;
    size_t gbuf_bytes = 0;
    void *ebuf = nullptr;   // emission rows of split LDS buffers
    size_t ebuf_bytes = 0;
    int32_t *glist = nullptr;            // walk lists of the fallback pass
    int32_t *ovf = nullptr;              // items queued for it
    int64_t ovf_cap = 0;
    // angular-weight table (built in tr_set_domains)
    int32_t *atab_idx = nullptr, *atab_pool = nullptr;
    AtabGeom atab{};
    // delta scratch
    unsigned int *hist = nullptr;
    unsigned long long *dprefix = nullptr, *drank = nullptr, *dmax = nullptr;
    double *solve_tmp = nullptr;
    int64_t solve_tmp_n = 0;
    // state
    bool built = false;
    tr_precision built_prec = TR_FP64;
    int32_t waves = 0, tpc = 0, bufmode = 0, intmode = 0, atommode = 0;   // user launch shape (0 = default)
    int32_t last_waves = 0, last_tpc = 0, last_lds = 0, last_intw = 0, last_cas = 0, last_int32 = 0;
    int tuned_waves[2] = {0, 0};         // per precision after tr_autotune
    int tuned_buf[2] = {0, 0};
    int tuned_int[2] = {0, 0};
    int tuned_atom[2] = {0, 0};
    float last_ms = 0.f;
    bool timed_valid = false;            // ev0/ev1 bracket a recorded sweep
    // one outer iteration captured as a hipGraph (tr_step)
    // (two cached graphs, so that an iteration alternating between two
    // buffers replays instead of capturing again)
    struct GraphSlot {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        const void *key[4] = {nullptr, nullptr, nullptr, nullptr};
        uint64_t used = 0;
    } gslot[2];
    uint64_t graph_clock = 0;
    hipStream_t cap_stream = nullptr;
    void *pinned = nullptr;              // host copies of the flags and deltas
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

tr_status fail(tr_ctx *c, tr_status s, const std::string &m)
{
    if (c) c->err = m;
    return s;
}

#define HIPCHK(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(c, TR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
    } while (0)

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void drop_slot(tr_ctx::GraphSlot &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = tr_ctx::GraphSlot();
}

void drop_graph(tr_ctx *c)
{
    for (auto &g : c->gslot) drop_slot(g);
}

void free_domains(tr_ctx *c)
{
    drop_graph(c);
    dfree(c->geo); dfree(c->olo); dfree(c->oext); dfree(c->topo_d);
    dfree(c->cell_node); dfree(c->cell_dom); dfree(c->order); dfree(c->doms);
    dfree(c->r64); dfree(c->r32); dfree(c->mom); dfree(c->packA); dfree(c->packB);
    dfree(c->ndot); dfree(c->d_sxyz); dfree(c->d_sq); dfree(c->d_sdom);
    dfree(c->hist); dfree(c->dprefix); dfree(c->drank); dfree(c->dmax);
    dfree(c->atab_idx); dfree(c->atab_pool);
    dfree(c->solve_tmp);
    dfree(c->gbuf);
    c->gbuf_bytes = 0;
    dfree(c->ebuf);
    c->ebuf_bytes = 0;
    dfree(c->glist);
    dfree(c->ovf);
    c->ovf_cap = 0;
    c->solve_tmp_n = 0;
    c->built = false;
}

tr_status check_params(tr_ctx *c, const tr_params &p)
{
    if (p.nside < 1 || p.nside > 64 || (p.nside & (p.nside - 1))) return fail(c, TR_EINVAL, "nside must be a power of two in [1, 64]");
    if (p.n_radial < 0 || p.n_radial == 1 || p.n_radial == 2 || p.n_radial > kMaxRadial)
        return fail(c, TR_EINVAL, "n_radial must be 0 or in [3, 128]");
    if (p.n_radial == 0 && !(p.eta_r > 0)) return fail(c, TR_EINVAL, "eta_r must be > 0");
    if (!(p.theta >= 0) || !std::isfinite(p.theta)) return fail(c, TR_EINVAL, "theta must be >= 0");
    if (!std::isfinite(p.theta_if) || !std::isfinite(p.theta_src))
        return fail(c, TR_EINVAL, "theta_if and theta_src must be finite");
    if (!(p.src_radius_cm >= 0) || !std::isfinite(p.src_radius_cm))
        return fail(c, TR_EINVAL, "src_radius_cm must be >= 0");
    if (p.eps_kernel < 0 || p.eps_kernel > 6) return fail(c, TR_EINVAL, "eps_kernel must be in [0, 6]");
    if (p.mass_kernel != 0 && p.mass_kernel != 5 && p.mass_kernel != 6)
        return fail(c, TR_EINVAL, "mass_kernel must be 0, 5 (W_p) or 6 (W_g)");
    if (!(p.alpha_b >= 0) || !std::isfinite(p.alpha_b)) return fail(c, TR_EINVAL, "alpha_b must be >= 0");
    if (p.subsample < 1 || p.subsample > 4) return fail(c, TR_EINVAL, "subsample must be in [1, 4]");
    if (p.max_iter < 0) return fail(c, TR_EINVAL, "max_iter must be >= 0");
    if (!(p.eps_lim >= 0)) return fail(c, TR_EINVAL, "eps_lim must be >= 0");
    if (p.precision != TR_FP64 && p.precision != TR_FP32C) return fail(c, TR_EINVAL, "unknown precision");
    return TR_OK;
}

inline unsigned grid1(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

template <typename T>
tr_status upload(tr_ctx *c, T *&dst, const std::vector<T> &src)
{
    dfree(dst);
    if (src.empty()) return TR_OK;
    if (hipMalloc((void **)&dst, src.size() * sizeof(T)) != hipSuccess) return fail(c, TR_ENOMEM, "hipMalloc failed");
    HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return TR_OK;
}

tr_status dalloc(tr_ctx *c, void **p, size_t bytes)
{
    if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) return fail(c, TR_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return TR_OK;
}

// LDS bytes of one sweep workgroup (must mirror the carve-up in k_sweep)
size_t sweep_lds_bytes(size_t real, int npix, int stride_k, int nrm, int fmax, int amax, int waves, bool ldsbuf)
{
    size_t b = 0;
    if (ldsbuf) b += (((size_t)npix * stride_k * real + 15) / 16) * 16;
    b += 2 * (((size_t)nrm * real + 15) / 16) * 16;
    b += 2 * (size_t)nrm * 8;
    b += 2 * (size_t)fmax * 4 + (size_t)amax * 4;
    b += 2 * 16 * 4;
    b += (size_t)waves * 8;
    b += (size_t)npix * 8 * (nrm > 64 ? 2 : 1);
    return b;
}

constexpr size_t kLdsMax = 160 * 1024;

using KernelFn = void (*)(SweepArgs);

template <typename Real>
KernelFn pick_kernel_kv(int waves, bool ldsbuf, bool fallback)
{
    if (waves == 4) {
        if (fallback) return ldsbuf ? (KernelFn)k_sweep_kv_fallback<Real, 4, true> : (KernelFn)k_sweep_kv_fallback<Real, 4, false>;
        return ldsbuf ? (KernelFn)k_sweep_kv<Real, 4, true> : (KernelFn)k_sweep_kv<Real, 4, false>;
    }
    if (waves == 8) {
        if (fallback) return ldsbuf ? (KernelFn)k_sweep_kv_fallback<Real, 8, true> : (KernelFn)k_sweep_kv_fallback<Real, 8, false>;
        return ldsbuf ? (KernelFn)k_sweep_kv<Real, 8, true> : (KernelFn)k_sweep_kv<Real, 8, false>;
    }
    return nullptr;
}

template <typename Real>
KernelFn pick_kernel_pass(int waves, bool fallback)
{
    if (waves == 4) return fallback ? (KernelFn)k_sweep_pass_fallback<Real, 4> : (KernelFn)k_sweep_pass<Real, 4>;
    if (waves == 8) return fallback ? (KernelFn)k_sweep_pass_fallback<Real, 8> : (KernelFn)k_sweep_pass<Real, 8>;
    if (waves == 16) return fallback ? (KernelFn)k_sweep_pass_fallback<Real, 16> : (KernelFn)k_sweep_pass<Real, 16>;
    return nullptr;
}

KernelFn pick_kernel_cas(int waves, bool fallback)
{
    if (waves == 8) return fallback ? (KernelFn)k_sweep_cas_fallback<8> : (KernelFn)k_sweep_cas<8>;
    return fallback ? (KernelFn)k_sweep_cas_fallback<16> : (KernelFn)k_sweep_cas<16>;
}

template <typename Real>
KernelFn pick_kernel(int waves, bool ldsbuf, bool fallback)
{
#define TR_CASE(W)                                                                                      \
    case W:                                                                                             \
        if (fallback)                                                                                   \
            return ldsbuf ? (KernelFn)k_sweep_fallback<Real, W, true> : (KernelFn)k_sweep_fallback<Real, W, false>; \
        return ldsbuf ? (KernelFn)k_sweep<Real, W, true> : (KernelFn)k_sweep<Real, W, false>;
    switch (waves) {
        TR_CASE(1)
        TR_CASE(2)
        TR_CASE(4)
        TR_CASE(8)
        TR_CASE(16)
        default:
            return nullptr;
    }
#undef TR_CASE
}

struct LaunchPlan {
    KernelFn fn = nullptr, fn_fb = nullptr;
    int waves = 0, blocks = 0, per_cu = 0, fmax = 0, amax = 0, stride_k = 0;
    size_t lds = 0;
    bool ldsbuf = true;
    bool cas = false;   // FP32 LDS buffers accumulated by compare-and-swap
    bool split = false; // A, E, V rows in LDS, emission rows in device memory
    int pass_rays = 0;  // > 0: four rows per ray in LDS for this many rays at a time (passes)
    int intm = 1;   // integration: 1 a lane per ray, 2 a wave per ray, 3/4/5 a group of 4/8/16 lanes,
                    // 6/7/8 the same groups with the FP32 march (FP32 buffers only)
};

// lanes that integrate one ray in integration mode m
inline int lanes_per_ray(int m) { return m == 2 ? 64 : (m >= 3 ? 4 << ((m - 3) % 3) : 1); }

tr_status plan_sweep(tr_ctx *c, int64_t n_items, int waves_req, int tpc_req, int buf_req, int int_req, LaunchPlan &L,
                     int atom_req = 0)
{
    const bool f32 = c->p.precision == TR_FP32C;
    const size_t real = f32 ? 4 : 8;
    const int npix = 12 * c->p.nside * c->p.nside;
    const int nrm = c->nr_max;
    int waves = waves_req;
    if (waves <= 0) {
        waves = c->tuned_waves[f32 ? 1 : 0];
        if (waves <= 0) waves = npix >= 192 ? 16 : 8;   // the tuned picks at N_side 4 and 2
    }
    // the radial-kernel variants are built for 4 and 8 waves per target only
    const bool kv = !((c->p.eps_kernel == 0 || c->p.eps_kernel == 3) && (c->p.mass_kernel == 0 || c->p.mass_kernel == 5));
    if (kv) waves = waves <= 4 ? 4 : 8;
    L.waves = waves;
    // per-level frontier and per-target accepted-node capacities (overflow is reported)
    L.fmax = 512;
    L.amax = 2048;
    int bm = buf_req > 0 ? buf_req : c->tuned_buf[f32 ? 1 : 0];
    // four rows per ray in LDS (odd stride: ray k of lane k hits distinct banks); else, in
    // FP32, the A, E, V rows in LDS and the emission rows in device memory; else all in
    // device memory
    const int stride4 = 4 * nrm + 1, stride3 = 3 * nrm + 1;
    const bool fits4 = sweep_lds_bytes(real, npix, stride4, nrm, L.fmax, L.amax, waves, true) <= kLdsMax;
    const bool fits3 = f32 && !kv && sweep_lds_bytes(real, npix, stride3, nrm, L.fmax, L.amax, waves, true) <= kLdsMax;
    // else (FP64, or radial-kernel variants) the rays in LDS for as many as fit, with four rows
    // per ray or (fewer passes) the split rows, a target's rays mapped and integrated in
    // passes over equal pixel ranges
    int pass_rays = 0;
    bool pass_split = false;
    if (!fits4 && !fits3 && bm != 2 && !kv && (waves == 4 || waves == 8 || waves == 16)) {
        auto passes = [&](int stride) {   // passes of the largest ray count that fits (0: none)
            for (int r = npix - 1; r >= 16; --r)
                if (sweep_lds_bytes(real, r, stride, nrm, L.fmax, L.amax, waves, true) <= kLdsMax) return (npix + r - 1) / r;
            return 0;
        };
        const int n4 = passes(stride4), n3 = kv ? 0 : passes(stride3);
        const int n = n3 > 0 && (n4 == 0 || n3 < n4) ? n3 : n4;
        if (n > 0) {
            pass_rays = (npix + n - 1) / n;
            pass_split = n == n3 && n3 != n4;
        }
    }
    if (bm == 1 && !fits4 && !fits3 && pass_rays == 0)
        return fail(c, TR_EINVAL, "ray buffers do not fit in LDS for this N_PIX and N_R");
    L.ldsbuf = bm == 2 ? false : (fits4 || fits3 || pass_rays > 0);
    L.pass_rays = L.ldsbuf && !fits4 && !fits3 ? pass_rays : 0;
    L.split = L.ldsbuf && !fits4 && (fits3 || (L.pass_rays > 0 && pass_split));
    L.stride_k = L.split ? stride3 : stride4;
    if (!L.ldsbuf) {
        L.fmax = 1024;
        L.amax = 4096;
    }
    L.lds = sweep_lds_bytes(real, L.pass_rays > 0 ? L.pass_rays : npix, L.stride_k, nrm, L.fmax, L.amax, waves, L.ldsbuf);
    if (kv) {
        L.fn = f32 ? pick_kernel_kv<float>(waves, L.ldsbuf, false) : pick_kernel_kv<double>(waves, L.ldsbuf, false);
        L.fn_fb = f32 ? pick_kernel_kv<float>(waves, L.ldsbuf, true) : pick_kernel_kv<double>(waves, L.ldsbuf, true);
    } else {
        L.fn = f32 ? pick_kernel<float>(waves, L.ldsbuf, false) : pick_kernel<double>(waves, L.ldsbuf, false);
        L.fn_fb = f32 ? pick_kernel<float>(waves, L.ldsbuf, true) : pick_kernel<double>(waves, L.ldsbuf, true);
    }
    if (!L.fn || !L.fn_fb) return fail(c, TR_EINVAL, "waves per target must be 1, 2, 4, 8 or 16");
    // accumulation: compare-and-swap by default (FP32, LDS, 8 or 16 waves)
    {
        const int am = atom_req > 0 ? atom_req : (c->atommode > 0 ? c->atommode : c->tuned_atom[f32 ? 1 : 0]);
        L.cas = f32 && L.ldsbuf && !kv && L.pass_rays == 0 && (waves == 8 || waves == 16) && (am > 0 ? am == 2 : true);
        if (L.cas) {
            L.fn = pick_kernel_cas(waves, false);
            L.fn_fb = pick_kernel_cas(waves, true);
        }
    }
    if (L.pass_rays > 0) {   // (hardware atomics)
        L.fn = f32 ? pick_kernel_pass<float>(waves, false) : pick_kernel_pass<double>(waves, false);
        L.fn_fb = f32 ? pick_kernel_pass<float>(waves, true) : pick_kernel_pass<double>(waves, true);
    }
    HIPCHK(hipFuncSetAttribute((const void *)L.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds));
    HIPCHK(hipFuncSetAttribute((const void *)L.fn_fb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds));
    int occ = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)L.fn, waves * 64, L.lds));
    if (occ <= 0) return fail(c, TR_EINVAL, "sweep kernel does not fit on a compute unit (LDS " + std::to_string(L.lds) + " B)");
    L.per_cu = tpc_req > 0 ? std::min(tpc_req, occ) : occ;
    // integration: by default a group of lanes per ray, so that a target's few
    // emitting rays share a wave (rays with more emitting points than the group
    // has lanes take a wave): 16 lanes from N_side 4 on, where a ray crosses
    // more nodes, else 8
    const int im = int_req > 0 ? int_req : c->tuned_int[f32 ? 1 : 0];
    // (FP32 buffers march in FP32 by default, the FP64 form in FP64)
    L.intm = im > 0 ? im : (npix >= 192 ? 5 : 4) + (f32 ? 3 : 0);
    if (L.intm >= 6 && !f32) L.intm -= 3;
    int64_t blocks = (int64_t)c->n_cu * L.per_cu;
    if (blocks > n_items) blocks = std::max<int64_t>(1, n_items);
    L.blocks = (int)blocks;
    if (!c->glist &&
        dalloc(c, (void **)&c->glist, sizeof(int32_t) * (size_t)c->n_cu * kFallbackPerCu * 3 * kGlobalList))
        return TR_ENOMEM;
    // a captured step graph holds the scratch pointers as kernel arguments:
    // it is dropped whenever one of them is reallocated below
    if (c->ovf_cap < n_items) {   // every item may need the second pass
        drop_graph(c);
        dfree(c->ovf);
        c->ovf_cap = 0;
        if (dalloc(c, (void **)&c->ovf, sizeof(int32_t) * (size_t)n_items)) return TR_ENOMEM;
        c->ovf_cap = n_items;
    }
    // per-workgroup slabs for the larger of the two grids (the second pass has
    // n_cu x min(per_cu, kFallbackPerCu) workgroups)
    const size_t nblk = (size_t)std::max<int64_t>(L.blocks, (int64_t)c->n_cu * std::min(L.per_cu, kFallbackPerCu));
    if (!L.ldsbuf) {
        const size_t need = nblk * npix * L.stride_k * real;
        if (need > c->gbuf_bytes) {
            drop_graph(c);
            dfree(c->gbuf);
            c->gbuf_bytes = 0;
            if (dalloc(c, &c->gbuf, need)) return TR_ENOMEM;
            c->gbuf_bytes = need;
        }
    }
    if (L.split) {
        const size_t need = nblk * npix * nrm * real;
        if (need > c->ebuf_bytes) {
            drop_graph(c);
            dfree(c->ebuf);
            c->ebuf_bytes = 0;
            if (dalloc(c, &c->ebuf, need)) return TR_ENOMEM;
            c->ebuf_bytes = need;
            // the sweeps keep the plane zero between targets
            hipLaunchKernelGGL(k_fill_i32, dim3(grid1((int64_t)(need / 4))), dim3(256), 0, c->stream, (int32_t *)c->ebuf,
                               (int64_t)(need / 4), 0);
        }
    }
    return TR_OK;
}

tr_status launch_sweep(tr_ctx *c, const int64_t *targets, int64_t n, double *f_out, uint8_t *ion, bool timed,
                       int waves_req, int tpc_req, int buf_req, int int_req, int atom_req = 0)
{
    if (!c->built) return fail(c, TR_ESTATE, "tr_sweep needs tr_build first");
    if (c->built_prec != c->p.precision) return fail(c, TR_ESTATE, "precision changed since tr_build; build again");
    if (n == 0) return TR_OK;
    LaunchPlan L;
    tr_status s = plan_sweep(c, n, waves_req > 0 ? waves_req : c->waves, tpc_req > 0 ? tpc_req : c->tpc,
                             buf_req > 0 ? buf_req : c->bufmode, int_req > 0 ? int_req : c->intmode, L, atom_req);
    if (s) return s;
    SweepArgs a{};
    a.geo = c->geo;
    a.olo = c->olo;
    a.oext = c->oext;
    a.topo = c->topo_d;
    a.pA = c->packA;
    a.pB = c->packB;
    a.cell_node = c->cell_node;
    a.cell_dom = c->cell_dom;
    a.doms = c->doms;
    a.r64 = c->r64;
    a.r32 = c->r32;
    a.targets = targets;
    a.order = c->order;
    a.n_items = n;
    a.n_cells = c->n_cells;
    a.f_out = f_out;
    a.ion_out = ion;
    a.queue = c->queue;
    a.stats = c->stats;
    a.gbuf = c->gbuf;
    a.ebuf = c->ebuf;
    a.split = L.split ? 1 : 0;
    a.pass_rays = L.pass_rays;
    a.theta2 = c->p.theta * c->p.theta;
    a.theta_if2 = c->p.theta_if > 0.0 ? c->p.theta_if * c->p.theta_if : 0.0;
    a.theta_src2 = c->p.theta_src > 0.0 ? c->p.theta_src * c->p.theta_src : 0.0;
    // guard band: 1e-5 N_side (at least 2e-5), several times the worst-case
    // FP32 error of the pixel-edge quantities (a few 1e-7 N_side)
    a.guard_tol = 1e-5f * std::max(2.0f, (float)c->p.nside);
    a.nside = c->p.nside;
    a.npix = 12 * c->p.nside * c->p.nside;
    a.subsample = c->p.subsample;
    a.fmax = L.fmax;
    a.amax = L.amax;
    a.nr_max = c->nr_max;
    a.stride_k = L.stride_k;
    a.zeta_g = c->p.zeta_g;
    a.int_wave = L.intm == 2 ? 1 : 0;
    a.int_group = L.intm >= 3 ? lanes_per_ray(L.intm) : 0;
    a.int_fp32 = L.intm >= 6 ? 1 : 0;
    a.front_ratio = 1e-2f;
    a.eps_kernel = c->p.eps_kernel;
    a.periodic = c->p.periodic ? 1 : 0;
    a.mass_gauss = c->p.mass_kernel == 6 ? 1 : 0;
    a.ovf = c->ovf;
    a.ovf_cap = c->ovf_cap;
    a.glist = c->glist;
    a.gfmax = kGlobalList;
    a.gamax = kGlobalList;
    a.atab_idx = c->atab_idx;
    a.atab_pool = c->atab_pool;
    for (int q = 0; q < kAtabRatios; ++q) {
        a.atab_w[q] = c->atab.w[q];
        a.atab_base[q] = c->atab.base[q];
    }
    (void)hipGetLastError();   // a stale error of an earlier, unrelated call is not ours
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, c->queue, (int64_t)4, 0);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, c->stream, c->stats, (int64_t)8);
    if (timed) HIPCHK(hipEventRecord(c->ev0, c->stream));
    hipLaunchKernelGGL(L.fn, dim3(L.blocks), dim3(L.waves * 64), L.lds, c->stream, a);
    // the targets whose walk lists did not fit in LDS, again with lists in device memory
    // (one workgroup per compute unit; it ends at once when none was queued)
    {
        const size_t lds = sweep_lds_bytes(c->p.precision == TR_FP32C ? 4 : 8, L.pass_rays > 0 ? L.pass_rays : a.npix,
                                           L.stride_k, c->nr_max, 0, 0, L.waves, L.ldsbuf);
        hipLaunchKernelGGL(L.fn_fb, dim3(c->n_cu * std::min(L.per_cu, kFallbackPerCu)), dim3(L.waves * 64), lds,
                           c->stream, a);
    }
    HIPCHK(hipGetLastError());
    if (timed) {
        HIPCHK(hipEventRecord(c->ev1, c->stream));
        c->timed_valid = true;
    }
    c->last_waves = L.waves;
    c->last_tpc = L.per_cu;
    c->last_lds = L.ldsbuf ? (L.pass_rays > 0 ? 3 : (L.split ? 2 : 1)) : 0;
    c->last_intw = lanes_per_ray(L.intm);
    c->last_int32 = L.intm >= 6 ? 1 : 0;
    c->last_cas = L.cas ? 1 : 0;
    return TR_OK;
}

tr_status upload_sources(tr_ctx *c)
{
    std::vector<double> xyz, q;
    std::vector<int32_t> dom;
    double qmax = 0;
    for (int d = 0; d < c->n_dom; ++d) {
        for (size_t s = 0; s < c->sq[d].size(); ++s) {
            for (int a = 0; a < 3; ++a) xyz.push_back(c->sxyz[d][3 * s + a]);
            q.push_back(c->sq[d][s]);
            dom.push_back(d);
            qmax = std::max(qmax, c->sq[d][s]);
        }
    }
    tr_status s;
    if ((s = upload(c, c->d_sxyz, xyz))) return s;
    if ((s = upload(c, c->d_sq, q))) return s;
    if ((s = upload(c, c->d_sdom, dom))) return s;
    c->n_src_dev = (int32_t)q.size();
    // internal rate unit: the power of two nearest the largest source rate
    c->rate_unit = std::ldexp(1.0, (int)std::lround(std::log2(std::max(qmax, 1.0))));
    for (int d = 0; d < c->n_dom; ++d) {
        DomDev &D = c->domh[d];
        D.rate_unit = c->rate_unit;
        D.flux_unit = c->rate_unit / (D.dx_cm * D.dx_cm);
        D.alpha_int = c->p.alpha_b * D.dx_cm * D.dx_cm * D.dx_cm / c->rate_unit;
    }
    HIPCHK(hipMemcpyAsync(c->doms, c->domh.data(), sizeof(DomDev) * c->n_dom, hipMemcpyHostToDevice, c->stream));
    c->src_dirty = false;
    return TR_OK;
}

// Gauss-Legendre nodes and weights on [0, 1] for the sphere deposit: the
// roots of P_n by Newton's method from Tricomi's initial estimates.
tr_status upload_gauss_legendre(tr_ctx *c)
{
    double t[kGlNodes], w[kGlNodes];
    const int n = kGlNodes;
    for (int i = 1; i <= n; ++i) {
        double x = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) * std::cos(kPi * (4 * i - 1) / (4.0 * n + 2.0));
        double d = 0.0;
        for (int it = 0; it < 50; ++it) {
            double pm = 1.0, p = x;   // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double pn = ((2 * k - 1) * x * p - (k - 1) * pm) / k;
                pm = p;
                p = pn;
            }
            d = n * (pm - x * p) / (1.0 - x * x);   // P_n'
            const double step = p / d;
            x -= step;
            if (std::fabs(step) < 1e-17) break;
        }
        t[i - 1] = 0.5 * (1.0 + x);
        w[i - 1] = 1.0 / ((1.0 - x * x) * d * d);
    }
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_t), t, sizeof(t)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), w, sizeof(w)));
    return TR_OK;
}

// The angular-weight table of the context's N_side and s: offsets up to
// (2/theta + 1) r target sizes per axis for nodes of r = 1, 2, 4 target sizes
// (every node the Barnes-Hut walk accepts at theta_lim lies inside), capped so
// that the table stays small; nodes outside classify their sub-points.
tr_status build_angular_table(tr_ctx *c)
{
    const int s = c->p.subsample, ns = c->p.nside;
    const double th = c->p.theta > 0.05 ? c->p.theta : 0.05;
    const int cap[kAtabRatios] = {12, 20, 24, 40};
    AtabGeom G{};
    int64_t nk = 0;
    for (int q = 0; q < kAtabRatios; ++q) {
        const int w = std::min(cap[q], (int)std::ceil((2.0 / th + 1.0) * (double)(1 << q)));
        G.w[q] = w;
        G.base[q] = (int32_t)nk;
        nk += (int64_t)(2 * w + 1) * (2 * w + 1) * (2 * w + 1);
    }
    G.nkeys = (int32_t)nk;
    int32_t *cnt = nullptr;
    tr_status st;
    if ((st = dalloc(c, (void **)&cnt, sizeof(int32_t) * (size_t)nk))) return st;
    hipLaunchKernelGGL(k_atab_count, dim3(grid1(nk, 64)), dim3(64), 0, c->stream, G, ns, s, cnt);
    std::vector<int32_t> h((size_t)nk);
    if (hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * (size_t)nk, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        dfree(cnt);
        return fail(c, TR_EHIP, "angular table: counting failed");
    }
    int64_t tot = 0;
    for (auto &v : h) {
        const int32_t n = v;
        v = (int32_t)tot;   // first pair of each entry
        tot += n;
    }
    if (tot >= (1ll << 24)) {   // (first << 7) | pairs must fit an int: keep classifying instead
        dfree(cnt);
        return TR_OK;
    }
    if ((st = dalloc(c, (void **)&c->atab_pool, sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1))) ||
        (st = dalloc(c, (void **)&c->atab_idx, sizeof(int32_t) * (size_t)nk))) {
        dfree(cnt);
        return st;
    }
    if (hipMemcpyAsync(cnt, h.data(), sizeof(int32_t) * (size_t)nk, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        dfree(cnt);
        return fail(c, TR_EHIP, "angular table: upload failed");
    }
    hipLaunchKernelGGL(k_atab_fill, dim3(grid1(nk, 64)), dim3(64), 0, c->stream, G, ns, s, cnt, c->atab_idx,
                       c->atab_pool);
    const hipError_t e = hipStreamSynchronize(c->stream);
    dfree(cnt);
    if (e != hipSuccess) return fail(c, TR_EHIP, std::string("angular table: ") + hipGetErrorString(e));
    c->atab = G;
    return TR_OK;
}

tr_status read_flags(tr_ctx *c)
{
    int32_t f[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(f, c->err_flags, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (f[0] & 1) return fail(c, TR_EINVAL, "a source lies outside its domain or has a bad rate");
    if (f[0] & 2) return fail(c, TR_EINVAL, "n_h or f_prev holds a negative or non-finite value");
    if (f[0] & 4) return fail(c, TR_EINVAL, "source deposit stack overflow");
    return TR_OK;
}

// Device address of the static scratch, resolved once per device with that
// device current (the array's host-side name is only a stand-in for it).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// message of the last call made without a context, per thread
thread_local std::string g_free_err;

tr_status fail_free(tr_status s, const std::string &m)
{
    g_free_err = m;
    return s;
}

}  // namespace

extern "C" {

tr_status tr_create(tr_ctx **out, const tr_params *p, void *stream)
{
    if (!out || !p) return TR_EINVAL;
    *out = nullptr;
    tr_ctx *c = new (std::nothrow) tr_ctx();
    if (!c) return TR_ENOMEM;
    tr_status s = check_params(c, *p);
    if (s) {
        delete c;
        return s;
    }
    c->p = *p;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return TR_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
        delete c;
        return TR_EHIP;
    }
    c->n_cu = prop.multiProcessorCount;
    void *sp = nullptr;
    if (static_scratch(c->device, &sp) != hipSuccess) {   // resolved here, outside any capture
        delete c;
        return TR_EHIP;
    }
    if (hipMalloc((void **)&c->queue, 64) != hipSuccess || hipMalloc((void **)&c->stats, 64) != hipSuccess ||
        hipMalloc((void **)&c->err_flags, 64) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess) {
        tr_destroy(c);
        return TR_ENOMEM;
    }
    // flags and counters start at zero (a sync before any launch reads them)
    if (hipMemset(c->queue, 0, 64) != hipSuccess || hipMemset(c->stats, 0, 64) != hipSuccess ||
        hipMemset(c->err_flags, 0, 64) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        tr_destroy(c);
        return TR_EHIP;
    }
    if (upload_gauss_legendre(c) != TR_OK) {
        tr_destroy(c);
        return TR_EHIP;
    }
    *out = c;
    return TR_OK;
}

void tr_destroy(tr_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_domains(c);
    dfree(c->queue);
    dfree(c->stats);
    dfree(c->err_flags);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

const char *tr_last_error(const tr_ctx *c) { return c ? c->err.c_str() : g_free_err.c_str(); }

tr_status tr_set_domains(tr_ctx *c, int32_t n_domains, const tr_domain *doms)
{
    if (!c) return TR_EINVAL;
    if (n_domains <= 0 || !doms) return fail(c, TR_EINVAL, "need at least one domain");
    HIPCHK(hipStreamSynchronize(c->stream));
    free_domains(c);
    c->topo.assign(n_domains, DomTopo());
    for (int d = 0; d < n_domains; ++d) {
        const std::string m = build_topology(doms[d], c->p, c->topo[d]);
        if (!m.empty()) return fail(c, TR_EINVAL, "domain " + std::to_string(d) + ": " + m);
    }
    c->n_dom = n_domains;
    c->depth_max = 0;
    c->nr_max = 0;
    for (auto &t : c->topo) {
        c->depth_max = std::max(c->depth_max, t.depth);
        c->nr_max = std::max(c->nr_max, t.n_radial);
    }
    // global node numbering: level-major, domains in order inside a level
    const int L = c->depth_max;
    std::vector<std::vector<int64_t>> off(L, std::vector<int64_t>(n_domains, 0));
    std::vector<std::vector<int64_t>> lbase(n_domains);   // local first index of each level
    c->level_begin.assign(L + 1, 0);
    int64_t g = 0;
    for (int l = 0; l < L; ++l) {
        c->level_begin[l] = g;
        for (int d = 0; d < n_domains; ++d) {
            off[l][d] = g;
            const auto &t = c->topo[d];
            if (l < t.depth) g += t.level_count[l];
        }
    }
    c->level_begin[L] = g;
    c->n_nodes = g;
    for (int d = 0; d < n_domains; ++d) {
        const auto &t = c->topo[d];
        int64_t b = 0;
        for (int l = 0; l < t.depth; ++l) {
            lbase[d].push_back(b);
            b += t.level_count[l];
        }
    }
    auto gidx = [&](int d, int64_t local) -> int64_t {
        const auto &lb = lbase[d];
        int l = (int)(std::upper_bound(lb.begin(), lb.end(), local) - lb.begin()) - 1;
        return off[l][d] + (local - lb[l]);
    };
    std::vector<int4> geo(g), olo(g), oext(g);
    std::vector<int2> topo(g);
    int64_t ncell = 0;
    for (auto &t : c->topo) ncell += t.n_cells;
    if (ncell > INT32_MAX) return fail(c, TR_EINVAL, "too many cells");
    c->n_cells = ncell;
    std::vector<int32_t> cnode(ncell), cdom(ncell), order(ncell);
    std::vector<double> r64;
    std::vector<float> r32;
    c->domh.assign(n_domains, DomDev());
    int64_t cbase = 0;
    for (int d = 0; d < n_domains; ++d) {
        const auto &t = c->topo[d];
        const int64_t nn = (int64_t)t.size.size();
        int64_t first_level_end = t.level_count.empty() ? 0 : 0;
        (void)first_level_end;
        for (int64_t i = 0; i < nn; ++i) {
            const int64_t gi = gidx(d, i);
            const int32_t sz = t.size[i];
            bool partial = false;
            for (int a = 0; a < 3; ++a)
                if (t.olo[3 * i + a] != t.lo[3 * i + a] || t.oext[3 * i + a] != sz) partial = true;
            geo[gi] = int4{t.lo[3 * i], t.lo[3 * i + 1], t.lo[3 * i + 2], sz | (partial ? kPartialBit : 0)};
            olo[gi] = int4{t.olo[3 * i], t.olo[3 * i + 1], t.olo[3 * i + 2], 0};
            oext[gi] = int4{t.oext[3 * i], t.oext[3 * i + 1], t.oext[3 * i + 2], 0};
            if (t.nchild[i] == 0) topo[gi] = int2{(int)(cbase + t.first[i]), 0};
            else topo[gi] = int2{(int)gidx(d, t.first[i]), t.nchild[i]};
        }
        for (int64_t q = 0; q < t.n_cells; ++q) {
            cnode[cbase + q] = (int32_t)gidx(d, t.cell_node[q]);
            cdom[cbase + q] = d;
            order[cbase + q] = (int32_t)(cbase + t.morton[q]);
        }
        DomDev &D = c->domh[d];
        D.root = (int32_t)gidx(d, 0);
        D.nr = t.n_radial;
        D.r_off = (int32_t)r64.size();
        D.cell_off = (int32_t)cbase;
        D.n_cells = (int32_t)t.n_cells;
        D.dx_cm = t.dx_cm;
        for (int q = 0; q < 3; ++q) D.ext[q] = t.ext[q];
        D.rate_unit = 1.0;
        D.flux_unit = 1.0 / (t.dx_cm * t.dx_cm);
        D.alpha_int = c->p.alpha_b * t.dx_cm * t.dx_cm * t.dx_cm;
        D.rc_inv = 1.0 / t.r_coef;
        for (double r : t.r_cells) {
            r64.push_back(r);
            r32.push_back((float)r);
        }
        cbase += t.n_cells;
    }
    tr_status s;
    if ((s = upload(c, c->geo, geo)) || (s = upload(c, c->olo, olo)) || (s = upload(c, c->oext, oext)) ||
        (s = upload(c, c->topo_d, topo)) || (s = upload(c, c->cell_node, cnode)) ||
        (s = upload(c, c->cell_dom, cdom)) || (s = upload(c, c->order, order)) || (s = upload(c, c->r64, r64)) ||
        (s = upload(c, c->r32, r32)) || (s = upload(c, c->doms, c->domh)))
        return s;
    if ((s = dalloc(c, (void **)&c->mom, sizeof(double) * MO_COUNT * (size_t)g))) return s;
    if ((s = dalloc(c, &c->packA, 32 * (size_t)g))) return s;
    if ((s = dalloc(c, &c->packB, 32 * (size_t)g))) return s;
    if ((s = dalloc(c, (void **)&c->ndot, sizeof(double) * (size_t)ncell))) return s;
    if ((s = dalloc(c, (void **)&c->hist, sizeof(unsigned int) * 256 * (size_t)n_domains))) return s;
    if ((s = dalloc(c, (void **)&c->dprefix, sizeof(unsigned long long) * n_domains))) return s;
    if ((s = dalloc(c, (void **)&c->drank, sizeof(unsigned long long) * n_domains))) return s;
    if ((s = dalloc(c, (void **)&c->dmax, sizeof(unsigned long long) * n_domains))) return s;
    c->sxyz.assign(n_domains, {});
    c->sq.assign(n_domains, {});
    c->src_dirty = true;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->p.subsample * c->p.subsample * c->p.subsample <= 64 && (s = build_angular_table(c))) return s;
    return TR_OK;
}

tr_status tr_cell_count(const tr_ctx *c, int32_t dom, int64_t *n)
{
    if (!c || !n) return TR_EINVAL;
    if (dom == -1) {
        *n = c->n_cells;
        return TR_OK;
    }
    if (dom < 0 || dom >= c->n_dom) return TR_EINVAL;
    *n = c->topo[dom].n_cells;
    return TR_OK;
}

tr_status tr_set_sources(tr_ctx *c, int32_t dom, int64_t n, const double *xyz, const double *q)
{
    if (!c) return TR_EINVAL;
    if (dom < 0 || dom >= c->n_dom) return fail(c, TR_EINVAL, "bad domain index");
    if (n < 0 || (n > 0 && (!xyz || !q))) return fail(c, TR_EINVAL, "bad source arrays");
    const auto &t = c->topo[dom];
    for (int64_t s = 0; s < n; ++s) {
        if (!(q[s] >= 0) || !std::isfinite(q[s])) return fail(c, TR_EINVAL, "source rates must be finite and >= 0");
        for (int a = 0; a < 3; ++a) {
            const double u = xyz[3 * s + a] / t.dx_cm;
            if (!std::isfinite(u) || u < -1e-9 || u > t.ext[a] + 1e-9)
                return fail(c, TR_EINVAL, "source " + std::to_string(s) + " lies outside domain " + std::to_string(dom));
        }
    }
    c->sxyz[dom].assign(xyz, xyz + 3 * n);
    c->sq[dom].assign(q, q + n);
    c->src_dirty = true;
    c->built = false;
    drop_graph(c);
    return TR_OK;
}

}  // extern "C"

namespace {

// Enqueues the tree build (no host synchronisation; capturable).
tr_status enqueue_build(tr_ctx *c, const double *n_h, const double *f_prev, int32_t thin)
{
    const int64_t nn = c->n_nodes, ncell = c->n_cells;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, c->err_flags, (int64_t)2, 0);
    hipLaunchKernelGGL(k_fill_f64, dim3(grid1(ncell)), dim3(256), 0, c->stream, c->ndot, ncell, 0.0);
    if (c->n_src_dev > 0)
    {
        if (c->p.src_radius_cm > 0.0)
            hipLaunchKernelGGL(k_deposit_spheres, dim3(grid1(c->n_src_dev, 64)), dim3(64), 0, c->stream, c->d_sxyz,
                               c->d_sq, c->d_sdom, c->n_src_dev, c->doms, c->geo, c->topo_d, c->p.src_radius_cm,
                               c->ndot, c->err_flags);
        else
            hipLaunchKernelGGL(k_deposit, dim3(grid1(c->n_src_dev, 64)), dim3(64), 0, c->stream, c->d_sxyz, c->d_sq,
                               c->d_sdom, c->n_src_dev, c->doms, c->geo, c->topo_d, c->ndot, c->err_flags);
    }
    hipLaunchKernelGGL(k_cell_quantities, dim3(grid1(ncell)), dim3(256), 0, c->stream, ncell, n_h, c->ndot, f_prev,
                       c->cell_node, c->cell_dom, c->doms, c->geo, thin, c->mom, nn, c->err_flags);
    for (int l = c->depth_max - 2; l >= 0; --l) {
        const int64_t b = c->level_begin[l], e = c->level_begin[l + 1];
        if (e > b)
            hipLaunchKernelGGL(k_reduce_level, dim3(grid1(e - b)), dim3(256), 0, c->stream, b, e, c->topo_d, c->mom, nn);
    }
    if (c->p.precision == TR_FP32C)
        hipLaunchKernelGGL((k_pack<float, float4>), dim3(grid1(nn)), dim3(256), 0, c->stream, nn, c->mom, (float4 *)c->packA,
                           (float4 *)c->packB, c->geo);
    else
        hipLaunchKernelGGL((k_pack<double, double4>), dim3(grid1(nn)), dim3(256), 0, c->stream, nn, c->mom,
                           (double4 *)c->packA, (double4 *)c->packB, c->geo);
    HIPCHK(hipGetLastError());
    return TR_OK;
}

// Enqueues delta_cell per domain into c->dmax (capturable).
tr_status enqueue_delta(tr_ctx *c, const double *f_new, const double *f_old)
{
    const int nd = c->n_dom;
    const int64_t ncell = c->n_cells;
    hipLaunchKernelGGL(k_rank_init, dim3(grid1(nd, 64)), dim3(64), 0, c->stream, nd, c->doms, c->drank, c->dprefix,
                       c->dmax);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1(256 * nd)), dim3(256), 0, c->stream, (int32_t *)c->hist,
                       (int64_t)256 * nd, 0);
    const DomByArray by{c->cell_dom};
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_hist<DomByArray>, dim3(grid1(ncell)), dim3(256), 0, c->stream, ncell, f_old, by,
                           c->dprefix, shift, c->hist);
        hipLaunchKernelGGL(k_select, dim3(grid1(nd, 64)), dim3(64), 0, c->stream, nd, shift, c->hist, c->dprefix,
                           c->drank);
    }
    hipLaunchKernelGGL(k_delta<DomByArray>, dim3(grid1(ncell)), dim3(256), 0, c->stream, ncell, f_new, f_old, by,
                       c->dprefix, c->dmax);
    HIPCHK(hipGetLastError());
    return TR_OK;
}

tr_status check_build_args(tr_ctx *c, const double *n_h)
{
    if (c->n_dom == 0) return fail(c, TR_ESTATE, "tr_build needs tr_set_domains first");
    if (!n_h) return fail(c, TR_EINVAL, "n_h is NULL");
    tr_status s;
    if (c->src_dirty && (s = upload_sources(c))) return s;
    return TR_OK;
}

}  // namespace

extern "C" {

tr_status tr_build(tr_ctx *c, const double *n_h, const double *f_prev, int32_t thin)
{
    if (!c) return TR_EINVAL;
    tr_status s;
    if ((s = check_build_args(c, n_h))) return s;
    (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
    if ((s = enqueue_build(c, n_h, f_prev, thin))) return s;
    if ((s = read_flags(c))) return s;
    c->built = true;
    c->built_prec = c->p.precision;
    return TR_OK;
}

tr_status tr_sweep(tr_ctx *c, double *f_out, uint8_t *ion)
{
    if (!c) return TR_EINVAL;
    if (!f_out) return fail(c, TR_EINVAL, "f_out is NULL");
    return launch_sweep(c, nullptr, c->n_cells, f_out, ion, true, 0, 0, 0, 0);
}

tr_status tr_sweep_targets(tr_ctx *c, const int64_t *targets, int64_t n, double *f_out, uint8_t *ion)
{
    if (!c) return TR_EINVAL;
    if (n < 0 || (n > 0 && (!targets || !f_out))) return fail(c, TR_EINVAL, "bad target list");
    return launch_sweep(c, targets, n, f_out, ion, true, 0, 0, 0, 0);
}

tr_status tr_delta(tr_ctx *c, const double *f_new, const double *f_old, double *delta_host)
{
    if (!c) return TR_EINVAL;
    if (!f_new || !f_old || !delta_host) return fail(c, TR_EINVAL, "NULL argument");
    if (c->n_dom == 0) return fail(c, TR_ESTATE, "no domains");
    (void)hipGetLastError();
    tr_status s;
    if ((s = enqueue_delta(c, f_new, f_old))) return s;
    const int nd = c->n_dom;
    std::vector<unsigned long long> dm(nd);
    HIPCHK(hipMemcpyAsync(dm.data(), c->dmax, sizeof(unsigned long long) * nd, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int d = 0; d < nd; ++d) std::memcpy(&delta_host[d], &dm[d], 8);
    return TR_OK;
}

tr_status tr_step(tr_ctx *c, const double *n_h, const double *f_prev, double *f_out, uint8_t *ion, double *delta_host)
{
    if (!c) return TR_EINVAL;
    if (!f_prev || !f_out || !delta_host) return fail(c, TR_EINVAL, "NULL argument");
    if (f_prev == f_out) return fail(c, TR_EINVAL, "f_prev and f_out must be different buffers");
    tr_status s;
    if ((s = check_build_args(c, n_h))) return s;
    const int nd = c->n_dom;
    const void *key[4] = {n_h, f_prev, f_out, ion};
    tr_ctx::GraphSlot *slot = nullptr;
    for (auto &g : c->gslot) {
        bool same = g.exec != nullptr;
        for (int q = 0; q < 4 && same; ++q) same = key[q] == g.key[q];
        if (same) slot = &g;
    }
    (void)hipGetLastError();
    if (!slot) {
        slot = c->gslot[0].used <= c->gslot[1].used ? &c->gslot[0] : &c->gslot[1];
        drop_slot(*slot);
        // plan (and allocate) the sweep before capturing it
        LaunchPlan L;
        if ((s = plan_sweep(c, c->n_cells, c->waves, c->tpc, c->bufmode, c->intmode, L))) return s;
        if (!c->cap_stream) HIPCHK(hipStreamCreate(&c->cap_stream));
        if (!c->pinned) HIPCHK(hipHostMalloc(&c->pinned, 64 + sizeof(unsigned long long) * (size_t)nd));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        tr_status cs = enqueue_build(c, n_h, f_prev, 0);
        const bool built = c->built;
        const tr_precision bp = c->built_prec;
        c->built = true;
        c->built_prec = c->p.precision;
        if (!cs) cs = launch_sweep(c, nullptr, c->n_cells, f_out, ion, false, 0, 0, 0, 0);
        c->built = built;
        c->built_prec = bp;
        if (!cs) cs = enqueue_delta(c, f_out, f_prev);
        if (!cs && (hipMemcpyAsync(c->pinned, c->err_flags, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
                    hipMemcpyAsync((char *)c->pinned + 8, c->queue, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess))
            cs = fail(c, TR_EHIP, "capture of the flag copy failed");
        if (!cs && hipMemcpyAsync((char *)c->pinned + 64, c->dmax, sizeof(unsigned long long) * (size_t)nd,
                                  hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            cs = fail(c, TR_EHIP, "capture of the delta copy failed");
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(c->cap_stream, &g);
        c->stream = user;
        if (cs) {
            if (g) (void)hipGraphDestroy(g);
            return cs;
        }
        if (ee != hipSuccess) return fail(c, TR_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
        slot->graph = g;
        HIPCHK(hipGraphInstantiate(&slot->exec, slot->graph, nullptr, nullptr, 0));
        for (int q = 0; q < 4; ++q) slot->key[q] = key[q];
    }
    slot->used = ++c->graph_clock;
    HIPCHK(hipGraphLaunch(slot->exec, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->timed_valid = false;   // no timed sweep in a step
    int32_t flags[4];
    std::memcpy(flags, c->pinned, 16);
    if (flags[3] & 4) return fail(c, TR_EHIP, "internal error: a HEALPix pixel index fell outside [0, N_PIX)");
    if (flags[3]) return fail(c, TR_EOVERFLOW, "a walk list overflowed; affected cells hold NaN");
    if (flags[0] & 1) return fail(c, TR_EINVAL, "a source lies outside its domain or has a bad rate");
    if (flags[0] & 2) return fail(c, TR_EINVAL, "n_h or f_prev holds a negative or non-finite value");
    if (flags[0] & 4) return fail(c, TR_EINVAL, "source deposit stack overflow");
    for (int d = 0; d < nd; ++d) std::memcpy(&delta_host[d], (char *)c->pinned + 64 + 8 * d, 8);
    c->built = true;
    c->built_prec = c->p.precision;
    return TR_OK;
}

tr_status tr_solve(tr_ctx *c, const double *n_h, double *f_out, uint8_t *ion, int32_t *iters_out, double *delta_out)
{
    if (!c) return TR_EINVAL;
    if (!n_h || !f_out) return fail(c, TR_EINVAL, "NULL argument");
    tr_status s;
    const int64_t ncell = c->n_cells;
    if (c->solve_tmp_n < ncell) {
        drop_graph(c);
        dfree(c->solve_tmp);
        if ((s = dalloc(c, (void **)&c->solve_tmp, sizeof(double) * (size_t)ncell))) return s;
        c->solve_tmp_n = ncell;
    }
    // F^0: the optically thin sweep
    if ((s = tr_build(c, n_h, nullptr, 1))) return s;
    if ((s = tr_sweep(c, f_out, ion))) return s;
    std::vector<double> dl(c->n_dom, 0.0);
    int32_t it = 0;
    double dmax = INFINITY;
    bool conv = false;
    // iterations alternate between f_out and the scratch field; each is one graph launch
    double *cur = f_out, *nxt = c->solve_tmp;
    while (it < c->p.max_iter) {
        if ((s = tr_step(c, n_h, cur, nxt, ion, dl.data()))) return s;
        std::swap(cur, nxt);
        ++it;
        dmax = 0;
        for (double v : dl) dmax = std::max(dmax, v);
        if (dmax < c->p.eps_lim) {
            conv = true;
            break;
        }
    }
    if (cur != f_out)
        HIPCHK(hipMemcpyAsync(f_out, cur, sizeof(double) * (size_t)ncell, hipMemcpyDeviceToDevice, c->stream));
    if (iters_out) *iters_out = it;
    if (delta_out) *delta_out = dmax;
    if ((s = tr_sync(c))) return s;
    if (!conv && c->p.max_iter > 0) return fail(c, TR_ENOCONV, "delta_cell did not fall below eps_lim");
    return TR_OK;
}

tr_status tr_set_precision(tr_ctx *c, tr_precision prec)
{
    if (!c) return TR_EINVAL;
    if (prec != TR_FP64 && prec != TR_FP32C) return fail(c, TR_EINVAL, "unknown precision");
    if (c->p.precision != prec) drop_graph(c);
    c->p.precision = prec;
    return TR_OK;
}

tr_status tr_set_launch(tr_ctx *c, int32_t waves, int32_t tpc, int32_t buffer, int32_t integration, int32_t atomics)
{
    if (!c) return TR_EINVAL;
    if (atomics < 0 || atomics > 2)
        return fail(c, TR_EINVAL, "atomics must be 0 (auto), 1 (hardware atomic adds) or 2 (compare-and-swap)");
    if (buffer < 0 || buffer > 2) return fail(c, TR_EINVAL, "buffer must be 0 (auto), 1 (LDS) or 2 (device memory)");
    if (integration < 0 || integration > 8)
        return fail(c, TR_EINVAL,
                    "integration must be 0 (auto), 1 (a lane per ray), 2 (a wave per ray), 3, 4, 5 (a group of 4, 8, "
                    "16 lanes per ray) or 6, 7, 8 (the same groups with the FP32 march)");
    if (!(waves == 0 || waves == 1 || waves == 2 || waves == 4 || waves == 8 || waves == 16))
        return fail(c, TR_EINVAL, "waves per target must be 0, 1, 2, 4, 8 or 16");
    if (tpc < 0) return fail(c, TR_EINVAL, "targets per CU must be >= 0");
    c->waves = waves;
    c->tpc = tpc;
    c->bufmode = buffer;
    c->intmode = integration;
    c->atommode = atomics;
    drop_graph(c);
    return TR_OK;
}

tr_status tr_autotune(tr_ctx *c, double *best_ms)
{
    if (!c) return TR_EINVAL;
    if (!c->built) return fail(c, TR_ESTATE, "tr_autotune needs tr_build first");
    c->tuned_int[c->p.precision == TR_FP32C ? 1 : 0] = 0;   // the first stages time the default forms
    c->tuned_atom[c->p.precision == TR_FP32C ? 1 : 0] = 0;
    // sample: every m-th cell in Morton order, enough to fill the chip a few times
    const int64_t want = std::min<int64_t>(c->n_cells, (int64_t)c->n_cu * 64);
    const int64_t step = std::max<int64_t>(1, c->n_cells / std::max<int64_t>(1, want));
    std::vector<int64_t> tg;
    std::vector<int32_t> ord(c->n_cells);
    HIPCHK(hipMemcpyAsync(ord.data(), c->order, sizeof(int32_t) * c->n_cells, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < c->n_cells && (int64_t)tg.size() < want; i += step) tg.push_back(ord[i]);
    int64_t *dt = nullptr;
    double *fo = nullptr;
    tr_status s;
    if ((s = dalloc(c, (void **)&dt, sizeof(int64_t) * tg.size()))) return s;
    if ((s = dalloc(c, (void **)&fo, sizeof(double) * tg.size()))) { dfree(dt); return s; }
    HIPCHK(hipMemcpyAsync(dt, tg.data(), sizeof(int64_t) * tg.size(), hipMemcpyHostToDevice, c->stream));
    const int cand[5] = {1, 2, 4, 8, 16};
    double best = INFINITY;
    int bw = 0, bb = 0, bi = 0;
    // mean of two timed sweeps after one untimed; false if the shape does not run
    auto timed = [&](int w, int bm, int im, double &ms_out, int am = 0) {
        LaunchPlan L;
        if (plan_sweep(c, (int64_t)tg.size(), w, 0, bm, im, L, am) != TR_OK) return false;
        float ms = 0, tot = 0;
        for (int rep = 0; rep < 3; ++rep) {
            if (launch_sweep(c, dt, (int64_t)tg.size(), fo, nullptr, true, w, 0, bm, im, am) != TR_OK) return false;
            if (hipEventSynchronize(c->ev1) != hipSuccess) return false;
            (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
            if (rep > 0) tot += ms;
        }
        ms_out = tot / 2;
        return true;
    };
    // waves and buffer place with the default integration, then the integration form
    for (int bm = 1; bm <= 2; ++bm)
        for (int w : cand) {
            double ms;
            if (timed(w, bm, 0, ms) && ms < best) {
                best = ms;
                bw = w;
                bb = bm;
                bi = 0;
            }
        }
    if (bw > 0)
        for (int im : {1, 2, 3, 4, 5, 6, 7, 8}) {
            if (im >= 6 && c->p.precision != TR_FP32C) break;
            double ms;
            if (timed(bw, bb, im, ms) && ms < best) {
                best = ms;
                bi = im;
            }
        }
    // and the accumulation form where there is a choice (FP32 buffers in LDS, 8 or 16 waves)
    int ba = 0;
    if (bw >= 8 && bb == 1 && c->p.precision == TR_FP32C)
        for (int am : {1, 2}) {
            double ms;
            if (timed(bw, bb, bi, ms, am) && ms < best) {
                best = ms;
                ba = am;
            }
        }
    dfree(dt);
    dfree(fo);
    c->err.clear();
    (void)hipGetLastError();
    drop_graph(c);   // trial plans may have reallocated the scratch a graph refers to
    if (bw == 0) return fail(c, TR_EHIP, "no launch shape ran");
    c->tuned_waves[c->p.precision == TR_FP32C ? 1 : 0] = bw;
    c->tuned_buf[c->p.precision == TR_FP32C ? 1 : 0] = bb;
    c->tuned_int[c->p.precision == TR_FP32C ? 1 : 0] = bi;
    c->tuned_atom[c->p.precision == TR_FP32C ? 1 : 0] = ba;
    if (best_ms) *best_ms = best;
    return TR_OK;
}

tr_status tr_get_stats(tr_ctx *c, tr_stats *out)
{
    if (!c || !out) return TR_EINVAL;
    std::memset(out, 0, sizeof(*out));
    unsigned long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int32_t q[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(st, c->stats, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(q, c->queue, sizeof(q), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    out->n_cells = c->n_cells;
    out->n_nodes = c->n_nodes;
    out->nodes_accepted = (int64_t)st[0];
    out->nodes_tested = (int64_t)st[1];
    out->guard_recomputes = (int64_t)st[2];
    out->n_radial_max = c->nr_max;
    out->depth_max = c->depth_max;
    out->waves_per_target = c->last_waves;
    out->targets_per_cu = c->last_tpc;
    out->buffer_in_lds = c->last_lds;
    out->integration_wave = c->last_intw;
    out->lds_cas = c->last_cas;
    out->integration_fp32 = c->last_int32;
    out->rays_fp32 = (int64_t)st[3];
    out->rays_fp64_again = (int64_t)st[4];
    out->nodes_tabulated = (int64_t)st[5];
    out->rays_regrouped = (int64_t)st[6];
    out->overflow = q[1];
    float ms = 0;
    if (c->timed_valid && hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) out->last_sweep_ms = ms;
    (void)hipGetLastError();
    return TR_OK;
}

tr_status tr_delta_noalloc(const double *f_new, const double *f_old, const int64_t *dom_offsets, int32_t n_domains,
                           double *delta_dev, void *stream)
{
    if (!f_new || !f_old || !dom_offsets || !delta_dev) return fail_free(TR_EINVAL, "NULL argument");
    if (n_domains < 1 || n_domains > kStaticDomains)
        return fail_free(TR_EINVAL, "n_domains must be in [1, " + std::to_string(kStaticDomains) +
                                        "]: the static scratch holds " + std::to_string(kStaticDomains) + " domains");
    DomByRanges R{};
    R.n = n_domains;
    if (dom_offsets[0] != 0) return fail_free(TR_EINVAL, "dom_offsets[0] must be 0");
    for (int d = 0; d <= n_domains; ++d) {
        R.off[d] = dom_offsets[d];
        if (d > 0 && dom_offsets[d] <= dom_offsets[d - 1])
            return fail_free(TR_EINVAL, "every domain needs at least one cell (dom_offsets strictly increasing)");
    }
    const int64_t ncell = R.off[n_domains];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail_free(TR_EHIP, "hipGetDevice failed");
    void *sp = nullptr;
    const hipError_t e = static_scratch(dev, &sp);
    if (e != hipSuccess) return fail_free(TR_EHIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    unsigned int *hist = (unsigned int *)sp;
    unsigned long long *prefix = (unsigned long long *)sp + (size_t)kStaticDomains * 128;
    unsigned long long *rank = prefix + kStaticDomains, *dmax = rank + kStaticDomains;
    hipStream_t st = (hipStream_t)stream;
    const int nd = n_domains;
    (void)hipGetLastError();
    // the last call's contents stay in the scratch: everything read is set here first
    hipLaunchKernelGGL(k_rank_init_ranges, dim3(1), dim3(64), 0, st, R, rank, prefix, dmax);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1(256 * nd)), dim3(256), 0, st, (int32_t *)hist, (int64_t)256 * nd, 0);
    for (int shift = 56; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_hist<DomByRanges>, dim3(grid1(ncell)), dim3(256), 0, st, ncell, f_old, R, prefix, shift,
                           hist);
        hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, st, nd, shift, hist, prefix, rank);
    }
    hipLaunchKernelGGL(k_delta<DomByRanges>, dim3(grid1(ncell)), dim3(256), 0, st, ncell, f_new, f_old, R, prefix,
                       dmax);
    hipLaunchKernelGGL(k_store_delta, dim3(1), dim3(64), 0, st, nd, dmax, delta_dev);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) return fail_free(TR_EHIP, std::string("launch failed: ") + hipGetErrorString(le));
    return TR_OK;
}

#ifndef TR_SOURCE_DIGEST
#define TR_SOURCE_DIGEST "unknown"
#endif
const char *tr_source_digest(void) { return TR_SOURCE_DIGEST; }

tr_status tr_sync(tr_ctx *c)
{
    if (!c) return TR_EINVAL;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    int32_t q[2] = {0, 0};
    HIPCHK(hipMemcpy(q, c->queue, sizeof(q), hipMemcpyDeviceToHost));
    if (q[1] & 4) return fail(c, TR_EHIP, "internal error: a HEALPix pixel index fell outside [0, N_PIX)");
    if (q[1] & 2) return fail(c, TR_EINVAL, "a target index lies outside [0, n_cells); those outputs hold NaN");
    if (q[1]) return fail(c, TR_EOVERFLOW, "a walk list overflowed; affected targets hold NaN");
    return TR_OK;
}

}  // extern "C"
