// mmoc_trace.hip -- the RK4 particle-trace kernels for CDNA4 (gfx950).
//
// One lane traces one particle through a whole MMOC advection step
// (Sec. 2.3.1 steps (i)-(iii)): it creates the particle at its P2 DoF, runs
// the S x 4 RK4 stages -- each a macro walk, an O(1) micro location and a P2
// gather of both velocity levels (Sec. 2.3.2) -- accumulates the departure
// point in float64, and evaluates the old scalar there.  Particles are
// independent; lanes only meet in the per-wave ballots that count flagged
// particles into the statistics.
//
// Memory (device resident, see mmoc_internal.h):
//   geo    MacroGeo[n_macros], 256 B each, L2 resident
//   owned  uint64 (macro, I, J, K) per DoF in unique order; lane t traces
//          DoF t, so the 64 lanes of a wave run along a lattice line of one
//          macro and their gathers hit neighbouring slots
//   fields per-component arrays over the block slots (slot = macro * npm +
//          lattice index): small records give few cache lines per wave-level
//          load.  A node costs two 16-byte + two 8-byte loads (float64, two
//          levels) or two 12-byte loads (float32, two levels).
//   The velocity at a particle's own DoF (first stage) is its nodal value.
//
// Precision paths (one kernel each):
//   fp64  every operation in float64;
//   fp32  (mixed) the offset of a stage point from the macro origin is formed
//         in float64, then location, shape functions and sums run in float32
//         on float32 records; a macro decision whose smallest barycentric is
//         within eps32_macro of zero, and a micro decision whose sorted
//         coordinates come within eps32_micro * n of a tie, is re-taken in
//         float64; the departure point is accumulated in float64.
//
// Workgroups are remapped so that each of the 8 XCDs (own L2 each) receives
// one contiguous eighth of the particle range.
#include "mmoc_internal.h"
#include "mmoc_mlp_internal.h"

#include <limits.h>
#include <math.h>

// No implicit contraction of a * b + c into fma in this file: every fused
// multiply-add is written as fma().  The kernel variants (element cache on
// or off, finish pass, tie-band re-locations) then round identically, and a
// result does not depend on how the compiler inlined or scheduled a variant.
#pragma clang fp contract(off)

// 128-thread blocks and runs of 16 blocks per XCD: measured best across the
// three precisions at 2.7e5 and 1.7e7 particles (the plain contiguous eighth
// per XCD starves XCDs of the float32-mixed path's tie-band work)
#ifndef MMOC_TRACE_BLOCK
#define MMOC_TRACE_BLOCK 128
#endif
// occupancy floors: the float64 kernels need at least 3 waves per SIMD
// without spilling (the RK4 kernel fits 4 at 128 VGPRs), the float32-mixed
// kernel 4; the cached float64-arithmetic kernels ask for 4 (their 20 KB of
// LDS per block allow 4; where the LDS allows fewer the compiler keeps more
// registers)
#ifndef MMOC_WPE_FP64
#define MMOC_WPE_FP64 3
#endif
#ifndef MMOC_WPE_FP32
#define MMOC_WPE_FP32 4
#endif
// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// The trace kernels remap them so that each XCD receives runs of 2^k
// consecutive logical blocks (neighbouring particles, hence neighbouring
// field data in that XCD's L2), consecutive runs going to different XCDs;
// k = -1 gives each XCD one contiguous eighth of the range.
//  * float64 kernels, small launches: contiguous eighths.  Every field line
//    is pulled into about one L2 (runs of 16 blocks pulled each line into
//    several: 3.6x the fetch traffic) and the kernel is 7% faster.
//  * float64 kernels, launches of many rounds (>= 16384 blocks): runs of
//    256 blocks.  Work is uneven across a large flow (walks, plumes), and
//    the runs balance it over the XCDs: 7-11% faster than eighths.
//  * float32-mixed: runs of 16 blocks.  Its tie-band re-locations cluster
//    in regions, and short runs spread them over all XCDs.
#ifndef MMOC_XCD_LOG2_FP64_LARGE
#define MMOC_XCD_LOG2_FP64_LARGE 8
#endif
#ifndef MMOC_XCD_LARGE_BLOCKS
#define MMOC_XCD_LARGE_BLOCKS 16384
#endif
#ifndef MMOC_XCD_LOG2_FP32
#define MMOC_XCD_LOG2_FP32 4
#endif

namespace mmoc {
namespace {

constexpr int kTB = MMOC_TRACE_BLOCK;
static_assert(kTB == kSurrogateTile, "the surrogate finish pass takes one fallback tile per block");

__device__ __forceinline__ int64_t logical_block(int lg)
{
    const unsigned b = blockIdx.x, x = b & 7u, j = b >> 3;
    if (lg < 0) return (int64_t)x * (gridDim.x >> 3) + j;
    return ((((int64_t)(j >> lg) << 3) + x) << lg) + (j & ((1u << lg) - 1u));
}

// ------------------------------------------------------------------ geometry

// a.b over the first DIM components
template <int DIM>
__device__ __forceinline__ double dotd(const double* a, const double* b)
{
    if constexpr (DIM == 2) return fma(a[0], b[0], a[1] * b[1]);
    else return fma(a[2], b[2], fma(a[0], b[0], a[1] * b[1]));
}

// 1/a and sqrt(a) for the inverse blending map, from the hardware's
// reciprocal and reciprocal-square-root estimates: two Newton-Raphson steps
// for 1/a, and for sqrt(a) the coupled iteration on s ~ sqrt(a), h ~
// 1/(2 sqrt(a)) (Goldschmidt) with two residual corrections.  Within an
// ulp or two of the correctly rounded results, without their range
// scaling: a is a squared radius or a projection, positive and far from
// the overflow and denormal ranges on a blended shell.
__device__ __forceinline__ double recip64(double a)
{
    double x = __builtin_amdgcn_rcp(a);
    double e = fma(-a, x, 1.0);
    x = fma(x, e, x);
    e = fma(-a, x, 1.0);
    return fma(x, e, x);
}

__device__ __forceinline__ double sqrt64(double a)
{
    const double g = __builtin_amdgcn_rsq(a);
    double s = a * g, h = 0.5 * g;
    const double e = fma(-h, s, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    double d = fma(-s, s, a);
    s = fma(d, h, s);
    d = fma(-s, s, a);
    return fma(d, h, s);
}

template <int DIM, int BLEND>
struct Geo64 {
    double v0[DIM];
    double bi[DIM][DIM];
    double pn[3];
    double pc;

    template <typename P>
    __device__ __forceinline__ void load(P g, int M)
    {
#pragma unroll
        for (int i = 0; i < DIM; ++i) v0[i] = g[M].v0[i];
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) bi[r][c] = g[M].binv[r * 3 + c];
        if constexpr (BLEND) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) pn[i] = g[M].pn[i];
            pc = g[M].pc;
        }
    }

    // physical y -> offset from the macro origin in the computational domain
    __device__ __forceinline__ void offset(const double* y, double* p) const
    {
        if constexpr (BLEND) {
            // Phi^-1(z) = z c |z| / (n.z)
            const double nz = dotd<DIM>(pn, y);
            const double r = sqrt64(dotd<DIM>(y, y));
            const double f = pc * r * recip64(nz);
#pragma unroll
            for (int i = 0; i < DIM; ++i) p[i] = fma(y[i], f, -v0[i]);
        } else {
#pragma unroll
            for (int i = 0; i < DIM; ++i) p[i] = y[i] - v0[i];
        }
    }

    // reference coordinates s of y, returns lambda_0 = 1 - sum s
    __device__ __forceinline__ double ref(const double* y, double* s) const
    {
        double p[DIM];
        offset(y, p);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double acc = bi[a][0] * p[0];
#pragma unroll
            for (int i = 1; i < DIM; ++i) acc = fma(bi[a][i], p[i], acc);
            s[a] = acc;
        }
        double sum = s[0];
#pragma unroll
        for (int a = 1; a < DIM; ++a) sum += s[a];
        return 1.0 - sum;
    }
};

// Reference coordinates of y in macro M, the geometry read afresh for each
// evaluation instead of being kept in registers across the loop.  When every
// active lane of the wave is in the same macro (the common case) the record
// is read through scalar loads into scalar registers; otherwise each lane
// reads its own, from the block's LDS copy when the mesh has few macros
// (sgeo, see stage_geo), else from global memory (an L1/L2 hit: the table
// is small).
typedef __attribute__((address_space(4))) const MacroGeo* ConstGeo;
typedef __attribute__((address_space(3))) const MacroGeo* LdsGeo;

// macros whose geometry the float64 trace kernel copies into LDS (4 KB)
constexpr int kLdsGeo = 16;

// Copies the geometry of a mesh of at most kLdsGeo macros into the block's
// LDS array and returns it (null for larger meshes).  Every thread of the
// block must call it.
__device__ __forceinline__ const MacroGeo* stage_geo(const MacroGeo* __restrict__ geo, int nm, MacroGeo* sgeo)
{
    const bool on = nm <= kLdsGeo;
    if (on) {
        const uint4* src = reinterpret_cast<const uint4*>(geo);
        uint4* dst = reinterpret_cast<uint4*>(sgeo);
        constexpr int kChunks = (int)(sizeof(MacroGeo) / sizeof(uint4));
        for (int i = (int)threadIdx.x; i < nm * kChunks; i += (int)blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    return on ? sgeo : nullptr;
}

template <int DIM, int BLEND>
__device__ __forceinline__ double ref_at(const MacroGeo* __restrict__ geo, int M, const double* y, double* s,
                                         const MacroGeo* sgeo = nullptr)
{
    const int M0 = __builtin_amdgcn_readfirstlane(M);
    Geo64<DIM, BLEND> G;
    if (__ballot(M != M0) == 0) {
        // the table is read-only for the whole launch: a load through the
        // constant address space at a uniform address is a scalar load
        G.load((ConstGeo)geo, M0);
        const double l0 = G.ref(y, s);
        // keeps the two branches apart, so that this one computes with the
        // geometry in scalar registers instead of copying it to vector ones
        __asm__ volatile("");
        return l0;
    }
    if (sgeo) G.load((LdsGeo)sgeo, M);
    else G.load(geo, M);
    return G.ref(y, s);
}

template <int DIM, typename R>
__device__ __forceinline__ R lam_min(R l0, const R* s)
{
    R m = l0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) m = fmin(m, s[a]);
    return m;
}

// Macro walk from M (Sec. 2.3.2: search the neighbourhood of the macro that
// held the previous evaluation).  Accept when min lambda >= -eps; otherwise
// hop across the face with the most negative lambda among faces that have a
// neighbour (ties: lowest face).  No such face: the point is outside the
// domain and stays in M.  After max_hops hops: brute force (argmax over
// macros of min lambda, ties: lowest macro).  Out of line and scalar-only so
// that the hot loop never spills; returns the macro in bits 0-26 and lane
// flags above.
template <int DIM, int BLEND>
__device__ __noinline__ __attribute__((pure)) unsigned walk64(const MacroGeo* __restrict__ geo, int nm, int max_hops, double eps, int M,
                                        double y0, double y1, double y2)
{
    const double y[3] = {y0, y1, y2};
    double s[DIM];
    unsigned flags = 0;
    Geo64<DIM, BLEND> G;
    G.load(geo, M);
    for (int hop = 0;; ++hop) {
        const double l0 = G.ref(y, s);
        if (lam_min<DIM, double>(l0, s) >= -eps) return (unsigned)M | (flags << 27);
        const int32_t* nb = geo[M].nbr;
        int kb = -1, nk = -1;
        double lb = 0.0;
#pragma unroll
        for (int k = 0; k <= DIM; ++k) {
            const double lk = k == 0 ? l0 : s[k - 1];
            if (lk < -eps) {
                const int q = nb[k];
                if (q >= 0 && (kb < 0 || lk < lb)) {
                    kb = k;
                    lb = lk;
                    nk = q;
                }
            }
        }
        if (kb < 0) return (unsigned)M | ((flags | LF_OUTSIDE) << 27);
        if (hop >= max_hops) break;
        if (hop >= 1) flags |= LF_MULTIHOP;
        M = nk;
        G.load(geo, M);
    }
    flags |= LF_BRUTE;
    int best = 0;
    double bestv = -INFINITY;
    for (int q = 0; q < nm; ++q) {
        G.load(geo, q);
        const double ll = G.ref(y, s);
        const double v = lam_min<DIM, double>(ll, s);
        if (v > bestv) {
            bestv = v;
            best = q;
        }
    }
    if (bestv < -eps) flags |= LF_OUTSIDE;
    return (unsigned)best | (flags << 27);
}

// ------------------------------------------------- micro element + P2 / P1

// ORD 2: P2 nodes, the vertices 0..DIM then the edges (a<b); ORD 1: P1, the
// vertices only (Sec. 3.1: P1 and P2 Lagrange elements)
template <int DIM, typename R, int ORD = 2>
struct Stencil {
    static constexpr int NN = ORD == 2 ? (DIM + 1) * (DIM + 2) / 2 : DIM + 1;
    int idx[NN];  // lattice index of the nodes
    R phi[NN];    // shape function values
    int k[3];     // the element: base cell k and the rank of each axis
    int r[3];     //   (filled by micro whether or not idx is)
};

__device__ __forceinline__ int tri_n(int x) { return (x * (x + 1)) >> 1; }
__device__ __forceinline__ int tet_n(int x) { return (x * (x + 1) * (x + 2)) / 6; }

// Lattice indices of an element's nodes from its base cell k and axis
// ranks r: micro vertex a is V_a = k + [r < a] (componentwise); P1 nodes
// are the vertices on the lattice of resolution n, P2 node (a, b) sits at
// V_a + V_b on the lattice of resolution 2n (vertex nodes a = b first,
// then the edges a < b).
//
// P2: along axis x node (a, b), a <= b, has the doubled coordinate
// 2 k_x + [r_x < b] + [r_x < a].  The lattice index is a sum of one term
// per axis, and from 2 k_x that term grows by P_x at the first unit and
// by a further Q_x at the second.  So idx(a, b) = base + Pc(b) + Qc(a),
// with Pc(t) and Qc(t) the sums of P_x and Q_x over the axes of rank below
// t: a few selects by rank per element instead of per node (base is
// carried in Qc below).
template <int DIM, int ORD>
__device__ __forceinline__ void stencil_idx(const int* k, const int* r, int* idx)
{
    if constexpr (ORD == 1) {
        const int I0 = k[0], J0 = k[1], K0 = k[2];
        const int TI0 = DIM == 3 ? tet_n(I0) : tri_n(I0);
        const int TI1 = TI0 + (DIM == 3 ? tri_n(I0 + 1) : I0 + 1);
        const int TJ0 = DIM == 3 ? tri_n(J0) : J0;
        const int TJ1 = TJ0 + (DIM == 3 ? J0 + 1 : 1);
#pragma unroll
        for (int a = 0; a <= DIM; ++a) {
            int id = ((r[0] < a) ? TI1 : TI0) + ((r[1] < a) ? TJ1 : TJ0);
            if constexpr (DIM == 3) id += K0 + (r[2] < a);
            idx[a] = id;
        }
    } else {
        const int I0 = 2 * k[0], J0 = 2 * k[1];
        int base, P[DIM], Q[DIM];
        if constexpr (DIM == 3) {
            base = tet_n(I0) + tri_n(J0) + 2 * k[2];
            P[0] = tri_n(I0 + 1);
            Q[0] = tri_n(I0 + 2);
            P[1] = J0 + 1;
            Q[1] = J0 + 2;
            P[2] = 1;
            Q[2] = 1;
        } else {
            base = tri_n(I0) + J0;
            P[0] = I0 + 1;
            Q[0] = I0 + 2;
            P[1] = 1;
            Q[1] = 1;
        }
        // the value of the axis of rank j
        auto by_rank = [&](const int* v, int j) {
            if constexpr (DIM == 3) return r[0] == j ? v[0] : (r[1] == j ? v[1] : v[2]);
            else return r[0] == j ? v[0] : v[1];
        };
        int Pc[DIM + 1], Qc[DIM + 1];
        Pc[0] = 0;
        Qc[0] = base;
#pragma unroll
        for (int t = 1; t < DIM; ++t) {
            Pc[t] = Pc[t - 1] + by_rank(P, t - 1);
            Qc[t] = Qc[t - 1] + by_rank(Q, t - 1);
        }
        Pc[DIM] = P[0] + P[1];
        Qc[DIM] = base + Q[0] + Q[1];
        if constexpr (DIM == 3) {
            Pc[DIM] += P[2];
            Qc[DIM] += Q[2];
        }
        int c = 0;
#pragma unroll
        for (int a = 0; a <= DIM; ++a) idx[c++] = Qc[a] + Pc[a];
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int b = a + 1; b <= DIM; ++b) idx[c++] = Qc[a] + Pc[b];
    }
}

// O(1) micro location in the Freudenthal lattice of the macro's Kuhn
// coordinates w (w_d = s_d, w_a = s_a + w_{a+1}), then the P2 shape
// functions at the (possibly unclamped) point.  A point outside the macro
// selects its element from the clamped, renormalised barycentrics and is
// evaluated by extrapolating that element.  With GAP, returns the smallest
// distance of the selection coordinates W = n w from a tie (an integer, or
// another coordinate), which the mixed-precision path compares with its
// micro band (1 without GAP).
template <int DIM, typename R, bool GAP = false, int ORD = 2, bool IDX = true>
__device__ __forceinline__ R micro(const R* s, R l0, R lmin, int n, Stencil<DIM, R, ORD>& st)
{
    R ssel[DIM];
    if (lmin >= R(0)) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) ssel[a] = s[a];
    } else {
        R sum = fmax(l0, R(0));
#pragma unroll
        for (int a = 0; a < DIM; ++a) sum += fmax(s[a], R(0));
        const R inv = R(1) / sum;
#pragma unroll
        for (int a = 0; a < DIM; ++a) ssel[a] = fmax(s[a], R(0)) * inv;
    }
    const R dn = (R)n;
    R W[DIM], Wu[DIM];
    W[DIM - 1] = ssel[DIM - 1];
    Wu[DIM - 1] = s[DIM - 1];
#pragma unroll
    for (int a = DIM - 2; a >= 0; --a) {
        W[a] = ssel[a] + W[a + 1];
        Wu[a] = s[a] + Wu[a + 1];
    }
    int k[3] = {0, 0, 0};
    R f[DIM], fu[DIM];
    R gap = R(1);
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        W[i] *= dn;
        const R kc = floor(fmin(fmax(W[i], R(0)), dn - R(1)));
        k[i] = (int)kc;
        f[i] = W[i] - kc;
        fu[i] = fma(Wu[i], dn, -kc);
        if constexpr (GAP) gap = fmin(gap, fmin(fabs(f[i]), fabs(R(1) - f[i])));
    }
    // rank of each axis in the descending order of f (ties: lower axis first)
    int r[3] = {0, 0, 0};
    R g[DIM];
    if constexpr (DIM == 3) {
        r[0] = (f[1] > f[0]) + (f[2] > f[0]);
        r[1] = (f[0] >= f[1]) + (f[2] > f[1]);
        r[2] = (f[0] >= f[2]) + (f[1] >= f[2]);
        g[0] = r[0] == 0 ? fu[0] : (r[1] == 0 ? fu[1] : fu[2]);
        g[1] = r[0] == 1 ? fu[0] : (r[1] == 1 ? fu[1] : fu[2]);
        g[2] = r[0] == 2 ? fu[0] : (r[1] == 2 ? fu[1] : fu[2]);
        if constexpr (GAP) gap = fmin(gap, fmin(fabs(f[0] - f[1]), fmin(fabs(f[0] - f[2]), fabs(f[1] - f[2]))));
    } else {
        r[0] = f[1] > f[0];
        r[1] = f[0] >= f[1];
        g[0] = r[0] == 0 ? fu[0] : fu[1];
        g[1] = r[0] == 1 ? fu[0] : fu[1];
        if constexpr (GAP) gap = fmin(gap, fabs(f[0] - f[1]));
    }
    R mu[DIM + 1];
    mu[0] = R(1) - g[0];
#pragma unroll
    for (int a = 1; a < DIM; ++a) mu[a] = g[a - 1] - g[a];
    mu[DIM] = g[DIM - 1];
    // the element (micro vertex a = k + the first a axes in rank order),
    // its node indices unless the caller takes them later (IDX false), and
    // the shape functions at the point
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        st.k[i] = k[i];
        st.r[i] = r[i];
    }
    if constexpr (IDX) stencil_idx<DIM, ORD>(k, r, st.idx);
    if constexpr (ORD == 1) {
#pragma unroll
        for (int a = 0; a <= DIM; ++a) st.phi[a] = mu[a];
        return gap;
    }
    int c = 0;
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        st.phi[c] = mu[a] * fma(R(2), mu[a], R(-1));
        ++c;
    }
#pragma unroll
    for (int a = 0; a <= DIM; ++a)
#pragma unroll
        for (int b = a + 1; b <= DIM; ++b) {
            st.phi[c] = R(4) * mu[a] * mu[b];
            ++c;
        }
    return gap;
}

// Particle creation (step (i)): physical position of lattice node (I, J, K)
// of macro M, x = Phi(v0 + B s), s = (I - J, J - K, K) / m.
template <int DIM, int BLEND>
__device__ __forceinline__ void dof_position(const MacroGeo* __restrict__ geo, uint64_t e, int lat_m, int& M,
                                             double* x)
{
    M = (int)(e >> 36);
    const int I = (int)((e >> 24) & 0xfffu), J = (int)((e >> 12) & 0xfffu), K = (int)(e & 0xfffu);
    const double invm = 1.0 / (double)lat_m;  // exact: m is a power of two
    double s[3];
    if constexpr (DIM == 2) {
        s[0] = (double)(I - J) * invm;
        s[1] = (double)J * invm;
    } else {
        s[0] = (double)(I - J) * invm;
        s[1] = (double)(J - K) * invm;
        s[2] = (double)K * invm;
    }
    const MacroGeo& G = geo[M];
    double p[3];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        double acc = G.v0[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc = fma(G.B[i * 3 + a], s[a], acc);
        p[i] = acc;
    }
    if constexpr (BLEND) {
        const double nx = dotd<DIM>(G.pn, p);
        const double r = sqrt(dotd<DIM>(p, p));
        const double f = nx / (G.pc * r);
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[i] = p[i] * f;
    } else {
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[i] = p[i];
    }
}

// ------------------------------------------------------------------ gathers

// load of a V from a uniform base plus a 32-bit byte offset (the SGPR-base
// addressing form: no 64-bit address arithmetic per load)
template <typename V, typename T>
__device__ __forceinline__ V ldv(const T* __restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}

struct alignas(4) F3 {
    float x, y, z;
};

// The two velocity levels around a stage time and the weight of the later
// one.  pos counts intervals back from the trace's start, the later end of
// interval iv = min(floor(pos), n_int - 1) is logical level first + n_int -
// iv.  A stationary run has one level.  Uniform across the wave.
template <typename T>
struct Levels {
    const T* ea;  // earlier level: va / vb records
    const T* eb;
    const T* la;  // later level
    const T* lb;
    uint32_t zsh;  // log2 of the bytes per slot in the vb records (a shift: the
                   // slot's byte offset without an integer multiply)
    bool efirst;  // paired u_z records (two-level float64 ring): the earlier level is ring slot 0
};

template <int NLEV, typename T, typename R>
__device__ __forceinline__ Levels<T> levels_at(const TraceArgs<T>& A, double pos, R& theta)
{
    Levels<T> L;
    if constexpr (NLEV == 1) {
        const int p = (A.rot + A.first) % A.lev_cap;
        L.ea = L.la = A.va + (int64_t)p * A.lsa;
        L.eb = L.lb = A.vb + (int64_t)p * A.lsb;
        L.efirst = true;
        theta = R(1);
    } else {
        int iv = (int)pos;
        iv = iv < A.n_int - 1 ? iv : A.n_int - 1;
        theta = (R)(1.0 - (pos - (double)iv));
        const int late = (A.rot + A.first + A.n_int - iv) % A.lev_cap;
        const int early = (late + A.lev_cap - 1) % A.lev_cap;
        L.la = A.va + (int64_t)late * A.lsa;
        L.lb = A.vb + (int64_t)late * A.lsb;
        L.ea = A.va + (int64_t)early * A.lsa;
        L.eb = A.vb + (int64_t)early * A.lsb;
        L.efirst = early == 0;
    }
    L.zsh = (A.zs > 1 ? 1u : 0u) + (sizeof(T) == 8 ? 3u : 2u);  // zs is 1 or 2
    return L;
}

// velocity vector of one level (records va, vb; 2^zsh bytes per vb slot) at slot q
template <int DIM, typename T>
__device__ __forceinline__ void load_vec(const T* va, const T* vb, uint32_t zsh, uint32_t q, T* u)
{
    if constexpr (sizeof(T) == 8) {
        const double2 xy = ldv<double2>(va, q * 16u);
        u[0] = xy.x;
        u[1] = xy.y;
        if constexpr (DIM == 3) u[2] = ldv<double>(vb, q << zsh);
    } else if constexpr (DIM == 3) {
        const F3 v = ldv<F3>(va, q * 12u);
        u[0] = v.x;
        u[1] = v.y;
        u[2] = v.z;
    } else {
        const float2 xy = ldv<float2>(va, q * 8u);
        u[0] = xy.x;
        u[1] = xy.y;
    }
}

// Both levels' velocity at slot q.  ZP: the u_z values of a two-level
// float64 ring sit side by side per slot (vb = ring slot 0's u_z, ring slot
// 1's next to it), so one 16-byte load brings both: three loads per node
// instead of four.  a[2] and b[2] are then ring slots 0 and 1, not the
// earlier and later level; the callers swap the two z sums once when the
// earlier level is ring slot 1 (Levels::efirst false).
template <int DIM, int NLEV, typename T, bool ZP>
__device__ __forceinline__ void load_levels(const Levels<T>& Lv, const T* vb, uint32_t q, T* a, T* b)
{
    if constexpr (ZP) {
        static_assert(DIM == 3 && NLEV == 2 && sizeof(T) == 8, "paired u_z records: float64, 3D, two levels");
        const double2 xe = ldv<double2>(Lv.ea, q * 16u);
        const double2 xl = ldv<double2>(Lv.la, q * 16u);
        const double2 zz = ldv<double2>(vb, q * 16u);
        a[0] = xe.x;
        a[1] = xe.y;
        a[2] = zz.x;
        b[0] = xl.x;
        b[1] = xl.y;
        b[2] = zz.y;
    } else {
        load_vec<DIM, T>(Lv.ea, Lv.eb, Lv.zsh, q, a);
        if constexpr (NLEV == 2) load_vec<DIM, T>(Lv.la, Lv.lb, Lv.zsh, q, b);
    }
}

// Velocity at a stage point: P2 sums of both levels weighted (1 - theta,
// theta), or the single level of a stationary run.
template <int DIM, int NLEV, typename T, typename R, int ORD, bool ZP = false>
__device__ __forceinline__ void gather_vel(const Levels<T>& Lv, const T* vb, uint32_t mbase,
                                           const Stencil<DIM, R, ORD>& st, R theta, R* k)
{
    constexpr int NN = Stencil<DIM, R, ORD>::NN;
    R ua[DIM], ub[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        ua[i] = R(0);
        ub[i] = R(0);
    }
#pragma unroll
    for (int q = 0; q < NN; ++q) {
        const uint32_t slot = mbase + (uint32_t)st.idx[q];
        T a[DIM], b[DIM];
        load_levels<DIM, NLEV, T, ZP>(Lv, vb, slot, a, b);
#pragma unroll
        for (int i = 0; i < DIM; ++i) ua[i] = fma(st.phi[q], (R)a[i], ua[i]);
        if constexpr (NLEV == 2) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) ub[i] = fma(st.phi[q], (R)b[i], ub[i]);
        }
    }
    if constexpr (ZP) {
        const R z0 = ua[2], z1 = ub[2];
        ua[2] = Lv.efirst ? z0 : z1;
        ub[2] = Lv.efirst ? z1 : z0;
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) k[i] = NLEV == 2 ? fma(R(1) - theta, ua[i], theta * ub[i]) : ua[i];
}

// velocity at a lattice node: the nodal values (P2 interpolation is the
// identity there)
template <int DIM, int NLEV, typename T, typename R, bool ZP = false>
__device__ __forceinline__ void nodal_vel(const Levels<T>& Lv, const T* vb, uint32_t slot, R theta, R* k)
{
    T a[DIM], b[DIM];
    load_levels<DIM, NLEV, T, ZP>(Lv, vb, slot, a, b);
    if constexpr (ZP) {
        const T z0 = a[2], z1 = b[2];
        a[2] = Lv.efirst ? z0 : z1;
        b[2] = Lv.efirst ? z1 : z0;
    }
    if constexpr (NLEV == 2) {
#pragma unroll
        for (int i = 0; i < DIM; ++i) k[i] = fma(R(1) - theta, (R)a[i], theta * (R)b[i]);
    } else {
#pragma unroll
        for (int i = 0; i < DIM; ++i) k[i] = (R)a[i];
    }
}

// ------------------------------------------------ per-lane element cache
//
// At CFL 5 a stage offset is a fraction of a micro element, so most stage
// evaluations of a particle (84% on the shell, 78-89% on the swirl) fall in
// the element of the evaluation before.  With the cache, a lane keeps the
// nodal velocity values of its last element in LDS and gathers from the
// field only when the element changes: the texture path's tag lookups, which
// bound the uncached kernels, fall with the gathers.  Layout: chunk c (16
// bytes) of lane l at lds[c * kTB + l], so a wave's access to one chunk is
// one contiguous 1 KB row (no bank conflicts).  An element is identified by
// the block slot of its vertex 0 and the lattice indices of its vertices 1
// and 2 (vertex 3 is k + (1, 1, 1) for every element of base k, and the
// first three vertices fix the axis order).  The cached values are the
// gathered ones, summed in the gather's order, so the results are bitwise
// those of the uncached kernel.  Used for the raw values of one velocity
// level (stationary runs), of two float32 levels, and of the earlier of two
// float64 levels in paired u_z records (cached_vel_zp), within one interval
// of the velocity ring (the two levels do not change during the trace).
template <typename T, int NV>
struct ElemCache {
    static constexpr int NCH = (NV * (int)sizeof(T) + 15) / 16;  // 16-byte chunks per lane
    static constexpr int NVP = NCH * 16 / (int)sizeof(T);        // values with padding
    uint4* lds;
    uint64_t key;

    __device__ __forceinline__ void init(uint4* base)
    {
        lds = base + threadIdx.x;
        key = ~0ull;
    }
    // the element's key: its macro's slot base, base cell and axis ranks
    // (ranks r0, r1 fix r2); 9 bits per cell coordinate cover level 9
    static __device__ __forceinline__ uint64_t key_of(uint32_t mbase, const int* k, const int* r)
    {
        const uint32_t lo = ((uint32_t)k[0] << 22) | ((uint32_t)k[1] << 13) | ((uint32_t)k[2] << 4) |
                            (uint32_t)(r[0] * 3 + r[1]);
        return ((uint64_t)mbase << 32) | lo;
    }
    __device__ __forceinline__ bool take(uint64_t k)
    {
        const bool hit = k == key;
        key = k;
        return hit;
    }
    __device__ __forceinline__ void put(const T (&v)[NVP])
    {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            uint4 x;
            __builtin_memcpy(&x, reinterpret_cast<const char*>(v) + 16 * c, 16);
            lds[c * kTB] = x;
        }
    }
    __device__ __forceinline__ void get(T (&v)[NVP]) const
    {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const uint4 x = lds[c * kTB];
            __builtin_memcpy(reinterpret_cast<char*>(v) + 16 * c, &x, 16);
        }
    }
};

// The cache of one float64 level: (u_x, u_y) of the element's nodes in LDS
// (160 B per lane, one chunk per node), u_z in ten registers.  With all 30
// values in LDS (240 B) five blocks of 128 lanes fit a CU; split, eight fit
// (20 KB each) and the kernel's registers allow them.
struct ElemCacheSplit {
    static constexpr int NCH = 10;
    static constexpr int NVP = 30;
    uint4* lds;
    uint64_t key;
    double z[10];

    __device__ __forceinline__ void init(uint4* base)
    {
        lds = base + threadIdx.x;
        key = ~0ull;
#pragma unroll
        for (int q = 0; q < 10; ++q) z[q] = 0.0;
    }
    static __device__ __forceinline__ uint64_t key_of(uint32_t mbase, const int* k, const int* r)
    {
        return ElemCache<double, 30>::key_of(mbase, k, r);
    }
    __device__ __forceinline__ bool take(uint64_t k)
    {
        const bool hit = k == key;
        key = k;
        return hit;
    }
    __device__ __forceinline__ void put(const double (&v)[30])
    {
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            double2 xy = {v[3 * q], v[3 * q + 1]};
            uint4 x;
            __builtin_memcpy(&x, &xy, 16);
            lds[q * kTB] = x;
            z[q] = v[3 * q + 2];
        }
    }
    __device__ __forceinline__ void get(double (&v)[30]) const
    {
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const uint4 x = lds[q * kTB];
            double2 xy;
            __builtin_memcpy(&xy, &x, 16);
            v[3 * q] = xy.x;
            v[3 * q + 1] = xy.y;
            v[3 * q + 2] = z[q];
        }
    }
};

// the nodal velocities of one element, v[(q * NLEV + level) * 3 + i] (3D P2,
// records without paired u_z; idx: the element's node indices)
template <int NLEV, typename T, int NVP>
__device__ __forceinline__ void fetch_elem(const Levels<T>& Lv, uint32_t mbase, const int* idx, T (&v)[NVP])
{
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const uint32_t slot = mbase + (uint32_t)idx[q];
        load_vec<3, T>(Lv.ea, Lv.eb, Lv.zsh, slot, v + q * 3 * NLEV);
        if constexpr (NLEV == 2) load_vec<3, T>(Lv.la, Lv.lb, Lv.zsh, slot, v + q * 6 + 3);
    }
#pragma unroll
    for (int i = 30 * NLEV; i < NVP; ++i) v[i] = T(0);
}

// the P2 sums of gather_vel (same operations, same order) from cached values
template <int NLEV, typename T, typename R>
__device__ __forceinline__ void sum_elem(const T* v, const R* phi, R theta, R* k)
{
    R ua[3], ub[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ua[i] = R(0);
        ub[i] = R(0);
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) {
#pragma unroll
        for (int i = 0; i < 3; ++i) ua[i] = fma(phi[q], (R)v[q * 3 * NLEV + i], ua[i]);
        if constexpr (NLEV == 2) {
#pragma unroll
            for (int i = 0; i < 3; ++i) ub[i] = fma(phi[q], (R)v[q * 6 + 3 + i], ub[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) k[i] = NLEV == 2 ? fma(R(1) - theta, ua[i], theta * ub[i]) : ua[i];
}

// Velocity at a located stage point through the cache: on a new element the
// lane computes its node indices (the stencil comes without them), gathers
// the nodes and stores them; then every lane sums from its cached copy.
// Counts the lane's hits.
template <int NLEV, typename T, typename R, typename C>
__device__ __forceinline__ void cached_vel(C& cache, const Levels<T>& Lv, uint32_t mbase, const Stencil<3, R, 2>& st,
                                           R theta, R* k, uint32_t& nhit)
{
    T v[C::NVP];
    if (!cache.take(C::key_of(mbase, st.k, st.r))) {
        int idx[10];
        stencil_idx<3, 2>(st.k, st.r, idx);
        fetch_elem<NLEV, T>(Lv, mbase, idx, v);
        cache.put(v);
    } else {
        ++nhit;
    }
    cache.get(v);
    sum_elem<NLEV, T, R>(v, st.phi, theta, k);
}

// The same through the cache for two float64 levels in paired u_z records
// (ZP): a lane keeps only the earlier level's (u_x, u_y) of its element's
// nodes (20 values, 160 bytes; the two levels do not change during a trace
// over one interval) and gathers the later level's (u_x, u_y) and the u_z
// pair at each evaluation: 20 loads instead of 30 on a hit.  Keeping the
// u_z pair too (40 values) halves the blocks that fit a CU and was slower
// (4.50 against 3.90 ms on the 1.7e7-particle plumes).  The sums are those
// of gather_vel, in its order (bitwise the uncached result).
template <typename C>
__device__ __forceinline__ void cached_vel_zp(C& cache, const Levels<double>& Lv, const double* vb, uint32_t mbase,
                                               const Stencil<3, double, 2>& st, double theta, double* k,
                                               uint32_t& nhit)
{
    double v[C::NVP];
    int idx[10];
    stencil_idx<3, 2>(st.k, st.r, idx);
    if (!cache.take(C::key_of(mbase, st.k, st.r))) {
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const double2 xe = ldv<double2>(Lv.ea, (mbase + (uint32_t)idx[q]) * 16u);
            v[2 * q] = xe.x;
            v[2 * q + 1] = xe.y;
        }
        cache.put(v);
    } else {
        ++nhit;
    }
    cache.get(v);
    double ua[3] = {0.0, 0.0, 0.0}, ub[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const uint32_t slot = mbase + (uint32_t)idx[q];
        const double2 xl = ldv<double2>(Lv.la, slot * 16u);
        const double2 zz = ldv<double2>(vb, slot * 16u);
        const double ph = st.phi[q];
        ua[0] = fma(ph, v[2 * q], ua[0]);
        ua[1] = fma(ph, v[2 * q + 1], ua[1]);
        ua[2] = fma(ph, zz.x, ua[2]);
        ub[0] = fma(ph, xl.x, ub[0]);
        ub[1] = fma(ph, xl.y, ub[1]);
        ub[2] = fma(ph, zz.y, ub[2]);
    }
    const double z0 = ua[2], z1 = ub[2];
    ua[2] = Lv.efirst ? z0 : z1;
    ub[2] = Lv.efirst ? z1 : z0;
#pragma unroll
    for (int i = 0; i < 3; ++i) k[i] = fma(1.0 - theta, ua[i], theta * ub[i]);
}

template <int DIM, typename T, typename R, int ORD>
__device__ __forceinline__ R gather_scalar(const TraceArgs<T>& A, uint32_t mbase, const Stencil<DIM, R, ORD>& st)
{
    constexpr int NN = Stencil<DIM, R, ORD>::NN;
    R acc = R(0);
#pragma unroll
    for (int q = 0; q < NN; ++q)
        acc = fma(st.phi[q], (R)ldv<T>(A.cs, (mbase + (uint32_t)st.idx[q]) * (uint32_t)sizeof(T)), acc);
    return acc;
}

template <int DIM>
__device__ __forceinline__ int own_lat_idx(uint64_t e)
{
    const int I = (int)((e >> 24) & 0xfffu), J = (int)((e >> 12) & 0xfffu), K = (int)(e & 0xfffu);
    if constexpr (DIM == 2) return tri_n(I) + J;
    else return tet_n(I) + tri_n(J) + K;
}

// A value the whole wave shares (derived from kernel arguments), held in
// scalar registers so that stage-dependent choices between such values are
// scalar selects.
__device__ __forceinline__ double uniform64(double x)
{
    int v[2];
    __builtin_memcpy(v, &x, 8);
    v[0] = __builtin_amdgcn_readfirstlane(v[0]);
    v[1] = __builtin_amdgcn_readfirstlane(v[1]);
    double r;
    __builtin_memcpy(&r, v, 8);
    return r;
}

__device__ __forceinline__ float uniform32(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// A particle at rest (zero velocity at its DoF, e.g. on a no-slip wall or a
// stagnation line) stays at its DoF.  P2 interpolation at a node is the
// nodal value, so an evaluation there needs no location and one nodal load.
// `home` tracks Y == the DoF position (no departure-point update has changed
// a bit of it): the scalar step then reads the DoF's own value, and the
// general-tableau loop evaluates a stage point y == Y of such a particle
// from the nodal values.  (The RK4 chain locates every stage point after the
// first: a branch around the evaluation costs every wave register copies of
// the element cache, more than the at-rest lanes save.)
template <int DIM>
__device__ __forceinline__ bool same_point(const double* y, const double* x)
{
    bool same = true;
#pragma unroll
    for (int i = 0; i < DIM; ++i) same &= y[i] == x[i];
    return same;
}

// this block's word of statistic row `which`
__device__ __forceinline__ unsigned long long* stat_word(unsigned long long* stats, int which)
{
    return stats + which * kStatSpread + (blockIdx.x & (kStatSpread - 1));
}

// per-wave counts of the lane flags, one atomic per non-zero count
__device__ __forceinline__ void count_flags(unsigned long long* stats, bool active, unsigned flags)
{
    const unsigned long long nact = __popcll(__ballot(active));
    const unsigned long long no = __popcll(__ballot((flags & LF_OUTSIDE) != 0));
    const unsigned long long nm = __popcll(__ballot((flags & LF_MULTIHOP) != 0));
    const unsigned long long nb = __popcll(__ballot((flags & LF_BRUTE) != 0));
    const unsigned long long nt = __popcll(__ballot((flags & LF_TIEBAND) != 0));
    const unsigned long long nn = __popcll(__ballot((flags & LF_NAN) != 0));
    const unsigned long long nf = __popcll(__ballot((flags & LF_FALLBACK) != 0));
    if ((threadIdx.x & 63) == 0) {
        if (nact) atomicAdd(stat_word(stats, ST_PARTICLES), nact);
        if (no) atomicAdd(stat_word(stats, ST_OUTSIDE), no);
        if (nm) atomicAdd(stat_word(stats, ST_MULTIHOP), nm);
        if (nb) atomicAdd(stat_word(stats, ST_BRUTE), nb);
        if (nt) atomicAdd(stat_word(stats, ST_TIEBAND), nt);
        if (nn) atomicAdd(stat_word(stats, ST_NAN), nn);
        if (nf) atomicAdd(stat_word(stats, ST_FALLBACK), nf);
    }
}

// one atomic per wave: the summed lane counts of cache lookups and hits
__device__ __forceinline__ void count_cache(unsigned long long* stats, uint32_t nlook, uint32_t nhit)
{
    unsigned long long a = nlook, b = nhit;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0 && a) {
        atomicAdd(stat_word(stats, ST_CACHE_LOOKUPS), a);
        atomicAdd(stat_word(stats, ST_CACHE_HITS), b);
    }
}

// Surrogate finish: the tile's checked particles decide whether it keeps
// the surrogate's departure points (every thread of the block must call).
// Counts the checked particles and the largest residual into the stats.
// Whether any thread of the block has p (every thread must call).  word:
// a 4-byte LDS word the block does not use otherwise until this returns
// (the trace kernels lend the first word of their cache array, which their
// traces write only later; a library reduction would take LDS of its own).
__device__ __forceinline__ bool block_any(bool p, unsigned* word)
{
    if (threadIdx.x == 0) *word = 0u;
    __syncthreads();
    if (__ballot(p) != 0 && (threadIdx.x & 63) == 0) atomicOr(word, 1u);
    __syncthreads();
    const bool any = *word != 0u;
    __syncthreads();
    return any;
}

__device__ __forceinline__ bool finish_keep(const double* __restrict__ X, const double* __restrict__ xc,
                                            const unsigned char* __restrict__ checked, int dim, int64_t xstride,
                                            double tol_half, int64_t pid, bool active, bool& chk,
                                            unsigned long long* stats, unsigned* lds_word)
{
    const unsigned char cv = active ? checked[pid] : 0;
    chk = cv == 1;
    double r = cv == 2 ? (double)INFINITY : 0.0;  // selected but not traced: the tile falls back
    if (chk) {
        for (int i = 0; i < dim; ++i) {
            const double e = fabs(X[(int64_t)i * xstride + pid] - xc[(int64_t)i * xstride + pid]);
            r = (e > r || e != e) ? e : r;
        }
        if (r != r) r = INFINITY;
    }
    const bool keep = !block_any(cv != 0 && !(r <= tol_half), lds_word);
    // one atomic per wave for the count and the largest residual (the bits of
    // a non-negative double order like the double)
    unsigned long long bits;
    __builtin_memcpy(&bits, &r, sizeof bits);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(bits, off, 64);
        bits = o > bits ? o : bits;
    }
    const unsigned long long cnt = __popcll(__ballot(chk));
    if ((threadIdx.x & 63) == 0 && cnt) {
        atomicMax(stat_word(stats, ST_MAXRES_BITS), bits);
        atomicAdd(stat_word(stats, ST_CHECKED), cnt);
    }
    return keep;
}

// --------------------------------------------------------------- fp64 trace

// T is the storage type of the fields: double (MMOC_FP64) or float
// (MMOC_FP32_FIELDS: float32 records, float64 arithmetic throughout).
// ZP: the u_z records of a two-level float64 ring are paired per slot.
// GENERIC: a general explicit Runge-Kutta method from A.rk (the paper uses
// RK4 and notes that any explicit RK method applies, Sec. 3.1); otherwise the
// classical RK4 with its weights folded into the code.
// CACHE: the per-lane element cache (3D P2 RK4, one velocity level or two
// float32 levels); the block's LDS then holds the cache instead of the
// geometry copy.
template <int DIM, int NLEV, int BLEND, typename T, bool GENERIC, int ORD, bool ZP = false, bool CACHE = false>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(CACHE ? 4 : MMOC_WPE_FP64)))
void trace_fp64_kernel(const TraceArgs<T> A, const MacroGeo* __restrict__ geo, T* __restrict__ c_hat,
                       double* __restrict__ X, unsigned long long* __restrict__ stats)
{
    static_assert(!CACHE || (DIM == 3 && ORD == 2 && !GENERIC &&
                             (ZP ? NLEV == 2 && sizeof(T) == 8 : (NLEV == 1 || sizeof(T) == 4))),
                  "element cache: 3D P2 RK4, one level, float32 records or paired float64 levels");
    using Cache = std::conditional_t<NLEV == 1 && sizeof(T) == 8, ElemCacheSplit, ElemCache<T, ZP ? 20 : 30 * NLEV>>;
    // the cached kernels keep no geometry in LDS (their whole LDS budget is
    // the cache: the unused array is not allocated)
    __shared__ MacroGeo sgeo[kLdsGeo];
    __shared__ uint4 lcache[CACHE ? Cache::NCH * kTB : 1];
    const MacroGeo* sg = nullptr;
    if constexpr (!CACHE) sg = stage_geo(geo, A.nm, sgeo);
    const int64_t t = logical_block(A.xcd_log2) * kTB + threadIdx.x;
    // a lane traces particle pid: t itself, or the t-th entry of a list
    // (entries outside [0, N) are skipped)
    const bool listed = t < A.n && (!A.n_dev || (unsigned long long)t < *A.n_dev);
    const int64_t pid = listed && A.order ? (int64_t)A.order[t] : t;
    const bool active = listed && (uint64_t)pid < (uint64_t)A.xstride;
    unsigned flags = 0;
    uint32_t nlook = 0, nhit = 0;
    Cache cache;
    if constexpr (CACHE) cache.init(lcache);
    bool keep = false, chk = false;
    if (A.checked)
        keep = finish_keep(X, A.xcheck, A.checked, DIM, A.xstride, A.tol_half, t, active, chk, stats,
                           reinterpret_cast<unsigned*>(lcache));
    if (active) {
        const uint64_t e = A.owned[pid];
        int M;
        double Y[DIM];
        dof_position<DIM, BLEND>(geo, e, A.lat_m, M, Y);
        bool home = true;
        uint32_t mbase = (uint32_t)M * (uint32_t)A.npm;
        const uint32_t own_slot = mbase + (uint32_t)own_lat_idx<DIM>(e);
        // surrogate finish: a tile that passed the check keeps the departure
        // points (uniform over the block: tiles are blocks), checked
        // particles their RK4 ones; a tile that failed is traced
        if (A.checked && !keep && !chk) flags |= LF_FALLBACK;
        if (keep) {
            const double* src = chk ? A.xcheck : X;
#pragma unroll
            for (int i = 0; i < DIM; ++i) Y[i] = src[(int64_t)i * A.xstride + pid];
            home = false;
        }
        const double h = uniform64(A.dt / (double)A.substeps);
        const double hh = uniform64(0.5 * h);
        const double h6 = uniform64(h / 6.0);
        const double invS = uniform64(1.0 / (double)A.substeps);
        double s[DIM], l0, lmin;
        Stencil<DIM, double, ORD> st;
        // velocity at stage point y and stage time theta (Sec. 2.3.2: walk
        // from the previous macro, micro element, P2 sums of both levels)
        auto velocity = [&](const double* y, const Levels<T>& Lv, double theta, double* k) {
            l0 = ref_at<DIM, BLEND>(geo, M, y, s, sg);
            lmin = lam_min<DIM, double>(l0, s);
            if (lmin < -A.eps_in) {
                const unsigned r = walk64<DIM, BLEND>(geo, A.nm, A.max_hops, A.eps_in, M, y[0], y[1],
                                                     DIM == 3 ? y[DIM - 1] : 0.0);
                flags |= r >> 27;
                M = (int)(r & ((1u << 27) - 1));
                mbase = (uint32_t)M * (uint32_t)A.npm;
                l0 = ref_at<DIM, BLEND>(geo, M, y, s, sg);
                lmin = lam_min<DIM, double>(l0, s);
            }
            micro<DIM, double, false, ORD, !CACHE>(s, l0, lmin, A.level_n, st);
            if constexpr (CACHE) {
                ++nlook;
                if constexpr (ZP) cached_vel_zp(cache, Lv, A.vb, mbase, st, theta, k, nhit);
                else cached_vel<NLEV, T, double>(cache, Lv, mbase, st, theta, k, nhit);
            } else {
                gather_vel<DIM, NLEV, T, double, ORD, ZP>(Lv, A.vb, mbase, st, theta, k);
            }
        };
        const int nsub = keep ? 0 : A.substeps * A.n_int;
        if constexpr (GENERIC) {
#pragma unroll 1
            for (int j = 0; j < nsub; ++j) {
                double K[kMaxStages][DIM];
#pragma unroll
                for (int q = 0; q < kMaxStages; ++q) {
                    if (q < A.rk.s) {
                        // y_q = Y - h sum_{l<q} a_ql k_l at theta = 1 - (j + c_q)/S
                        double y[DIM];
#pragma unroll
                        for (int i = 0; i < DIM; ++i) {
                            double sum = 0.0;
#pragma unroll
                            for (int l = 0; l < q; ++l) sum = fma(A.rk.a[q * kMaxStages + l], K[l][i], sum);
                            y[i] = fma(-h, sum, Y[i]);
                        }
                        double theta;
                        const Levels<T> Lv = levels_at<NLEV, T, double>(A, ((double)j + A.rk.c[q]) * invS, theta);
                        if ((j == 0 && q == 0) || (home && same_point<DIM>(y, Y)))
                            nodal_vel<DIM, NLEV, T, double, ZP>(Lv, A.vb, own_slot, theta, K[q]);
                        else
                            velocity(y, Lv, theta, K[q]);
                    }
                }
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    double sum = 0.0;
#pragma unroll
                    for (int q = 0; q < kMaxStages; ++q)
                        if (q < A.rk.s) sum = fma(A.rk.b[q], K[q][i], sum);
                    const double yn = fma(-h, sum, Y[i]);
                    home = home && yn == Y[i];
                    Y[i] = yn;
                }
            }
        } else if (nsub > 0) {
            // RK4 as one chain of 4 S evaluations: evaluation e is stage
            // e mod 4 of sub-step e / 4, at (j + a_s)/S intervals back
            // (a_s = 0, 1/2, 1/2, 1; one interval: theta = 1 - (j + a_s)/S).
            // The first is the particle's own DoF (the nodal value); every
            // later one is located, so the loop has no divergent branch
            // around the evaluation (a particle at rest evaluates at its DoF
            // through the element like any other point).
            double ks[DIM], acc[DIM], y[DIM];
            {
                double theta;
                const Levels<T> Lv = levels_at<NLEV, T, double>(A, 0.0, theta);
                nodal_vel<DIM, NLEV, T, double, ZP>(Lv, A.vb, own_slot, theta, ks);
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) acc[i] = 0.0;
            const int neval = 4 * nsub;
#pragma unroll 1
            for (int e = 0; e < neval; ++e) {
                const int stg = e & 3;
                // k1 + 2 k2 + 2 k3 + k4 accumulated in stage order; next stage point
                const double wst = (stg == 0 || stg == 3) ? 1.0 : 2.0;
#pragma unroll
                for (int i = 0; i < DIM; ++i) acc[i] = fma(wst, ks[i], acc[i]);
                if (stg == 3) {
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        const double yn = fma(-h6, acc[i], Y[i]);
                        home = home && yn == Y[i];
                        Y[i] = yn;
                        y[i] = yn;
                        acc[i] = 0.0;
                    }
                } else {
                    const double cnext = stg == 2 ? h : hh;
#pragma unroll
                    for (int i = 0; i < DIM; ++i) y[i] = fma(-cnext, ks[i], Y[i]);
                }
                if (e + 1 < neval) {
                    const int e1 = e + 1, s1 = e1 & 3;
                    const double as = s1 == 0 ? 0.0 : (s1 == 3 ? 1.0 : 0.5);
                    double theta;
                    const Levels<T> Lv = levels_at<NLEV, T, double>(A, ((double)(e1 >> 2) + as) * invS, theta);
                    velocity(y, Lv, theta, ks);
                }
            }
        }
        // step (iii): the scalar at the departure point
        double v;
        if (home) {
            v = (double)ldv<T>(A.cs, own_slot * (uint32_t)sizeof(T));
        } else {
            l0 = ref_at<DIM, BLEND>(geo, M, Y, s, sg);
            lmin = lam_min<DIM, double>(l0, s);
            if (lmin < -A.eps_in) {
                const unsigned r =
                    walk64<DIM, BLEND>(geo, A.nm, A.max_hops, A.eps_in, M, Y[0], Y[1], DIM == 3 ? Y[DIM - 1] : 0.0);
                flags |= r >> 27;
                M = (int)(r & ((1u << 27) - 1));
                mbase = (uint32_t)M * (uint32_t)A.npm;
                l0 = ref_at<DIM, BLEND>(geo, M, Y, s, sg);
                lmin = lam_min<DIM, double>(l0, s);
            }
            micro<DIM, double, false, ORD>(s, l0, lmin, A.level_n, st);
            v = gather_scalar<DIM, T, double>(A, mbase, st);
        }
        bool bad = v != v;
#pragma unroll
        for (int i = 0; i < DIM; ++i) bad |= Y[i] != Y[i];
        if (bad) flags |= LF_NAN;
        if (c_hat) c_hat[pid] = (T)v;
        if (A.c_next) A.c_next[own_slot] = (T)v;
        if (X) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) X[(int64_t)i * A.xstride + pid] = Y[i];
        }
    }
    count_flags(stats, active, flags);
    if constexpr (CACHE) count_cache(stats, nlook, nhit);
}

// --------------------------------------------------------- fp32 mixed trace

template <int DIM, int BLEND>
struct Geo32 {
    double v0[DIM];
    float bi[DIM][DIM];
    double pn[3];
    double pc;

    template <typename P>
    __device__ __forceinline__ void load(P g, int M)
    {
#pragma unroll
        for (int i = 0; i < DIM; ++i) v0[i] = g[M].v0[i];
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) bi[r][c] = g[M].binvf[r * 3 + c];
        if constexpr (BLEND) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) pn[i] = g[M].pn[i];
            pc = g[M].pc;
        }
    }

    // Reference coordinates in float32: the offset from the macro origin is
    // formed in float64 (the only float64 work of an ordinary stage), then
    // rounded and mapped with the float32 inverse.
    __device__ __forceinline__ float ref(const double* y, float* s) const
    {
        float p[DIM];
        if constexpr (BLEND) {
            const double nz = dotd<DIM>(pn, y);
            const double r = sqrt64(dotd<DIM>(y, y));
            const double f = pc * r * recip64(nz);
#pragma unroll
            for (int i = 0; i < DIM; ++i) p[i] = (float)fma(y[i], f, -v0[i]);
        } else {
#pragma unroll
            for (int i = 0; i < DIM; ++i) p[i] = (float)(y[i] - v0[i]);
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            float acc = bi[a][0] * p[0];
#pragma unroll
            for (int i = 1; i < DIM; ++i) acc = fmaf(bi[a][i], p[i], acc);
            s[a] = acc;
        }
        float sum = s[0];
#pragma unroll
        for (int a = 1; a < DIM; ++a) sum += s[a];
        return 1.0f - sum;
    }
};

// float32 reference coordinates of y in macro M (geometry read per
// evaluation, through scalar loads when the wave is in one macro)
template <int DIM, int BLEND>
__device__ __forceinline__ float ref32_at(const MacroGeo* __restrict__ geo, int M, const double* y, float* s,
                                          const MacroGeo* sgeo = nullptr)
{
    const int M0 = __builtin_amdgcn_readfirstlane(M);
    Geo32<DIM, BLEND> G;
    if (__ballot(M != M0) == 0) {
        G.load((ConstGeo)geo, M0);
        const float l0 = G.ref(y, s);
        __asm__ volatile("");
        return l0;
    }
    if (sgeo) G.load((LdsGeo)sgeo, M);
    else G.load(geo, M);
    return G.ref(y, s);
}

// The float64 re-evaluation of a location whose macro float32 could not
// decide: with `walk`, the macro walk in float64, then the micro element in
// float64
// (shape functions handed back in float32; node indices only with IDX, the
// cached kernels take them from the element's base cell and axis ranks).
// Out of line: it runs for a small fraction of the evaluations and must not
// cost the hot loop registers.
template <int DIM, int BLEND, int ORD, bool IDX = true>
__device__ __noinline__ unsigned locate64(const MacroGeo* __restrict__ geo, int nm, int max_hops, double eps, int M,
                                          int level_n, int walk, double y0, double y1, double y2,
                                          Stencil<DIM, float, ORD>* out)
{
    unsigned r = (unsigned)M;
    if (walk) r = walk64<DIM, BLEND>(geo, nm, max_hops, eps, M, y0, y1, y2);
    const int M2 = (int)(r & ((1u << 27) - 1));
    Geo64<DIM, BLEND> G;
    G.load(geo, M2);
    const double y[3] = {y0, y1, y2};
    double s[DIM];
    const double l0 = G.ref(y, s);
    const double lmin = lam_min<DIM, double>(l0, s);
    Stencil<DIM, double, ORD> st;
    micro<DIM, double, false, ORD, IDX>(s, l0, lmin, level_n, st);
#pragma unroll
    for (int q = 0; q < Stencil<DIM, double, ORD>::NN; ++q) {
        if constexpr (IDX) out->idx[q] = st.idx[q];
        out->phi[q] = (float)st.phi[q];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out->k[i] = st.k[i];
        out->r[i] = st.r[i];
    }
    return r;
}

// Location of a stage point in float32.  A macro decision that float32
// cannot take with certainty -- the smallest barycentric within eps32_macro
// of zero on a face that has a neighbour, or a macro change -- is re-taken
// in float64, and so is a micro decision within eps32_micro * n of a tie
// (in line: the macro is certain then, so only its float64 barycentrics and
// the micro element from them are needed).  Near a boundary face there is no
// second macro to choose: the point stays, and its element is selected from
// the clamped barycentrics as in float64.
template <int DIM, int BLEND, int ORD, bool IDX = true>
__device__ __forceinline__ void locate32(const TraceArgs<float>& A, int& M, uint32_t& mbase, const double* y,
                                         Stencil<DIM, float, ORD>& st, unsigned& flags, const MacroGeo* sg = nullptr)
{
    float s[DIM];
    const float l0 = ref32_at<DIM, BLEND>(A.geo, M, y, s, sg);
    const float lmin = lam_min<DIM, float>(l0, s);
    bool macro_redo = lmin < A.eps32_macro;
    if (macro_redo && lmin > -A.eps32_macro) {
        // inside the band: only faces with a neighbour carry a decision
        const int32_t* nb = A.geo[M].nbr;
        bool interior = false;
#pragma unroll
        for (int k = 0; k <= DIM; ++k) {
            const float lk = k == 0 ? l0 : s[k - 1];
            interior |= (lk < A.eps32_macro) && (nb[k] >= 0);
        }
        macro_redo = interior;
    }
    if (macro_redo && lmin > -A.eps32_macro) {
        // The float64 tie-break: the barycentrics of the current macro in
        // float64.  Inside (the float64 walk would stay) -- the common case of
        // a point on or next to an interior face -- the micro element follows
        // from them; otherwise the full float64 re-location below walks.
        double s64[DIM];
        const double l064 = ref_at<DIM, BLEND>(A.geo, M, y, s64, sg);
        const double lmin64 = lam_min<DIM, double>(l064, s64);
        if (lmin64 >= -A.eps_in) {
            flags |= LF_TIEBAND;
            float sf[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) sf[i] = (float)s64[i];
            micro<DIM, float, false, ORD, IDX>(sf, (float)l064, (float)lmin64, A.level_n, st);
            return;
        }
    }
    bool redo = macro_redo;
    if (!macro_redo) {
        if (A.eps32_micro > 0.0f) {
            const float gap = micro<DIM, float, true, ORD, IDX>(s, l0, lmin, A.level_n, st);
            if (gap < A.eps32_micro * (float)A.level_n) {
                // a micro tie in a certain macro: the float64 barycentrics
                // of this macro and the micro element from them, in line
                flags |= LF_TIEBAND;
                double s64[DIM];
                const double l064 = ref_at<DIM, BLEND>(A.geo, M, y, s64, sg);
                const double lmin64 = lam_min<DIM, double>(l064, s64);
                Stencil<DIM, double, ORD> st64;
                micro<DIM, double, false, ORD, IDX>(s64, l064, lmin64, A.level_n, st64);
#pragma unroll
                for (int q = 0; q < Stencil<DIM, double, ORD>::NN; ++q) {
                    st.phi[q] = (float)st64.phi[q];
                    if constexpr (IDX) st.idx[q] = st64.idx[q];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    st.k[i] = st64.k[i];
                    st.r[i] = st64.r[i];
                }
            }
        } else {
            micro<DIM, float, false, ORD, IDX>(s, l0, lmin, A.level_n, st);
        }
    }
    if (redo) {
        if (!macro_redo || lmin > -A.eps32_macro) flags |= LF_TIEBAND;
        Stencil<DIM, float, ORD> s64;
        const unsigned r = locate64<DIM, BLEND, ORD, IDX>(A.geo, A.nm, A.max_hops, A.eps_in, M, A.level_n, macro_redo, y[0],
                                                     y[1], DIM == 3 ? y[DIM - 1] : 0.0, &s64);
        flags |= r >> 27;
        M = (int)(r & ((1u << 27) - 1));
        mbase = (uint32_t)M * (uint32_t)A.npm;
        st = s64;
    }
}

template <int DIM, int NLEV, int BLEND, int ORD, bool CACHE = false>
__global__ __launch_bounds__(kTB) __attribute__((amdgpu_waves_per_eu(CACHE && NLEV == 2 ? 3 : MMOC_WPE_FP32)))
void trace_fp32_kernel(const TraceArgs<float> A)
{
    static_assert(!CACHE || (DIM == 3 && ORD == 2), "element cache: 3D P2");
    using Cache = ElemCache<float, 30 * NLEV>;
    __shared__ MacroGeo sgeo[kLdsGeo];
    __shared__ uint4 lcache[CACHE ? Cache::NCH * kTB : 1];
    const MacroGeo* sg = nullptr;
    if constexpr (!CACHE) sg = stage_geo(A.geo, A.nm, sgeo);
    const int64_t t = logical_block(A.xcd_log2) * kTB + threadIdx.x;
    // a lane traces particle pid: t itself, or the t-th entry of a list
    // (entries outside [0, N) are skipped)
    const bool listed = t < A.n && (!A.n_dev || (unsigned long long)t < *A.n_dev);
    const int64_t pid = listed && A.order ? (int64_t)A.order[t] : t;
    const bool active = listed && (uint64_t)pid < (uint64_t)A.xstride;
    unsigned flags = 0;
    uint32_t nlook = 0, nhit = 0;
    Cache cache;
    if constexpr (CACHE) cache.init(lcache);
    bool keep = false, chk = false;
    if (A.checked)
        keep = finish_keep(A.X, A.xcheck, A.checked, DIM, A.xstride, A.tol_half, t, active, chk, A.stats,
                           reinterpret_cast<unsigned*>(lcache));
    if (active) {
        const uint64_t e = A.owned[pid];
        int M;
        double Y[DIM];
        dof_position<DIM, BLEND>(A.geo, e, A.lat_m, M, Y);
        bool home = true;
        uint32_t mbase = (uint32_t)M * (uint32_t)A.npm;
        const uint32_t own_slot = mbase + (uint32_t)own_lat_idx<DIM>(e);
        if (A.checked && !keep && !chk) flags |= LF_FALLBACK;
        if (keep) {
            const double* src = chk ? A.xcheck : A.X;
#pragma unroll
            for (int i = 0; i < DIM; ++i) Y[i] = src[(int64_t)i * A.xstride + pid];
            home = false;
        }
        const double hd = A.dt / (double)A.substeps;
        const float h = uniform32((float)hd);
        const float hh = uniform32(0.5f * h);
        const float h6 = uniform32(h / 6.0f);
        const double invSd = uniform64(1.0 / (double)A.substeps);
        Stencil<DIM, float, ORD> st;
        const int nsub = keep ? 0 : A.substeps * A.n_int;
        if (nsub > 0) {
            // one chain of 4 S evaluations, as in the float64 kernel: the
            // first at the particle's own DoF, every later one located
            float ks[DIM], acc[DIM];
            double y[DIM];
            {
                float theta;
                const Levels<float> Lv = levels_at<NLEV, float, float>(A, 0.0, theta);
                nodal_vel<DIM, NLEV, float, float>(Lv, A.vb, own_slot, theta, ks);
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) acc[i] = 0.0f;
            const int neval = 4 * nsub;
#pragma unroll 1
            for (int e = 0; e < neval; ++e) {
                const int stg = e & 3;
                const float wst = (stg == 0 || stg == 3) ? 1.0f : 2.0f;
#pragma unroll
                for (int i = 0; i < DIM; ++i) acc[i] = fmaf(wst, ks[i], acc[i]);
                if (stg == 3) {
                    // departure point accumulated in float64
#pragma unroll
                    for (int i = 0; i < DIM; ++i) {
                        const double yn = Y[i] - (double)(h6 * acc[i]);
                        home = home && yn == Y[i];
                        Y[i] = yn;
                        y[i] = yn;
                        acc[i] = 0.0f;
                    }
                } else {
                    const float cnext = stg == 2 ? h : hh;
#pragma unroll
                    for (int i = 0; i < DIM; ++i) y[i] = Y[i] - (double)(cnext * ks[i]);
                }
                if (e + 1 < neval) {
                    const int e1 = e + 1, s1 = e1 & 3;
                    const double as = s1 == 0 ? 0.0 : (s1 == 3 ? 1.0 : 0.5);
                    float theta;
                    const Levels<float> Lv = levels_at<NLEV, float, float>(A, ((double)(e1 >> 2) + as) * invSd, theta);
                    locate32<DIM, BLEND, ORD, !CACHE>(A, M, mbase, y, st, flags, sg);
                    if constexpr (CACHE) {
                        ++nlook;
                        cached_vel<NLEV, float, float>(cache, Lv, mbase, st, theta, ks, nhit);
                    } else {
                        gather_vel<DIM, NLEV, float, float>(Lv, A.vb, mbase, st, theta, ks);
                    }
                }
            }
        }
        float v;
        if (home) {
            v = ldv<float>(A.cs, own_slot * 4u);
        } else {
            locate32<DIM, BLEND, ORD>(A, M, mbase, Y, st, flags, sg);
            v = gather_scalar<DIM, float, float>(A, mbase, st);
        }
        bool bad = v != v;
#pragma unroll
        for (int i = 0; i < DIM; ++i) bad |= Y[i] != Y[i];
        if (bad) flags |= LF_NAN;
        if (A.c_hat) A.c_hat[pid] = v;
        if (A.c_next) A.c_next[own_slot] = v;
        if (A.X) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) A.X[(int64_t)i * A.xstride + pid] = Y[i];
        }
    }
    count_flags(A.stats, active, flags);
    if constexpr (CACHE) count_cache(A.stats, nlook, nhit);
}

// ------------------------------------------------- scalar at given points

// chat_i = c_h^n(X_i) for departure points produced elsewhere (the
// surrogate): the walk starts in the particle's own macro.
template <int DIM, int BLEND, typename T, int ORD>
__global__ __launch_bounds__(kTB) void scalar_eval_fp64_kernel(const TraceArgs<T> A)
{
    const int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x;
    const bool active = t < A.n;
    unsigned flags = 0;
    if (active) {
        int M = (int)(A.owned[t] >> 36);
        double Y[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) Y[i] = A.X[(int64_t)i * A.xstride + t];
        double s[DIM];
        double l0 = ref_at<DIM, BLEND>(A.geo, M, Y, s);
        double lmin = lam_min<DIM, double>(l0, s);
        if (lmin < -A.eps_in) {
            const unsigned r =
                walk64<DIM, BLEND>(A.geo, A.nm, A.max_hops, A.eps_in, M, Y[0], Y[1], DIM == 3 ? Y[DIM - 1] : 0.0);
            flags |= r >> 27;
            M = (int)(r & ((1u << 27) - 1));
            l0 = ref_at<DIM, BLEND>(A.geo, M, Y, s);
            lmin = lam_min<DIM, double>(l0, s);
        }
        Stencil<DIM, double, ORD> st;
        micro<DIM, double, false, ORD>(s, l0, lmin, A.level_n, st);
        const double v = gather_scalar<DIM, T, double>(A, (uint32_t)M * (uint32_t)A.npm, st);
        if (v != v) flags |= LF_NAN;
        A.c_hat[t] = (T)v;
    }
    (void)flags;
}

template <int DIM, int BLEND, int ORD>
__global__ __launch_bounds__(kTB) void scalar_eval_fp32_kernel(const TraceArgs<float> A)
{
    const int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x;
    if (t >= A.n) return;
    int M = (int)(A.owned[t] >> 36);
    double Y[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) Y[i] = A.X[(int64_t)i * A.xstride + t];
    uint32_t mbase = (uint32_t)M * (uint32_t)A.npm;
    Stencil<DIM, float, ORD> st;
    unsigned flags = 0;
    locate32<DIM, BLEND, ORD>(A, M, mbase, Y, st, flags);
    A.c_hat[t] = gather_scalar<DIM, float, float>(A, mbase, st);
}

// 32-bit hash of particle i under a step's seed: the murmur3 finaliser
// (Appleby, MurmurHash3 fmix32) of i spread by the golden-ratio constant and
// xored with the seed
__device__ __forceinline__ uint32_t hash32(uint32_t seed, uint32_t i)
{
    uint32_t x = (i * 0x9E3779B1u) ^ seed;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

constexpr int kListBlock = 1024;
constexpr int kSelRounds = 16;  // most particles per thread of the selection

// Particle i is checked when its 32-bit hash is below thresh = fraction 2^32
// (every particle for fraction 1); a tile (one or two waves, `tile`
// particles) with no such particle checks its particle of smallest hash
// (compared in the upper 25 bits; ties: lowest index).  Appends the selected
// particles to the list, up to `cap` entries, and marks them in `checked`
// (1: in the list, 2: beyond the capacity).  A block takes `rounds` (at
// most kSelRounds) rounds of kListBlock consecutive particles and reserves
// its list entries with one atomic: an atomic per 1024 particles on the one
// list length serialises (16,600 of them at 1.7e7 particles took 0.6 ms),
// while small launches keep one round per block so that enough blocks run.
// The list's order is that of the reservations; only the set matters.
__global__ __launch_bounds__(kListBlock) void select_check_kernel(int64_t n, int tile, int rounds, uint32_t seed,
                                                                  uint32_t thresh, int32_t* ids,
                                                                  unsigned long long* n_ids, unsigned long long cap,
                                                                  unsigned char* checked)
{
    constexpr int NW = kListBlock / 64;
    __shared__ uint32_t skey[NW];
    __shared__ int sany[NW];
    __shared__ unsigned cnt[kSelRounds * NW];  // per (round, wave): count, then its offset in the block's share
    __shared__ unsigned long long base;
    static_assert(kSelRounds * NW % 64 == 0, "offsets: whole lanes");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wpt = tile / 64, w0 = wave - wave % wpt;
    const int64_t first = (int64_t)blockIdx.x * kListBlock * rounds + threadIdx.x;
    uint32_t picks = 0;  // bit q: the particle of round q is selected
    for (int q = 0; q < rounds; ++q) {
        const int64_t i = first + (int64_t)q * kListBlock;
        const bool in = i < n;
        const uint32_t h = hash32(seed, (uint32_t)i);
        bool c = in && (h < thresh || thresh == 0xFFFFFFFFu);
        // the tile's smallest hash, made unique by the particle's place in
        // its tile (tiles are 64 or 128 particles: 7 bits)
        uint32_t key = in ? ((h & ~127u) | (uint32_t)(i % tile)) : ~0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) key = min(key, (uint32_t)__shfl_xor((int)key, off, 64));
        const bool wany = __ballot(c) != 0;
        if (lane == 0) {
            skey[wave] = key;
            sany[wave] = wany;
        }
        __syncthreads();
        bool any = false;
        uint32_t best = ~0u;
        for (int w = w0; w < w0 + wpt; ++w) {
            any |= sany[w] != 0;
            best = min(best, skey[w]);
        }
        if (!any && in && (uint32_t)(i % tile) == (best & 127u)) c = true;
        picks |= (uint32_t)c << q;
        const unsigned long long m = __ballot(c);
        if (lane == 0) cnt[q * NW + wave] = (unsigned)__popcll(m);
        __syncthreads();  // skey / sany are rewritten by the next round
    }
    // unused rounds count zero; every count is written before wave 0 reads
    // them all
    for (int e = rounds * NW + (int)threadIdx.x; e < kSelRounds * NW; e += kListBlock) cnt[e] = 0;
    __syncthreads();
    // exclusive offsets over (round, wave) in order, by wave 0; one atomic
    if (wave == 0) {
        constexpr int PER = kSelRounds * NW / 64;
        unsigned v[PER], sum = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            v[j] = cnt[lane * PER + j];
            sum += v[j];
        }
        unsigned incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned o = (unsigned)__shfl_up((int)incl, off, 64);
            if (lane >= off) incl += o;
        }
        unsigned run = incl - sum;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            cnt[lane * PER + j] = run;
            run += v[j];
        }
        const unsigned tot = (unsigned)__shfl((int)incl, 63, 64);
        if (lane == 0) base = tot ? atomicAdd(n_ids, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    const unsigned long long below_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int q = 0; q < rounds; ++q) {
        const int64_t i = first + (int64_t)q * kListBlock;
        const bool c = (picks >> q) & 1u;
        const unsigned long long m = __ballot(c);
        const unsigned long long pos = base + cnt[q * NW + wave] + (unsigned long long)__popcll(m & below_mask);
        // a selected particle beyond the list's capacity is marked 2
        // (selected, not traced): the finish pass sends its tile to the
        // fallback
        if (i < n) checked[i] = c ? (pos < cap ? 1 : 2) : 0;
        if (c && pos < cap) ids[pos] = (int32_t)i;
    }
}

// grid of a remapped launch (a whole number of XCD rounds: blocks beyond the
// particle range have no active lane) and the run length it uses
inline unsigned grid_xcd(int64_t n, int lg)
{
    const int64_t round = 8 * (lg < 0 ? 1 : (int64_t)1 << lg);
    int64_t b = (n + kTB - 1) / kTB;
    b = (b + round - 1) / round * round;
    return (unsigned)b;
}

inline int xcd_log2_fp64(int64_t n)
{
    return (n + kTB - 1) / kTB >= MMOC_XCD_LARGE_BLOCKS ? MMOC_XCD_LOG2_FP64_LARGE : -1;
}

}  // namespace

template <typename T, bool G, int ORD>
hipError_t launch_trace_f64g(int dim, int blend, const TraceArgs<T>& a0, hipStream_t s)
{
    TraceArgs<T> a = a0;
    a.xcd_log2 = xcd_log2_fp64(a.n);
    const dim3 grid(grid_xcd(a.n, a.xcd_log2)), block(kTB);
    const bool st = a.nlev == 1;
    if constexpr (ORD == 2 && !G) {
        // the element cache: one stationary level, or two float32 levels or
        // two float64 levels in paired u_z records, within one interval of
        // the ring
        if constexpr (sizeof(T) == 8) {
            if (a.elem_cache && dim == 3 && !st && a.zs == 2 && a.n_int == 1) {
                if (blend) trace_fp64_kernel<3, 2, 1, T, false, 2, true, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
                else trace_fp64_kernel<3, 2, 0, T, false, 2, true, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
                return hipGetLastError();
            }
        }
        if (a.elem_cache && dim == 3 && (st || (sizeof(T) == 4 && a.n_int == 1))) {
            if (st) {
                if (blend) trace_fp64_kernel<3, 1, 1, T, false, 2, false, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
                else trace_fp64_kernel<3, 1, 0, T, false, 2, false, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
            } else if constexpr (sizeof(T) == 4) {
                if (blend) trace_fp64_kernel<3, 2, 1, T, false, 2, false, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
                else trace_fp64_kernel<3, 2, 0, T, false, 2, false, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
            }
            return hipGetLastError();
        }
    }
    if constexpr (sizeof(T) == 8) {
        // paired u_z records of a two-level ring (both levels in one load)
        if (a.zs == 2 && dim == 3 && !st) {
            if (!blend) trace_fp64_kernel<3, 2, 0, T, G, ORD, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
            else if (ORD == 2) trace_fp64_kernel<3, 2, 1, T, G, 2, true><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
            else return hipErrorNotSupported;
            return hipGetLastError();
        }
    }
    if (dim == 2 && !blend) {
        if (st) trace_fp64_kernel<2, 1, 0, T, G, ORD><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
        else trace_fp64_kernel<2, 2, 0, T, G, ORD><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
    } else if (dim == 3 && !blend) {
        if (st) trace_fp64_kernel<3, 1, 0, T, G, ORD><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
        else trace_fp64_kernel<3, 2, 0, T, G, ORD><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
    } else if (dim == 3 && blend && ORD == 2) {
        if (st) trace_fp64_kernel<3, 1, 1, T, G, 2><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
        else trace_fp64_kernel<3, 2, 1, T, G, 2><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
    } else if (dim == 2 && blend && ORD == 2) {
        if (st) trace_fp64_kernel<2, 1, 1, T, G, 2><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
        else trace_fp64_kernel<2, 2, 1, T, G, 2><<<grid, block, 0, s>>>(a, a.geo, a.c_hat, a.X, a.stats);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trace_f64(int dim, int blend, const TraceArgs<T>& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    if (a.ord == 1)
        return a.rk.s > 0 ? launch_trace_f64g<T, true, 1>(dim, blend, a, s)
                          : launch_trace_f64g<T, false, 1>(dim, blend, a, s);
    return a.rk.s > 0 ? launch_trace_f64g<T, true, 2>(dim, blend, a, s)
                      : launch_trace_f64g<T, false, 2>(dim, blend, a, s);
}

hipError_t launch_trace_fp64(int dim, int blend, const TraceArgs<double>& a, hipStream_t s)
{
    return launch_trace_f64(dim, blend, a, s);
}

hipError_t launch_trace_fp32_fields(int dim, int blend, const TraceArgs<float>& a, hipStream_t s)
{
    return launch_trace_f64(dim, blend, a, s);
}

template <typename T, typename K2, typename K3, typename K3b>
hipError_t launch_plain(int dim, int blend, const T& a, hipStream_t s, K2 k2, K3 k3, K2 k2b, K3b k3b)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + kTB - 1) / kTB)), block(kTB);
    if (dim == 2 && !blend) k2<<<grid, block, 0, s>>>(a);
    else if (dim == 3 && !blend) k3<<<grid, block, 0, s>>>(a);
    else if (dim == 2 && blend && k2b) k2b<<<grid, block, 0, s>>>(a);
    else if (dim == 3 && blend && k3b) k3b<<<grid, block, 0, s>>>(a);
    else return hipErrorNotSupported;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scalar_eval_f64(int dim, int blend, const TraceArgs<T>& a, hipStream_t s)
{
    if (a.ord == 1)
        return launch_plain(dim, blend, a, s, scalar_eval_fp64_kernel<2, 0, T, 1>, scalar_eval_fp64_kernel<3, 0, T, 1>,
                            (void (*)(TraceArgs<T>)) nullptr, (void (*)(TraceArgs<T>)) nullptr);
    return launch_plain(dim, blend, a, s, scalar_eval_fp64_kernel<2, 0, T, 2>, scalar_eval_fp64_kernel<3, 0, T, 2>,
                        scalar_eval_fp64_kernel<2, 1, T, 2>, scalar_eval_fp64_kernel<3, 1, T, 2>);
}

hipError_t launch_scalar_eval_fp64(int dim, int blend, const TraceArgs<double>& a, hipStream_t s)
{
    return launch_scalar_eval_f64(dim, blend, a, s);
}

hipError_t launch_scalar_eval_fp32_fields(int dim, int blend, const TraceArgs<float>& a, hipStream_t s)
{
    return launch_scalar_eval_f64(dim, blend, a, s);
}

hipError_t launch_scalar_eval_fp32(int dim, int blend, const TraceArgs<float>& a, hipStream_t s)
{
    if (a.ord == 1)
        return launch_plain(dim, blend, a, s, scalar_eval_fp32_kernel<2, 0, 1>, scalar_eval_fp32_kernel<3, 0, 1>,
                            (void (*)(TraceArgs<float>)) nullptr, (void (*)(TraceArgs<float>)) nullptr);
    return launch_plain(dim, blend, a, s, scalar_eval_fp32_kernel<2, 0, 2>, scalar_eval_fp32_kernel<3, 0, 2>,
                        scalar_eval_fp32_kernel<2, 1, 2>, scalar_eval_fp32_kernel<3, 1, 2>);
}

namespace mlp {

hipError_t launch_select_check(int64_t n, int tile, uint64_t seed, float fraction, int32_t* ids,
                               unsigned long long* n_ids, int64_t cap, unsigned char* checked, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (tile % 64 != 0 || tile > 128 || kListBlock % tile != 0 || n > INT32_MAX) return hipErrorInvalidValue;
    // particle i is checked when hash < fraction 2^32
    const double th = (double)fraction * 4294967296.0;
    const uint32_t thresh = th >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)th;
    // one round per block up to 256 blocks' worth of particles, then more
    // rounds per block (at most kSelRounds) instead of more blocks
    const int rounds = (int)std::min<int64_t>(kSelRounds, std::max<int64_t>(1, n / ((int64_t)kListBlock * 256)));
    const int64_t per_block = (int64_t)kListBlock * rounds;
    select_check_kernel<<<(unsigned)((n + per_block - 1) / per_block), kListBlock, 0, s>>>(
        n, tile, rounds, (uint32_t)(seed ^ (seed >> 32)), thresh, ids, n_ids, (unsigned long long)cap, checked);
    return hipGetLastError();
}

}  // namespace mlp

template <int ORD>
hipError_t launch_trace_fp32o(int dim, int blend, const TraceArgs<float>& a0, hipStream_t s)
{
    TraceArgs<float> a = a0;
    a.xcd_log2 = MMOC_XCD_LOG2_FP32;
    const dim3 grid(grid_xcd(a.n, a.xcd_log2)), block(kTB);
    const bool st = a.nlev == 1;
    if constexpr (ORD == 2) {
        if (a.elem_cache && dim == 3 && (st || a.n_int == 1)) {
            if (st) {
                if (blend) trace_fp32_kernel<3, 1, 1, 2, true><<<grid, block, 0, s>>>(a);
                else trace_fp32_kernel<3, 1, 0, 2, true><<<grid, block, 0, s>>>(a);
            } else {
                if (blend) trace_fp32_kernel<3, 2, 1, 2, true><<<grid, block, 0, s>>>(a);
                else trace_fp32_kernel<3, 2, 0, 2, true><<<grid, block, 0, s>>>(a);
            }
            return hipGetLastError();
        }
    }
    if (dim == 2 && !blend) {
        if (st) trace_fp32_kernel<2, 1, 0, ORD><<<grid, block, 0, s>>>(a);
        else trace_fp32_kernel<2, 2, 0, ORD><<<grid, block, 0, s>>>(a);
    } else if (dim == 3 && !blend) {
        if (st) trace_fp32_kernel<3, 1, 0, ORD><<<grid, block, 0, s>>>(a);
        else trace_fp32_kernel<3, 2, 0, ORD><<<grid, block, 0, s>>>(a);
    } else if (dim == 3 && blend && ORD == 2) {
        if (st) trace_fp32_kernel<3, 1, 1, 2><<<grid, block, 0, s>>>(a);
        else trace_fp32_kernel<3, 2, 1, 2><<<grid, block, 0, s>>>(a);
    } else if (dim == 2 && blend && ORD == 2) {
        if (st) trace_fp32_kernel<2, 1, 1, 2><<<grid, block, 0, s>>>(a);
        else trace_fp32_kernel<2, 2, 1, 2><<<grid, block, 0, s>>>(a);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t launch_trace_fp32(int dim, int blend, const TraceArgs<float>& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    return a.ord == 1 ? launch_trace_fp32o<1>(dim, blend, a, s) : launch_trace_fp32o<2>(dim, blend, a, s);
}

}  // namespace mmoc
