// mmoc_kernels.hip -- CDNA4 (gfx950) kernels of the MMOC particle tracer.
//
// One lane traces one particle through the whole step (Sec. 2.3.1 steps
// (i)-(iii)): it creates the particle at its P2 DoF, runs the S x 4 RK4
// stages (each a macro walk, an O(1) micro location and a P2 gather of both
// velocity levels, Sec. 2.3.2), accumulates the departure point in float64
// and evaluates the old scalar there.  Particles are independent, so there
// is no inter-lane communication except the per-wave ballots that count
// flagged particles into the statistics.
//
// Memory layout (all device resident):
//   geo   : MacroGeo[n_macros], 256 B each (L2 resident, at most ~1 MB)
//   owned : uint64[n] (macro, I, J, K) per particle, canonical DoF order
//   rec0  : T4[n_macros * npm]  (u_x, u_y, u_z, c) at t_n, macro-major
//           block layout, lattice nodes in lexicographic (I, J, K) order
//   rec1  : T4[n_macros * npm]  (u_x, u_y, u_z, -) at t_{n+1}
// The 4-wide records turn the gather of one node into one 16-byte (fp32)
// or 16+8-byte (fp64) load per level.
//
// Workgroups are remapped so that each of the 8 XCDs (own L2 each) receives
// one contiguous eighth of the particle range: neighbouring particles share
// stencils, and keeping them on one XCD keeps their nodes in one L2.
#include "mmoc_internal.h"

#include <math.h>

namespace mmoc {
namespace {

constexpr int kBlock = 256;

// position of lattice node (I, J, K), m >= I >= J >= K >= 0, in the
// lexicographic enumeration of the macro's lattice
template <int DIM>
__device__ __forceinline__ int lat_idx(int I, int J, int K)
{
    if constexpr (DIM == 2) {
        return ((I * (I + 1)) >> 1) + J;
    } else {
        return (I * (I + 1) * (I + 2)) / 6 + ((J * (J + 1)) >> 1) + K;
    }
}

// XCD-contiguous logical block index (grid padded to a multiple of 8)
__device__ __forceinline__ int64_t logical_block()
{
    const unsigned per = gridDim.x >> 3;
    return (int64_t)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
}

// ----------------------------------------------------------------- geometry

// Register copy of the current macro: origin, inverse map, shell plane.
template <int DIM, int BLEND>
struct Geo64 {
    double v0[DIM];
    double bi[DIM][DIM];
    double pn[3];
    double pc;

    __device__ __forceinline__ void load(const MacroGeo* __restrict__ g, int M)
    {
        const MacroGeo& G = g[M];
#pragma unroll
        for (int i = 0; i < DIM; ++i) v0[i] = G.v0[i];
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) bi[r][c] = G.binv[r * 3 + c];
        if constexpr (BLEND) {
            pn[0] = G.pn[0];
            pn[1] = G.pn[1];
            pn[2] = G.pn[2];
            pc = G.pc;
        }
    }

    // physical y -> reference coordinates s; returns lambda_0 = 1 - sum s
    __device__ __forceinline__ double ref(const double y[DIM], double s[DIM]) const
    {
        double p[DIM];
        if constexpr (BLEND) {
            // Phi^-1(z) = z c |z| / (n.z)
            const double nz = pn[0] * y[0] + pn[1] * y[1] + pn[2] * y[2];
            const double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
            const double f = pc * r / nz;
#pragma unroll
            for (int i = 0; i < DIM; ++i) p[i] = y[i] * f - v0[i];
        } else {
#pragma unroll
            for (int i = 0; i < DIM; ++i) p[i] = y[i] - v0[i];
        }
        double sum = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) acc = fma(bi[a][i], p[i], acc);
            s[a] = acc;
            sum += acc;
        }
        return 1.0 - sum;
    }
};

template <int DIM>
__device__ __forceinline__ double lam_min(double l0, const double s[DIM])
{
    double m = l0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) m = fmin(m, s[a]);
    return m;
}

// Macro walk from M (Sec. 2.3.2: search the neighbourhood of the macro that
// held the previous evaluation).  Accept when min lambda >= -eps; otherwise
// hop across the face with the most negative lambda among faces that have a
// neighbour (ties: lowest face).  No such face: the point is outside the
// domain and stays in M.  After max_hops hops: brute force (argmax over
// macros of min lambda, ties: lowest macro).
//
// The slow part is out of line and takes only scalars, so that the hot
// loop's registers never spill to the stack; it returns the macro in bits
// 0-26 and lane flags above.
template <int DIM, int BLEND>
__device__ __noinline__ unsigned walk_slow(const MacroGeo* __restrict__ geo, int nm, int max_hops, double eps,
                                           int M, double y0, double y1, double y2)
{
    const double y[3] = {y0, y1, y2};
    double s[DIM];
    unsigned flags = 0;
    Geo64<DIM, BLEND> G;
    G.load(geo, M);
    for (int hop = 0;; ++hop) {
        const double l0 = G.ref(y, s);
        if (lam_min<DIM>(l0, s) >= -eps) return (unsigned)M | (flags << 27);
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
        const double v = lam_min<DIM>(ll, s);
        if (v > bestv) {
            bestv = v;
            best = q;
        }
    }
    if (bestv < -eps) flags |= LF_OUTSIDE;
    return (unsigned)best | (flags << 27);
}

// On return G holds macro M and s, l0 are the reference coordinates of y in it.
template <int DIM, int BLEND>
__device__ __forceinline__ void walk(const TraceArgs<double>& A, int& M, Geo64<DIM, BLEND>& G,
                                     const double* y, double* s, double& l0, unsigned& flags)
{
    l0 = G.ref(y, s);
    if (lam_min<DIM>(l0, s) >= -A.eps_in) return;  // common case: still inside
    const unsigned r = walk_slow<DIM, BLEND>(A.geo, A.nm, A.max_hops, A.eps_in, M, y[0], y[1],
                                             DIM == 3 ? y[DIM - 1] : 0.0);
    const int M2 = (int)(r & ((1u << 27) - 1));
    flags |= r >> 27;
    if (M2 != M) {
        M = M2;
        G.load(A.geo, M);
    }
    l0 = G.ref(y, s);
}

// ------------------------------------------------------ micro element + P2

template <int DIM>
struct Stencil {
    static constexpr int NN = (DIM + 1) * (DIM + 2) / 2;
    int idx[NN];
    double phi[NN];
};

// O(1) micro location in the Freudenthal lattice of the macro's Kuhn
// coordinates w (w_d = s_d, w_a = s_a + w_{a+1}), then P2 shape functions at
// the (possibly unclamped) point.  A point outside the macro selects its
// element from the clamped, renormalised barycentrics and is evaluated by
// extrapolating that element.
template <int DIM>
__device__ __forceinline__ void micro(const double* s, double l0, int n, Stencil<DIM>& st)
{
    double ssel[DIM];
    if (lam_min<DIM>(l0, s) >= 0.0) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) ssel[a] = s[a];
    } else {
        double sum = fmax(l0, 0.0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) sum += fmax(s[a], 0.0);
        const double inv = 1.0 / sum;
#pragma unroll
        for (int a = 0; a < DIM; ++a) ssel[a] = fmax(s[a], 0.0) * inv;
    }
    const double dn = (double)n;
    double W[DIM], Wu[DIM];
    W[DIM - 1] = ssel[DIM - 1];
    Wu[DIM - 1] = s[DIM - 1];
#pragma unroll
    for (int a = DIM - 2; a >= 0; --a) {
        W[a] = ssel[a] + W[a + 1];
        Wu[a] = s[a] + Wu[a + 1];
    }
    int k[DIM];
    double f[DIM], fu[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        W[i] *= dn;
        Wu[i] *= dn;
        const double kc = floor(fmin(fmax(W[i], 0.0), dn - 1.0));
        k[i] = (int)kc;
        f[i] = W[i] - kc;
        fu[i] = Wu[i] - kc;
    }
    // rank of each axis in the descending order of f (ties: lower axis first)
    int r[DIM];
    double g[DIM];
    if constexpr (DIM == 3) {
        r[0] = (f[1] > f[0]) + (f[2] > f[0]);
        r[1] = (f[0] >= f[1]) + (f[2] > f[1]);
        r[2] = (f[0] >= f[2]) + (f[1] >= f[2]);
        g[0] = r[0] == 0 ? fu[0] : (r[1] == 0 ? fu[1] : fu[2]);
        g[1] = r[0] == 1 ? fu[0] : (r[1] == 1 ? fu[1] : fu[2]);
        g[2] = r[0] == 2 ? fu[0] : (r[1] == 2 ? fu[1] : fu[2]);
    } else {
        r[0] = f[1] > f[0];
        r[1] = f[0] >= f[1];
        g[0] = r[0] == 0 ? fu[0] : fu[1];
        g[1] = r[0] == 1 ? fu[0] : fu[1];
    }
    double mu[DIM + 1];
    mu[0] = 1.0 - g[0];
#pragma unroll
    for (int a = 1; a < DIM; ++a) mu[a] = g[a - 1] - g[a];
    mu[DIM] = g[DIM - 1];
    // micro vertex a in the n-lattice: V_a[i] = k_i + (r_i < a)
    int V[DIM + 1][3];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
#pragma unroll
        for (int i = 0; i < 3; ++i) V[a][i] = i < DIM ? k[i] + (r[i] < a ? 1 : 0) : 0;
    }
    int c = 0;
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        st.idx[c] = lat_idx<DIM>(2 * V[a][0], 2 * V[a][1], 2 * V[a][2]);
        st.phi[c] = mu[a] * fma(2.0, mu[a], -1.0);
        ++c;
    }
#pragma unroll
    for (int a = 0; a <= DIM; ++a)
#pragma unroll
        for (int b = a + 1; b <= DIM; ++b) {
            st.idx[c] = lat_idx<DIM>(V[a][0] + V[b][0], V[a][1] + V[b][1], V[a][2] + V[b][2]);
            st.phi[c] = 4.0 * mu[a] * mu[b];
            ++c;
        }
}

// Velocity at the stage point: P2 sums of both levels, linear in time.
template <int DIM, int NLEV>
__device__ __forceinline__ void gather_vel(const TraceArgs<double>& A, int M, const Stencil<DIM>& st,
                                           double theta, double* k)
{
    constexpr int NN = Stencil<DIM>::NN;
    const size_t base = (size_t)M * (size_t)A.npm;
    double ua[DIM], ub[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        ua[i] = 0.0;
        ub[i] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < NN; ++q) {
        const double* r0 = A.rec0 + (base + (size_t)st.idx[q]) * 4;
        const double2 a01 = *reinterpret_cast<const double2*>(r0);
        ua[0] = fma(st.phi[q], a01.x, ua[0]);
        ua[1] = fma(st.phi[q], a01.y, ua[1]);
        if constexpr (DIM == 3) ua[2] = fma(st.phi[q], r0[2], ua[2]);
        if constexpr (NLEV == 2) {
            const double* r1 = A.rec1 + (base + (size_t)st.idx[q]) * 4;
            const double2 b01 = *reinterpret_cast<const double2*>(r1);
            ub[0] = fma(st.phi[q], b01.x, ub[0]);
            ub[1] = fma(st.phi[q], b01.y, ub[1]);
            if constexpr (DIM == 3) ub[2] = fma(st.phi[q], r1[2], ub[2]);
        }
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        if constexpr (NLEV == 2) {
            k[i] = (1.0 - theta) * ua[i] + theta * ub[i];
        } else {
            k[i] = ua[i];
        }
    }
}

template <int DIM>
__device__ __forceinline__ double gather_scalar(const TraceArgs<double>& A, int M, const Stencil<DIM>& st)
{
    constexpr int NN = Stencil<DIM>::NN;
    const size_t base = (size_t)M * (size_t)A.npm;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NN; ++q) acc = fma(st.phi[q], A.rec0[(base + (size_t)st.idx[q]) * 4 + 3], acc);
    return acc;
}

// Particle creation (step (i)): physical position of lattice node (I, J, K)
// of macro M, x = Phi(v0 + B s), s = (I - J, J - K, K) / m.
template <int DIM, int BLEND>
__device__ __forceinline__ void dof_position(const MacroGeo* __restrict__ geo, uint64_t e, int level_n,
                                             int& M, double* x)
{
    M = (int)(e >> 36);
    const int I = (int)((e >> 24) & 0xfffu), J = (int)((e >> 12) & 0xfffu), K = (int)(e & 0xfffu);
    const double invm = 1.0 / (double)(2 * level_n);  // exact: m is a power of two
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
        const double nx = G.pn[0] * p[0] + G.pn[1] * p[1] + G.pn[2] * p[2];
        const double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        const double f = nx / (G.pc * r);
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[i] = p[i] * f;
    } else {
#pragma unroll
        for (int i = 0; i < DIM; ++i) x[i] = p[i];
    }
}

// Adds this wave's flagged-particle counts to the statistics: one atomic per
// wave and counter.
__device__ __forceinline__ void count_flags(unsigned long long* stats, bool active, unsigned flags)
{
    const unsigned long long nact = __popcll(__ballot(active));
    const unsigned long long no = __popcll(__ballot((flags & LF_OUTSIDE) != 0));
    const unsigned long long nm = __popcll(__ballot((flags & LF_MULTIHOP) != 0));
    const unsigned long long nb = __popcll(__ballot((flags & LF_BRUTE) != 0));
    const unsigned long long nt = __popcll(__ballot((flags & LF_TIEBAND) != 0));
    const unsigned long long nn = __popcll(__ballot((flags & LF_NAN) != 0));
    if ((threadIdx.x & 63) == 0) {
        if (nact) atomicAdd(stats + ST_PARTICLES, nact);
        if (no) atomicAdd(stats + ST_OUTSIDE, no);
        if (nm) atomicAdd(stats + ST_MULTIHOP, nm);
        if (nb) atomicAdd(stats + ST_BRUTE, nb);
        if (nt) atomicAdd(stats + ST_TIEBAND, nt);
        if (nn) atomicAdd(stats + ST_NAN, nn);
    }
}

// ------------------------------------------------------------- trace fp64

template <int DIM, int NLEV, int BLEND>
__global__ __launch_bounds__(kBlock) void trace_fp64_kernel(const TraceArgs<double> A)
{
    const int64_t t = logical_block() * kBlock + threadIdx.x;
    const bool active = t < A.n;
    unsigned flags = 0;
    if (active) {
        const int64_t pid = A.ids ? (int64_t)A.ids[t] : t;
        int M;
        double Y[DIM];
        dof_position<DIM, BLEND>(A.geo, A.owned[pid], A.level_n, M, Y);
        Geo64<DIM, BLEND> G;
        G.load(A.geo, M);
        const double h = A.dt / (double)A.substeps;
        const double hh = 0.5 * h;
        const double h6 = h / 6.0;
        double s[DIM], l0;
        Stencil<DIM> st;
#pragma unroll 1
        for (int j = 0; j < A.substeps; ++j) {
            double ks[DIM], acc[DIM], y[DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) y[i] = Y[i];
#pragma unroll 1
            for (int stg = 0; stg < 4; ++stg) {
                // stage time: theta = 1 - (j + a_s)/S, a_s = 0, 1/2, 1/2, 1
                const double as = stg == 0 ? 0.0 : (stg == 3 ? 1.0 : 0.5);
                const double theta = 1.0 - ((double)j + as) / (double)A.substeps;
                walk<DIM, BLEND>(A, M, G, y, s, l0, flags);
                micro<DIM>(s, l0, A.level_n, st);
                gather_vel<DIM, NLEV>(A, M, st, theta, ks);
                // k1 + 2 k2 + 2 k3 + k4, accumulated in stage order
                const double w = (stg == 0 || stg == 3) ? 1.0 : 2.0;
                const double cnext = stg == 2 ? h : hh;
#pragma unroll
                for (int i = 0; i < DIM; ++i) {
                    acc[i] = stg == 0 ? ks[i] : fma(w, ks[i], acc[i]);
                    y[i] = Y[i] - cnext * ks[i];
                }
            }
#pragma unroll
            for (int i = 0; i < DIM; ++i) Y[i] = Y[i] - h6 * acc[i];
        }
        // step (iii): scalar at the departure point
        walk<DIM, BLEND>(A, M, G, Y, s, l0, flags);
        micro<DIM>(s, l0, A.level_n, st);
        const double v = gather_scalar<DIM>(A, M, st);
        bool bad = v != v;
#pragma unroll
        for (int i = 0; i < DIM; ++i) bad |= Y[i] != Y[i];
        if (bad) flags |= LF_NAN;
        if (A.c_hat) A.c_hat[pid] = v;
        if (A.X) {
#pragma unroll
            for (int i = 0; i < DIM; ++i) A.X[(int64_t)i * A.xstride + pid] = Y[i];
        }
    }
    count_flags(A.stats, active, flags);
}

template <int DIM, int BLEND>
__global__ __launch_bounds__(kBlock) void dof_coords_kernel(const MacroGeo* __restrict__ geo,
                                                            const uint64_t* __restrict__ owned, int64_t n,
                                                            int level_n, double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    int M;
    double x[DIM];
    dof_position<DIM, BLEND>(geo, owned[t], level_n, M, x);
#pragma unroll
    for (int i = 0; i < DIM; ++i) out[(int64_t)i * n + t] = x[i];
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void scatter_vec_kernel(const int32_t* __restrict__ slot_uid, int64_t nslots,
                                                             const double* __restrict__ u, int64_t nu,
                                                             T* __restrict__ rec)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nslots) return;
    const int64_t q = slot_uid[t];
#pragma unroll
    for (int i = 0; i < DIM; ++i) rec[t * 4 + i] = (T)u[(int64_t)i * nu + q];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scatter_scalar_kernel(const int32_t* __restrict__ slot_uid,
                                                                int64_t nslots, const double* __restrict__ c,
                                                                T* __restrict__ rec)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nslots) return;
    rec[t * 4 + 3] = (T)c[slot_uid[t]];
}

inline unsigned grid_xcd(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    b = (b + 7) / 8 * 8;
    return (unsigned)b;
}

inline unsigned grid_plain(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_trace_fp64(int dim, int blend, const TraceArgs<double>& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 grid(grid_xcd(a.n)), block(kBlock);
    const int stat = a.nlev == 1;
    if (dim == 2 && !blend) {
        if (stat) trace_fp64_kernel<2, 1, 0><<<grid, block, 0, s>>>(a);
        else trace_fp64_kernel<2, 2, 0><<<grid, block, 0, s>>>(a);
    } else if (dim == 3 && !blend) {
        if (stat) trace_fp64_kernel<3, 1, 0><<<grid, block, 0, s>>>(a);
        else trace_fp64_kernel<3, 2, 0><<<grid, block, 0, s>>>(a);
    } else if (dim == 3 && blend) {
        if (stat) trace_fp64_kernel<3, 1, 1><<<grid, block, 0, s>>>(a);
        else trace_fp64_kernel<3, 2, 1><<<grid, block, 0, s>>>(a);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t launch_dof_coords(int dim, int blend, const MacroGeo* geo, const uint64_t* owned, int64_t n,
                             int level_n, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid(grid_plain(n)), block(kBlock);
    if (dim == 2) dof_coords_kernel<2, 0><<<grid, block, 0, s>>>(geo, owned, n, level_n, out);
    else if (!blend) dof_coords_kernel<3, 0><<<grid, block, 0, s>>>(geo, owned, n, level_n, out);
    else dof_coords_kernel<3, 1><<<grid, block, 0, s>>>(geo, owned, n, level_n, out);
    return hipGetLastError();
}

hipError_t launch_scatter_vec(int dim, const int32_t* slot_uid, int64_t nslots, const double* u, int64_t n_unique,
                              void* rec, int fp32, hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    const dim3 grid(grid_plain(nslots)), block(kBlock);
    if (fp32) {
        if (dim == 2) scatter_vec_kernel<2, float><<<grid, block, 0, s>>>(slot_uid, nslots, u, n_unique, (float*)rec);
        else scatter_vec_kernel<3, float><<<grid, block, 0, s>>>(slot_uid, nslots, u, n_unique, (float*)rec);
    } else {
        if (dim == 2) scatter_vec_kernel<2, double><<<grid, block, 0, s>>>(slot_uid, nslots, u, n_unique, (double*)rec);
        else scatter_vec_kernel<3, double><<<grid, block, 0, s>>>(slot_uid, nslots, u, n_unique, (double*)rec);
    }
    return hipGetLastError();
}

hipError_t launch_scatter_scalar(const int32_t* slot_uid, int64_t nslots, const double* c, void* rec, int fp32,
                                 hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    const dim3 grid(grid_plain(nslots)), block(kBlock);
    if (fp32) scatter_scalar_kernel<float><<<grid, block, 0, s>>>(slot_uid, nslots, c, (float*)rec);
    else scatter_scalar_kernel<double><<<grid, block, 0, s>>>(slot_uid, nslots, c, (double*)rec);
    return hipGetLastError();
}

hipError_t launch_trace_fp32(int, int, const TraceArgs<float>&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace mmoc
