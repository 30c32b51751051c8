// mmoc_fe.hip -- finite-element operators on the refined mesh and the
// conjugate-gradient solve of the diffusion step (Sec. 2.2, eq.
// linear-system).
//
// Assembly: one thread per (micro element, local row) integrates its row of
// the element mass and stiffness matrices by quadrature through the
// element map x(xi) = Phi(p_0 + sum_a xi_a (p_a - p_0)); a second kernel sums
// the element entries of every CSR slot in a fixed order (no atomics, so the
// matrices are bitwise reproducible).
//
// Solve: conjugate gradients on the CSR matrix, float64.  The dot products
// reduce through per-block partials that the last block to finish sums in a
// fixed order (a ticket counter); the step scalars stay on the device, and
// each kernel returns at once when the solve has converged, so that the host
// can enqueue batches of iterations and read the state back once per batch.
#include "mmoc_fe_internal.h"

#include <math.h>

namespace mmoc {
namespace fe {
namespace {

constexpr int kB = 256;
constexpr int kWaves = kB / 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// coherent (L2) read of a value another block wrote in this launch
__device__ __forceinline__ double load_l2(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sums NV values over the block, publishes the block's sums as partials and
// takes a ticket.  Returns true in the last block to finish, whose thread 0
// then holds in tot[] the totals over all blocks, summed in block order.
template <int NV>
__device__ bool reduce_last(double (&v)[NV], double* part, unsigned* ticket, double (&tot)[NV])
{
    __shared__ double sh[NV][kWaves];
    __shared__ bool last;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double w = wave_sum(v[k]);
        if (lane == 0) sh[k][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = sh[k][0];
#pragma unroll
            for (int q = 1; q < kWaves; ++q) s += sh[k][q];
            part[k * kRedBlocks + blockIdx.x] = s;
        }
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        acc[k] = 0.0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += kB) acc[k] += load_l2(part + k * kRedBlocks + b);
    }
    __syncthreads();  // sh is reused
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double w = wave_sum(acc[k]);
        if (lane == 0) sh[k][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = sh[k][0];
#pragma unroll
            for (int q = 1; q < kWaves; ++q) s += sh[k][q];
            tot[k] = s;
        }
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

// ------------------------------------------------------------- assembly

// Lagrange shape functions on the reference simplex and their reference
// gradients: lambda_0 = 1 - sum xi, lambda_a = xi_a.  P1: lambda_a.  P2:
// lambda_a (2 lambda_a - 1) at the vertices a = 0..d, then 4 lambda_a lambda_b
// at the edge midpoints, edges (a, b), a < b, in lexicographic order.
template <int DIM, int ORD>
__device__ __forceinline__ void shapes(const double* xi, double* phi, double (*gr)[DIM])
{
    double lam[DIM + 1];
    lam[0] = 1.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lam[0] -= xi[a];
        lam[a + 1] = xi[a];
    }
    // d lambda_a / d xi_k: -1 for a = 0, delta_{a-1,k} otherwise
    auto dl = [](int a, int k) { return a == 0 ? -1.0 : (a - 1 == k ? 1.0 : 0.0); };
    int c = 0;
    if constexpr (ORD == 1) {
#pragma unroll
        for (int a = 0; a <= DIM; ++a, ++c) {
            phi[c] = lam[a];
#pragma unroll
            for (int k = 0; k < DIM; ++k) gr[c][k] = dl(a, k);
        }
    } else {
#pragma unroll
        for (int a = 0; a <= DIM; ++a, ++c) {
            phi[c] = lam[a] * (2.0 * lam[a] - 1.0);
#pragma unroll
            for (int k = 0; k < DIM; ++k) gr[c][k] = (4.0 * lam[a] - 1.0) * dl(a, k);
        }
#pragma unroll
        for (int a = 0; a <= DIM; ++a)
#pragma unroll
            for (int b = a + 1; b <= DIM; ++b, ++c) {
                phi[c] = 4.0 * lam[a] * lam[b];
#pragma unroll
                for (int k = 0; k < DIM; ++k) gr[c][k] = 4.0 * (lam[b] * dl(a, k) + lam[a] * dl(b, k));
            }
    }
}

template <int DIM>
__device__ __forceinline__ double det_inverse(const double (&J)[DIM][DIM], double (&Ji)[DIM][DIM])
{
    if constexpr (DIM == 2) {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double r = 1.0 / det;
        Ji[0][0] = J[1][1] * r;
        Ji[0][1] = -J[0][1] * r;
        Ji[1][0] = -J[1][0] * r;
        Ji[1][1] = J[0][0] * r;
        return det;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double r = 1.0 / det;
        Ji[0][0] = c00 * r;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
        Ji[1][0] = c01 * r;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
        Ji[2][0] = c02 * r;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
        return det;
    }
}

template <int DIM, int ORD, int BLEND>
__global__ __launch_bounds__(kB) void element_matrices_kernel(const MacroGeo* __restrict__ geo,
                                                              const Elem* __restrict__ el, int64_t nel, int n,
                                                              const QRule* __restrict__ rule, double* __restrict__ me,
                                                              double* __restrict__ ae)
{
    constexpr int NB = ORD == 2 ? (DIM + 1) * (DIM + 2) / 2 : DIM + 1;
    const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (t >= nel * NB) return;
    const int64_t e = t / NB;
    const int row = (int)(t - e * NB);
    const Elem E = el[e];
    const MacroGeo& G = geo[E.macro];
    const double inv_n = 1.0 / (double)n;  // exact: n is a power of two
    // computational vertex positions v0 + B s, s = (I - J, J - K, K) / n
    double p[DIM + 1][DIM];
#pragma unroll
    for (int a = 0; a <= DIM; ++a) {
        double s[DIM];
        s[0] = (double)(E.v[a][0] - E.v[a][1]) * inv_n;
        if constexpr (DIM == 2) {
            s[1] = (double)E.v[a][1] * inv_n;
        } else {
            s[1] = (double)(E.v[a][1] - E.v[a][2]) * inv_n;
            s[2] = (double)E.v[a][2] * inv_n;
        }
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            double acc = G.v0[i];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc = fma(G.B[i * 3 + k], s[k], acc);
            p[a][i] = acc;
        }
    }
    double Ed[DIM][DIM];  // columns p_{a+1} - p_0
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int a = 0; a < DIM; ++a) Ed[i][a] = p[a + 1][i] - p[0][i];
    double pn[DIM], pc = 1.0;
    if constexpr (BLEND) {
#pragma unroll
        for (int i = 0; i < DIM; ++i) pn[i] = G.pn[i];
        pc = G.pc;
    }
    double mrow[NB], arow[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) mrow[j] = arow[j] = 0.0;

    const int nq = rule->nq;
    for (int q = 0; q < nq; ++q) {
        double xi[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) xi[a] = rule->pt[q][a];
        double J[DIM][DIM];
        if constexpr (BLEND) {
            // Phi(x) = f x, f = (n.x)/(c|x|): DPhi = f I + x grad f^T,
            // grad f = n/(c|x|) - (n.x) x/(c|x|^3)
            double x[DIM], nx = 0.0, r2 = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                double acc = p[0][i];
#pragma unroll
                for (int a = 0; a < DIM; ++a) acc = fma(Ed[i][a], xi[a], acc);
                x[i] = acc;
                nx = fma(pn[i], x[i], nx);
                r2 = fma(x[i], x[i], r2);
            }
            const double r = sqrt(r2), cr = pc * r;
            const double f = nx / cr;
            double gf[DIM], D[DIM][DIM];
#pragma unroll
            for (int i = 0; i < DIM; ++i) gf[i] = pn[i] / cr - nx * x[i] / (cr * r2);
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int k = 0; k < DIM; ++k) D[i][k] = x[i] * gf[k] + (i == k ? f : 0.0);
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < DIM; ++k) acc = fma(D[i][k], Ed[k][a], acc);
                    J[i][a] = acc;
                }
        } else {
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int a = 0; a < DIM; ++a) J[i][a] = Ed[i][a];
        }
        double Ji[DIM][DIM];
        const double wdet = rule->w[q] * fabs(det_inverse<DIM>(J, Ji));
        double phi[NB], gr[NB][DIM];
        shapes<DIM, ORD>(xi, phi, gr);
        // physical gradients: J^-T times the reference gradients
        double gp[NB][DIM];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; ++k) acc = fma(Ji[k][i], gr[b][k], acc);
                gp[b][i] = acc;
            }
        double phr = 0.0, gpr[DIM];
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (b == row) {
                phr = phi[b];
#pragma unroll
                for (int i = 0; i < DIM; ++i) gpr[i] = gp[b][i];
            }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double dot = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; ++i) dot = fma(gpr[i], gp[j][i], dot);
            mrow[j] = fma(wdet * phr, phi[j], mrow[j]);
            arow[j] = fma(wdet, dot, arow[j]);
        }
    }
    const int64_t o = e * NB * NB + (int64_t)row * NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        me[o + j] = mrow[j];
        ae[o + j] = arow[j];
    }
}

__global__ __launch_bounds__(kB) void gather_kernel(int64_t nnz, const int64_t* __restrict__ cptr,
                                                    const int32_t* __restrict__ contrib, const double* __restrict__ me,
                                                    const double* __restrict__ ae, double* __restrict__ mv,
                                                    double* __restrict__ av)
{
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k >= nnz) return;
    double sm = 0.0, sa = 0.0;
    for (int64_t j = cptr[k]; j < cptr[k + 1]; ++j) {
        const int32_t c = contrib[j];
        sm += me[c];
        sa += ae[c];
    }
    mv[k] = sm;
    av[k] = sa;
}

// ------------------------------------------------------------ operators

__global__ __launch_bounds__(kB) void build_e_kernel(int64_t N, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ mv,
                                                     const double* __restrict__ av, double s1,
                                                     const uint8_t* __restrict__ is_dir, int precond,
                                                     double* __restrict__ ev, double* __restrict__ dinv)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= N) return;
    const bool di = is_dir && is_dir[i];
    double diag = 1.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = ci[k];
        double v;
        if (di || (is_dir && is_dir[j])) v = (j == i) ? 1.0 : 0.0;
        else v = fma(s1, av[k], mv[k]);
        ev[k] = v;
        if (j == i) diag = v;
    }
    dinv[i] = precond ? 1.0 / diag : 1.0;
}

__global__ __launch_bounds__(kB) void spmv_kernel(int64_t N, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                  const double* __restrict__ x, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc = fma(v[k], x[ci[k]], acc);
    y[i] = acc;
}

__global__ __launch_bounds__(kB) void rhs_kernel(RhsArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= a.N) return;
    if (a.is_dir && a.is_dir[i]) {
        a.b[i] = a.g[i];
        a.x[i] = a.g[i];
        return;
    }
    double acc = 0.0;
    for (int32_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
        const int32_t j = a.ci[k];
        const double m = a.mv[k], s = a.av[k];
        acc = fma(fma(-a.s2, s, m), a.chat[j], acc);
        if (a.is_dir && a.is_dir[j]) acc = fma(-fma(a.s1, s, m), a.g[j], acc);
    }
    if (a.q0) acc = fma(a.w0, a.q0[i], acc);
    if (a.q1) acc = fma(a.w1, a.q1[i], acc);
    a.b[i] = acc;
    a.x[i] = a.chat[i];
}

// ------------------------------------------------------------------- CG

__device__ __forceinline__ double row_dot(const CgArgs& a, int64_t i, const double* x)
{
    double acc = 0.0;
    for (int32_t k = a.rp[i]; k < a.rp[i + 1]; ++k) acc = fma(a.ev[k], x[a.ci[k]], acc);
    return acc;
}

__global__ __launch_bounds__(kB) void cg_init_kernel(CgArgs a)
{
    double v[3] = {0.0, 0.0, 0.0};  // r.z, r.r, b.b
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.N; i += (int64_t)gridDim.x * kB) {
        const double bi = a.b[i];
        const double r = bi - row_dot(a, i, a.x);
        const double z = a.dinv[i] * r;
        a.r[i] = r;
        a.p[i] = z;
        v[0] = fma(r, z, v[0]);
        v[1] = fma(r, r, v[1]);
        v[2] = fma(bi, bi, v[2]);
    }
    double tot[3];
    if (reduce_last<3>(v, a.part, a.ticket, tot) && threadIdx.x == 0) {
        CgScalars* s = a.sc;
        s->rz = tot[0];
        s->rr = tot[1];
        s->bb = tot[2];
        s->thresh = a.rtol2 * (tot[2] > 0.0 ? tot[2] : tot[1]);
        s->iters = 0;
        s->alpha = s->beta = s->pq = 0.0;
        s->done = tot[1] <= s->thresh ? (tot[2] > 0.0 ? 1 : 3) : 0;
    }
}

// q = E p, p.q; alpha = r.z / p.q
__global__ __launch_bounds__(kB) void cg_spmv_kernel(CgArgs a)
{
    if (a.sc->done) return;
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.N; i += (int64_t)gridDim.x * kB) {
        const double q = row_dot(a, i, a.p);
        a.q[i] = q;
        v[0] = fma(a.p[i], q, v[0]);
    }
    double tot[1];
    if (reduce_last<1>(v, a.part, a.ticket, tot) && threadIdx.x == 0) {
        CgScalars* s = a.sc;
        s->pq = tot[0];
        if (!(tot[0] > 0.0)) s->done = 2;
        else s->alpha = s->rz / tot[0];
    }
}

// x += alpha p, r -= alpha q, r.z and r.r; beta = r.z_new / r.z
__global__ __launch_bounds__(kB) void cg_update_kernel(CgArgs a)
{
    if (a.sc->done) return;
    const double alpha = a.sc->alpha;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < a.N; i += (int64_t)gridDim.x * kB) {
        a.x[i] = fma(alpha, a.p[i], a.x[i]);
        const double r = fma(-alpha, a.q[i], a.r[i]);
        a.r[i] = r;
        v[0] = fma(r, a.dinv[i] * r, v[0]);
        v[1] = fma(r, r, v[1]);
    }
    double tot[2];
    if (reduce_last<2>(v, a.part, a.ticket, tot) && threadIdx.x == 0) {
        CgScalars* s = a.sc;
        s->beta = tot[0] / s->rz;
        s->rz = tot[0];
        s->rr = tot[1];
        s->iters += 1;
        if (tot[1] <= s->thresh) s->done = 1;
    }
}

// p = D^-1 r + beta p
__global__ __launch_bounds__(kB) void cg_direction_kernel(CgArgs a)
{
    if (a.sc->done) return;
    const double beta = a.sc->beta;
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= a.N) return;
    a.p[i] = fma(beta, a.p[i], a.dinv[i] * a.r[i]);
}

inline unsigned grid_of(int64_t n) { return (unsigned)((n + kB - 1) / kB); }
inline unsigned red_grid(int64_t n)
{
    const int64_t g = (n + kB - 1) / kB;
    return (unsigned)(g < kRedBlocks ? (g > 0 ? g : 1) : kRedBlocks);
}

}  // namespace

hipError_t launch_element_matrices(int dim, int order, int blend, const MacroGeo* geo, const Elem* el, int64_t nel,
                                   int n, const QRule* rule, double* me, double* ae, hipStream_t s)
{
    if (nel <= 0) return hipSuccess;
    const int nb = order == 2 ? (dim + 1) * (dim + 2) / 2 : dim + 1;
    const dim3 grid(grid_of(nel * nb)), block(kB);
#define MMOC_EM(D, O, B) element_matrices_kernel<D, O, B><<<grid, block, 0, s>>>(geo, el, nel, n, rule, me, ae)
    if (dim == 2 && order == 2) {
        if (blend) MMOC_EM(2, 2, 1);
        else MMOC_EM(2, 2, 0);
    } else if (dim == 2 && order == 1 && !blend) {
        MMOC_EM(2, 1, 0);
    } else if (dim == 3 && order == 2) {
        if (blend) MMOC_EM(3, 2, 1);
        else MMOC_EM(3, 2, 0);
    } else if (dim == 3 && order == 1 && !blend) {
        MMOC_EM(3, 1, 0);
    } else {
        return hipErrorNotSupported;
    }
#undef MMOC_EM
    return hipGetLastError();
}

hipError_t launch_gather(int64_t nnz, const int64_t* cptr, const int32_t* contrib, const double* me,
                         const double* ae, double* mv, double* av, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    gather_kernel<<<grid_of(nnz), kB, 0, s>>>(nnz, cptr, contrib, me, ae, mv, av);
    return hipGetLastError();
}

hipError_t launch_build_e(int64_t N, const int32_t* rp, const int32_t* ci, const double* mv, const double* av,
                          double s1, const uint8_t* is_dir, int precond, double* ev, double* dinv, hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    build_e_kernel<<<grid_of(N), kB, 0, s>>>(N, rp, ci, mv, av, s1, is_dir, precond, ev, dinv);
    return hipGetLastError();
}

hipError_t launch_spmv(int64_t N, const int32_t* rp, const int32_t* ci, const double* v, const double* x, double* y,
                       hipStream_t s)
{
    if (N <= 0) return hipSuccess;
    spmv_kernel<<<grid_of(N), kB, 0, s>>>(N, rp, ci, v, x, y);
    return hipGetLastError();
}

hipError_t launch_rhs(const RhsArgs& a, hipStream_t s)
{
    if (a.N <= 0) return hipSuccess;
    rhs_kernel<<<grid_of(a.N), kB, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_cg_init(const CgArgs& a, hipStream_t s)
{
    cg_init_kernel<<<red_grid(a.N), kB, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const CgArgs& a, hipStream_t s)
{
    cg_spmv_kernel<<<red_grid(a.N), kB, 0, s>>>(a);
    cg_update_kernel<<<red_grid(a.N), kB, 0, s>>>(a);
    cg_direction_kernel<<<grid_of(a.N), kB, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fe
}  // namespace mmoc
