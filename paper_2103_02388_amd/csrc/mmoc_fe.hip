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
// Operators: a block takes a row block of the CSR matrix, stages the
// products of its entries in LDS with consecutive threads (coalesced reads
// of values and column indices), then each thread sums one row.
//
// Solve: conjugate gradients on the CSR matrix, float64.  Each reducing
// kernel writes one partial sum per block; the next kernel's blocks all sum
// those partials in the same fixed order, so every block derives the same
// step scalars and stop decision without atomics.  Each kernel returns at
// once when the solve has stopped, so that the host can enqueue batches of
// iterations and read the state back once per batch.
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

// Sum of v over the block, returned to every thread; fixed order (wave
// butterflies, then the waves in order), so every block that sums the same
// values gets the same bits.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[NV][kWaves];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double w = wave_sum(v[k]);
        if (lane == 0) sh[k][wave] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = sh[k][0];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) t += sh[k][q];
        v[k] = t;
    }
    __syncthreads();
}

// this thread's share of the partial-sum slots written by the previous
// kernel (G blocks), in block order
template <int NV>
__device__ __forceinline__ void partial_loads(const double* __restrict__ part, const int (&slot)[NV], int G,
                                              double (&out)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = 0.0;
    for (int b = threadIdx.x; b < G; b += kB)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] += part[slot[k] * kMaxRedBlocks + b];
}

// totals of partial-sum slots written by the previous kernel (G blocks)
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, const int (&slot)[NV], int G,
                                             double (&out)[NV])
{
    partial_loads<NV>(part, slot, G, out);
    block_sum<NV>(out);
}

// Row block blk of a CSR matrix: f(k) for each of its entries is staged in
// LDS by consecutive threads (coalesced reads of the values and column
// indices), then thread t returns the sum over row r0 + t in entry order
// (row = -1 for threads past the block's rows).
template <typename F>
__device__ __forceinline__ double stream_row_sum(const Csr& A, int4 h, double* __restrict__ buf, F f, int& row)
{
    const int r0 = h.x, r1 = h.y, base = h.z, end = h.w;
    int k = base + (int)threadIdx.x;
    // four independent entries in flight per thread
    for (; k + 3 * kB < end; k += 4 * kB) {
        const double a0 = f(k), a1 = f(k + kB), a2 = f(k + 2 * kB), a3 = f(k + 3 * kB);
        buf[k - base] = a0;
        buf[k + kB - base] = a1;
        buf[k + 2 * kB - base] = a2;
        buf[k + 3 * kB - base] = a3;
    }
    for (; k < end; k += kB) buf[k - base] = f(k);
    __syncthreads();
    double s = 0.0;
    row = -1;
    if ((int)threadIdx.x < r1 - r0) {
        row = r0 + (int)threadIdx.x;
        const int e = A.rp[row + 1];
        for (int k = A.rp[row]; k < e; ++k) s += buf[k - base];
    }
    __syncthreads();
    return s;
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

__global__ __launch_bounds__(kB) void spmv_kernel(Csr A, const double* __restrict__ v, const double* __restrict__ x,
                                                  double* __restrict__ y)
{
    __shared__ double buf[kLds];
    for (int64_t blk = blockIdx.x; blk < A.nrb; blk += gridDim.x) {
        int row;
        const double s = stream_row_sum(A, A.rb[blk], buf, [&](int k) { return v[k] * x[A.ci[k]]; }, row);
        if (row >= 0) y[row] = s;
    }
}

__global__ __launch_bounds__(kB) void rhs_kernel(RhsArgs a)
{
    __shared__ double buf[kLds];
    for (int64_t blk = blockIdx.x; blk < a.A.nrb; blk += gridDim.x) {
        int row;
        const double s = stream_row_sum(
            a.A, a.A.rb[blk], buf,
            [&](int k) {
                const int32_t j = a.A.ci[k];
                const double m = a.mv[k], st = a.av[k];
                double t = fma(-a.s2, st, m) * a.chat[j];
                if (a.is_dir && a.is_dir[j]) t = fma(-fma(a.s1, st, m), a.g[j], t);
                return t;
            },
            row);
        if (row < 0) continue;
        if (a.is_dir && a.is_dir[row]) {
            a.b[row] = a.g[row];
            a.x[row] = a.g[row];
            continue;
        }
        double acc = s;
        if (a.q0) acc = fma(a.w0, a.q0[row], acc);
        if (a.q1) acc = fma(a.w1, a.q1[row], acc);
        a.b[row] = acc;
        a.x[row] = a.chat[row];
    }
}

__global__ __launch_bounds__(kB) void quadform_kernel(Csr A, const double* __restrict__ v,
                                                      const double* __restrict__ a, const double* __restrict__ a_sub,
                                                      const double* __restrict__ b, const double* __restrict__ b_sub,
                                                      double* __restrict__ part)
{
    __shared__ double buf[kLds];
    double acc[1] = {0.0};
    for (int64_t blk = blockIdx.x; blk < A.nrb; blk += gridDim.x) {
        int i;
        const double mb = stream_row_sum(
            A, A.rb[blk], buf,
            [&](int k) {
                const int32_t j = A.ci[k];
                const double bj = b ? b[j] : 1.0;
                return v[k] * (b_sub ? bj - b_sub[j] : bj);
            },
            i);
        if (i < 0) continue;
        const double ai = (a ? a[i] : 1.0) - (a_sub ? a_sub[i] : 0.0);
        acc[0] = fma(ai, mb, acc[0]);
    }
    block_sum<1>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(kB) void sum_kernel(const double* __restrict__ part, int G, double* __restrict__ out)
{
    const int slot[1] = {0};
    double t[1];
    sum_partials<1>(part, slot, G, t);
    if (threadIdx.x == 0) *out = t[0];
}

// ------------------------------------------------------------------- CG
//
// Preconditioned CG in the Chronopoulos-Gear arrangement: the two inner
// products of an iteration, gamma = (r, u) and delta = (E u, u) with
// u = D^-1 r, come out of the same pass as the matrix product w = E u, so an
// iteration is two kernels with one reduction point:
//   beta = gamma_k / gamma_{k-1},  alpha = gamma_k / (delta_k - beta gamma_k / alpha_{k-1})
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,  u = D^-1 r
// (p = u, s = w, alpha = gamma / delta at k = 0).  In exact arithmetic this
// is the same iteration as the textbook CG; s stays equal to E p.

// r = b - E x, u = D^-1 r; partials of r.r and b.b
__global__ __launch_bounds__(kB) void cg_init_kernel(CgArgs a)
{
    __shared__ double buf[kLds];
    double v[2] = {0.0, 0.0};
    for (int64_t blk = blockIdx.x; blk < a.A.nrb; blk += gridDim.x) {
        int i;
        const double ex = stream_row_sum(a.A, a.A.rb[blk], buf, [&](int k) { return a.ev[k] * a.x[a.A.ci[k]]; }, i);
        if (i < 0) continue;
        const double bi = a.b[i];
        const double r = bi - ex;
        a.r[i] = r;
        a.u[i] = a.dinv[i] * r;
        v[0] = fma(r, r, v[0]);
        v[1] = fma(bi, bi, v[1]);
    }
    block_sum<2>(v);
    if (threadIdx.x == 0) {
        a.part[P_RR * kMaxRedBlocks + blockIdx.x] = v[0];
        a.part[P_BB * kMaxRedBlocks + blockIdx.x] = v[1];
    }
}

__global__ __launch_bounds__(kB) void cg_start_kernel(CgArgs a, int G)
{
    const int slot[2] = {P_RR, P_BB};
    double t[2];
    sum_partials<2>(a.part, slot, G, t);
    if (threadIdx.x == 0) {
        CgScalars* s = a.sc;
        s->rr = t[0];
        s->bb = t[1];
        s->thresh = a.rtol2 * (t[1] > 0.0 ? t[1] : t[0]);
        s->iters = 0;
        s->alpha[0] = s->alpha[1] = 0.0;
        s->done = t[0] <= s->thresh ? (t[1] > 0.0 ? 1 : 3) : 0;
    }
}

// w = E u; partials of gamma = r.u (slot by parity), delta = w.u and r.r
__global__ __launch_bounds__(kB) void cg_spmv_kernel(CgArgs a, int par)
{
    // the stop flag and the first row block's header load together
    const int done = a.sc->done;
    int4 h = a.A.rb[blockIdx.x];  // the grid never exceeds the row blocks
    if (done) return;
    __shared__ double buf[kLds];
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t blk = blockIdx.x; blk < a.A.nrb; blk += gridDim.x) {
        if (blk != blockIdx.x) h = a.A.rb[blk];
        // this thread's row values for the inner products, loaded while the
        // row block streams
        const int ir = h.x + (int)threadIdx.x;
        double r = 0.0, u = 0.0;
        if (ir < h.y) {
            r = a.r[ir];
            u = a.u[ir];
        }
        int i;
        const double w = stream_row_sum(a.A, h, buf, [&](int k) { return a.ev[k] * a.u[a.A.ci[k]]; }, i);
        if (i < 0) continue;
        a.w[i] = w;
        v[0] = fma(r, u, v[0]);
        v[1] = fma(w, u, v[1]);
        v[2] = fma(r, r, v[2]);
    }
    block_sum<3>(v);
    if (threadIdx.x == 0) {
        a.part[(P_G0 + par) * kMaxRedBlocks + blockIdx.x] = v[0];
        a.part[P_DE * kMaxRedBlocks + blockIdx.x] = v[1];
        a.part[P_RR * kMaxRedBlocks + blockIdx.x] = v[2];
    }
}

struct RowVals {
    double u, w, p, s, x, r, dinv;
};

__device__ __forceinline__ void load_row(const CgArgs& a, int i, RowVals& v)
{
    v.u = a.u[i];
    v.w = a.w[i];
    v.p = a.p[i];
    v.s = a.s[i];
    v.x = a.x[i];
    v.r = a.r[i];
    v.dinv = a.dinv[i];
}

// p = u + beta p, s = w + beta s (p = u, s = w at k = 0), x += alpha p,
// r -= alpha s, u = D^-1 r
__device__ __forceinline__ void update_row(const CgArgs& a, int i, const RowVals& v, int k, double alpha,
                                           double beta)
{
    const double p = k == 0 ? v.u : fma(beta, v.p, v.u);
    const double s = k == 0 ? v.w : fma(beta, v.s, v.w);
    a.p[i] = p;
    a.s[i] = s;
    a.x[i] = fma(alpha, p, v.x);
    const double r = fma(-alpha, s, v.r);
    a.r[i] = r;
    a.u[i] = v.dinv * r;
}

// the stop test on r.r, the step scalars, and the vector updates
__global__ __launch_bounds__(kB) void cg_update_kernel(CgArgs a, int k)
{
    // the rows of the first row block are loaded before the reduction, so
    // that the two latencies overlap
    const int done = a.sc->done;
    const int4 h = a.A.rb[blockIdx.x];
    const int par = k & 1;
    const int slot[4] = {P_G0 + par, P_DE, P_RR, P_G0 + (par ^ 1)};
    double t[4];
    partial_loads<4>(a.part, slot, gridDim.x, t);
    const int i0 = h.x + (int)threadIdx.x;
    RowVals v0{};
    if (i0 < h.y) load_row(a, i0, v0);
    if (done) return;
    block_sum<4>(t);
    const double gamma = t[0], delta = t[1], rr = t[2];
    CgScalars* sc = a.sc;
    if (rr <= sc->thresh) {  // r_k is small enough: x_k is the result
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rr = rr;
            sc->iters = k;
            sc->done = 1;
        }
        return;
    }
    double alpha, beta = 0.0;
    if (k == 0) {
        alpha = gamma / delta;
    } else {
        beta = gamma / t[3];
        alpha = gamma / (delta - beta * gamma / sc->alpha[par ^ 1]);
    }
    if (!(alpha > 0.0) || !isfinite(alpha)) {  // E is not positive definite, or NaN
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rr = rr;
            sc->iters = k;
            sc->done = 2;
        }
        return;
    }
    if (i0 < h.y) update_row(a, i0, v0, k, alpha, beta);
    for (int64_t blk = blockIdx.x + gridDim.x; blk < a.A.nrb; blk += gridDim.x) {
        const int4 hb = a.A.rb[blk];
        const int i = hb.x + (int)threadIdx.x;
        if (i >= hb.y) continue;
        RowVals v;
        load_row(a, i, v);
        update_row(a, i, v, k, alpha, beta);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->alpha[par] = alpha;
        sc->beta = beta;
        sc->rr = rr;
        sc->iters = k + 1;
    }
}

inline unsigned grid_of(int64_t n) { return (unsigned)((n + kB - 1) / kB); }
// grid of the reducing kernels: one block per row block, at most kMaxRedBlocks
inline int red_grid(int64_t nrb) { return (int)(nrb < kMaxRedBlocks ? (nrb > 0 ? nrb : 1) : kMaxRedBlocks); }

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

hipError_t launch_spmv(const Csr& A, const double* v, const double* x, double* y, hipStream_t s)
{
    if (A.nrb <= 0) return hipSuccess;
    spmv_kernel<<<(unsigned)A.nrb, kB, 0, s>>>(A, v, x, y);
    return hipGetLastError();
}

hipError_t launch_rhs(const RhsArgs& a, hipStream_t s)
{
    if (a.A.nrb <= 0) return hipSuccess;
    rhs_kernel<<<(unsigned)a.A.nrb, kB, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_quadform(const Csr& A, const double* v, const double* a, const double* a_sub, const double* b,
                           const double* b_sub, double* part, double* out, hipStream_t s)
{
    const int G = red_grid(A.nrb);
    quadform_kernel<<<G, kB, 0, s>>>(A, v, a, a_sub, b, b_sub, part);
    sum_kernel<<<1, kB, 0, s>>>(part, G, out);
    return hipGetLastError();
}

hipError_t launch_cg_init(const CgArgs& a, hipStream_t s)
{
    const int G = red_grid(a.A.nrb);
    cg_init_kernel<<<G, kB, 0, s>>>(a);
    cg_start_kernel<<<1, kB, 0, s>>>(a, G);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const CgArgs& a, int k, hipStream_t s)
{
    const int G = red_grid(a.A.nrb);
    cg_spmv_kernel<<<G, kB, 0, s>>>(a, k & 1);
    cg_update_kernel<<<G, kB, 0, s>>>(a, k);
    return hipGetLastError();
}

}  // namespace fe
}  // namespace mmoc
