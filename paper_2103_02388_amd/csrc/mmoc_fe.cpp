// mmoc_fe.cpp -- set-up and entry points of the finite-element operators
// (Galerkin mass and stiffness matrices) and of the diffusion step of the
// Theta-method (Sec. 2.2, eq. linear-system; the diffusion line of Alg. 1;
// Alg. 2 composes the same call with half steps).
//
// The set-up runs once per context, at the first call that needs the
// matrices: the host enumerates the micro elements and derives the CSR
// pattern and, per CSR slot, the list of element entries that sum into it
// (integer topology only); the device integrates the element matrices and
// sums them into the CSR values.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "mmoc_ctx.h"
#include "mmoc_fe_internal.h"

using mmoc::MacroGeo;
namespace fe = mmoc::fe;

struct fe_state {
    int nb = 0;
    int64_t nel = 0, nnz = 0;
    int32_t* rp_d = nullptr;  // [N + 1]
    int32_t* ci_d = nullptr;  // [nnz], ascending within a row
    int4* rb_d = nullptr;     // [nrb] row blocks: first row, end row, first entry, end entry
    int64_t nrb = 0;
    double* mv_d = nullptr;   // mass matrix values
    double* av_d = nullptr;   // stiffness matrix values
    double* ev_d = nullptr;   // system matrix of the last solve
    double* dinv_d = nullptr;
    uint8_t* dir_d = nullptr;  // boundary DoFs
    std::vector<uint8_t> bmask;
    double *b_d = nullptr, *r_d = nullptr, *u_d = nullptr, *w_d = nullptr, *p_d = nullptr, *s_d = nullptr;
    double* part_d = nullptr;
    fe::CgScalars* sc_d = nullptr;
    // what ev_d / dinv_d hold: s1, Dirichlet rows on/off, preconditioner
    double e_s1 = NAN;
    int e_dir = -1, e_pre = -1;
    int last_iters = 0;  // iterations of the last converged solve: the next one enqueues as many at once
};

namespace {

template <typename T>
mmoc_status fe_alloc(mmoc_ctx* c, T** p, size_t count, const char* what)
{
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, sizeof(T) * count) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, MMOC_E_NOMEM, "device allocation of %s (%zu bytes) failed", what, sizeof(T) * count);
    }
    return MMOC_OK;
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton's method on P_n from
// the three-term recurrence)
void gauss_legendre01(int n, double* x, double* w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (z + 1.0);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2 / ((1 - z^2) P'^2), halved for [0, 1]
    }
}

// collapsed Gauss rule on the reference simplex, n points per direction:
// xi = (u, v (1 - u)[, t (1 - u)(1 - v)]), weight times (1 - u)^(d-1) (1 - v)^(d-2)
fe::QRule simplex_rule(int dim, int n)
{
    fe::QRule R{};
    double g[16], w[16];
    gauss_legendre01(n, g, w);
    int q = 0;
    if (dim == 2) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j, ++q) {
                R.pt[q][0] = g[i];
                R.pt[q][1] = g[j] * (1.0 - g[i]);
                R.w[q] = w[i] * w[j] * (1.0 - g[i]);
            }
    } else {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k, ++q) {
                    R.pt[q][0] = g[i];
                    R.pt[q][1] = g[j] * (1.0 - g[i]);
                    R.pt[q][2] = g[k] * (1.0 - g[i]) * (1.0 - g[j]);
                    R.w[q] = w[i] * w[j] * w[k] * (1.0 - g[i]) * (1.0 - g[i]) * (1.0 - g[j]);
                }
    }
    R.nq = q;
    return R;
}
constexpr int kRulePoints = 4;  // exact to degree 6 (2D) / 5 (3D): the unblended P2 matrices need 4

// Micro simplices of one macro on the n-lattice: for every lattice cube with
// base k (n - 1 >= k_0 >= k_1 [>= k_2] >= 0) and every axis order pi, the
// path k, k + e_pi0, k + e_pi0 + e_pi1, ... when all its vertices stay in
// the macro's Kuhn simplex n >= I >= J [>= K] >= 0.
void micro_simplices(int d, int n, std::vector<std::array<std::array<int16_t, 3>, 4>>& out)
{
    int perm[6][3], np = 0;
    {
        int a[3] = {0, 1, 2};
        do {
            std::memcpy(perm[np++], a, sizeof a);
        } while (std::next_permutation(a, a + d));
    }
    for (int k0 = 0; k0 < n; ++k0)
        for (int k1 = 0; k1 <= k0; ++k1)
            for (int k2 = 0; k2 <= (d == 3 ? k1 : 0); ++k2)
                for (int p = 0; p < np; ++p) {
                    std::array<std::array<int16_t, 3>, 4> v{};
                    int cur[3] = {k0, k1, k2};
                    bool ok = true;
                    for (int a = 0; a <= d; ++a) {
                        if (a > 0) cur[perm[p][a - 1]] += 1;
                        for (int i = 0; i + 1 < d; ++i) ok &= cur[i] >= cur[i + 1];
                        for (int i = 0; i < 3; ++i) v[a][i] = (int16_t)cur[i];
                    }
                    if (ok) out.push_back(v);
                }
}

mmoc_status ensure_fe(mmoc_ctx* c)
{
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "upload a mesh first");
    if (c->fe) return MMOC_OK;
    const int d = c->dim, order = c->m == c->n ? 1 : 2;
    if (c->blend && order == 1) return fail(c, MMOC_E_UNSUPPORTED, "P1 elements are not built for blended meshes");
    const int nb = order == 2 ? (d + 1) * (d + 2) / 2 : d + 1;
    const int64_t N = c->N, npm = c->npm;

    std::vector<int32_t> slot_uid((size_t)c->nslots);
    HIPCHK(c, hipMemcpyAsync(slot_uid.data(), c->slot_uid_d, sizeof(int32_t) * c->nslots, hipMemcpyDeviceToHost,
                             c->stream),
           "slot map to host");
    HIPCHK(c, hipStreamSynchronize(c->stream), "slot map to host");

    // --- elements and their DoFs (P2: 2 V_a and V_a + V_b on the m-lattice; P1: V_a)
    std::vector<std::array<std::array<int16_t, 3>, 4>> simp;
    micro_simplices(d, c->n, simp);
    const int64_t nel = (int64_t)c->nm * (int64_t)simp.size();
    if (nel * nb * nb >= (int64_t)INT32_MAX) return fail(c, MMOC_E_UNSUPPORTED, "mesh too large for the assembly");
    std::vector<fe::Elem> el((size_t)nel);
    std::vector<int32_t> dof((size_t)nel * nb);
    for (int M = 0; M < c->nm; ++M)
        for (size_t s = 0; s < simp.size(); ++s) {
            const int64_t e = (int64_t)M * simp.size() + s;
            fe::Elem& E = el[e];
            E.macro = M;
            std::memset(E.v, 0, sizeof E.v);
            for (int a = 0; a <= d; ++a)
                for (int i = 0; i < 3; ++i) E.v[a][i] = simp[s][a][i];
            int q = 0;
            auto node = [&](int I, int J, int K) {
                dof[e * nb + q++] = slot_uid[(size_t)M * npm + mmoc_lattice_index(d, I, J, d == 3 ? K : 0)];
            };
            const auto& v = simp[s];
            if (order == 1) {
                for (int a = 0; a <= d; ++a) node(v[a][0], v[a][1], v[a][2]);
            } else {
                for (int a = 0; a <= d; ++a) node(2 * v[a][0], 2 * v[a][1], 2 * v[a][2]);
                for (int a = 0; a <= d; ++a)
                    for (int b = a + 1; b <= d; ++b) node(v[a][0] + v[b][0], v[a][1] + v[b][1], v[a][2] + v[b][2]);
            }
        }

    // --- CSR pattern: per row, the columns of every element that holds the
    // row's DoF (bucketed by row, then sorted and deduplicated row by row)
    std::vector<int64_t> off((size_t)N + 1, 0);
    for (int64_t t = 0; t < nel * nb; ++t) off[(size_t)dof[t] + 1] += nb;
    for (int64_t i = 0; i < N; ++i) off[i + 1] += off[i];
    std::vector<int32_t> all((size_t)off[N]);
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int64_t e = 0; e < nel; ++e)
            for (int i = 0; i < nb; ++i) {
                const int32_t r = dof[e * nb + i];
                for (int j = 0; j < nb; ++j) all[fill[r]++] = dof[e * nb + j];
            }
    }
    std::vector<int32_t> rp((size_t)N + 1, 0);
    int64_t nnz = 0;
    for (int64_t i = 0; i < N; ++i) {
        int32_t* b = all.data() + off[i];
        int32_t* en = all.data() + off[i + 1];
        std::sort(b, en);
        en = std::unique(b, en);
        std::memmove(all.data() + nnz, b, sizeof(int32_t) * (size_t)(en - b));  // compact: nnz <= off[i]
        nnz += en - b;
        rp[i + 1] = (int32_t)std::min<int64_t>(nnz, INT32_MAX);
    }
    if (nnz >= (int64_t)INT32_MAX) return fail(c, MMOC_E_UNSUPPORTED, "matrix too large for 32-bit indices");
    all.resize((size_t)nnz);
    std::vector<int32_t> ci = std::move(all);
    off.clear();
    off.shrink_to_fit();

    // --- per slot, the element entries that sum into it, in element order
    std::vector<int32_t> slot_of((size_t)nel * nb * nb);
    std::vector<int64_t> cptr((size_t)nnz + 1, 0);
    for (int64_t e = 0; e < nel; ++e)
        for (int i = 0; i < nb; ++i) {
            const int32_t r = dof[e * nb + i];
            const int32_t* b = ci.data() + rp[r];
            const int32_t* en = ci.data() + rp[r + 1];
            for (int j = 0; j < nb; ++j) {
                const int32_t k = (int32_t)(std::lower_bound(b, en, dof[e * nb + j]) - ci.data());
                slot_of[(e * nb + i) * nb + j] = k;
                cptr[k + 1] += 1;
            }
        }
    for (int64_t k = 0; k < nnz; ++k) cptr[k + 1] += cptr[k];
    std::vector<int32_t> contrib((size_t)nel * nb * nb);
    {
        std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t t = 0; t < nel * nb * nb; ++t) contrib[fill[slot_of[t]]++] = (int32_t)t;
    }
    slot_of.clear();
    slot_of.shrink_to_fit();

    // --- row blocks: consecutive rows, at most kRowsPerBlock of them and
    // at most kLds entries in all
    std::vector<int32_t> rb(1, 0);
    for (int64_t i = 0; i < N; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        if (len > fe::kLds) return fail(c, MMOC_E_UNSUPPORTED, "matrix row %lld has too many entries", (long long)i);
        const int32_t r0 = rb.back();
        if (i - r0 == fe::kRowsPerBlock || rp[i + 1] - rp[r0] > fe::kLds) rb.push_back((int32_t)i);
    }
    rb.push_back((int32_t)N);
    std::vector<int4> rbh(rb.size() - 1);
    for (size_t b = 0; b + 1 < rb.size(); ++b) rbh[b] = make_int4(rb[b], rb[b + 1], rp[rb[b]], rp[rb[b + 1]]);

    // --- boundary DoFs: lattice nodes on macro faces without a neighbour
    std::vector<uint8_t> bmask((size_t)N, 0);
    const int m = c->m;
    for (int M = 0; M < c->nm; ++M) {
        bool any = false;
        for (int k = 0; k <= d; ++k) any |= c->geo_h[M].nbr[k] < 0;
        if (!any) continue;
        int64_t idx = 0;
        for (int I = 0; I <= m; ++I)
            for (int J = 0; J <= I; ++J)
                for (int K = 0; K <= (d == 3 ? J : 0); ++K, ++idx) {
                    const int w[4] = {m - I, I - J, d == 3 ? J - K : J, d == 3 ? K : 0};
                    for (int k = 0; k <= d; ++k)
                        if (w[k] == 0 && c->geo_h[M].nbr[k] < 0) bmask[slot_uid[(size_t)M * npm + idx]] = 1;
                }
    }

    // --- device: element matrices, then the CSR sums
    fe_state* F = new fe_state();
    c->fe = F;
    F->nb = nb;
    F->nel = nel;
    F->nnz = nnz;
    F->bmask = std::move(bmask);
    mmoc_status st;
    fe::Elem* el_d = nullptr;
    fe::QRule* rule_d = nullptr;
    double *me_d = nullptr, *ae_d = nullptr;
    int64_t* cptr_d = nullptr;
    int32_t* contrib_d = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(el_d);
        (void)hipFree(rule_d);
        (void)hipFree(me_d);
        (void)hipFree(ae_d);
        (void)hipFree(cptr_d);
        (void)hipFree(contrib_d);
    };
    auto bail = [&](mmoc_status s) {
        cleanup();
        mmoc_fe_free_state(c);
        return s;
    };
    const size_t ne = (size_t)nel * nb * nb;
    if ((st = fe_alloc(c, &F->rp_d, (size_t)N + 1, "CSR rows")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->ci_d, (size_t)nnz, "CSR columns")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->rb_d, rbh.size(), "CSR row blocks")) != MMOC_OK) return bail(st);
    F->nrb = (int64_t)rbh.size();  // >= 1: a mesh has DoFs
    if ((st = fe_alloc(c, &F->mv_d, (size_t)nnz, "mass matrix")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->av_d, (size_t)nnz, "stiffness matrix")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->ev_d, (size_t)nnz, "system matrix")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->dinv_d, (size_t)N, "diagonal")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->dir_d, (size_t)N, "boundary mask")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->b_d, (size_t)N, "CG vector b")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->r_d, (size_t)N, "CG vector r")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->u_d, (size_t)N, "CG vector u")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->w_d, (size_t)N, "CG vector w")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->p_d, (size_t)N, "CG vector p")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->s_d, (size_t)N, "CG vector s")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &F->part_d, (size_t)fe::P_SLOTS * fe::kMaxRedBlocks, "CG partial sums")) != MMOC_OK)
        return bail(st);
    if ((st = fe_alloc(c, &F->sc_d, 1, "CG scalars")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &el_d, (size_t)nel, "element table")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &rule_d, 1, "quadrature rule")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &me_d, ne, "element mass matrices")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &ae_d, ne, "element stiffness matrices")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &cptr_d, (size_t)nnz + 1, "slot lists")) != MMOC_OK) return bail(st);
    if ((st = fe_alloc(c, &contrib_d, ne, "slot entries")) != MMOC_OK) return bail(st);
    const fe::QRule rule = simplex_rule(d, kRulePoints);
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    up(F->rp_d, rp.data(), sizeof(int32_t) * rp.size());
    up(F->ci_d, ci.data(), sizeof(int32_t) * ci.size());
    up(F->rb_d, rbh.data(), sizeof(int4) * rbh.size());
    up(F->dir_d, F->bmask.data(), F->bmask.size());
    up(el_d, el.data(), sizeof(fe::Elem) * el.size());
    up(rule_d, &rule, sizeof rule);
    up(cptr_d, cptr.data(), sizeof(int64_t) * cptr.size());
    up(contrib_d, contrib.data(), sizeof(int32_t) * contrib.size());
    if (e == hipSuccess)
        e = fe::launch_element_matrices(d, order, c->blend, c->geo_d, el_d, nel, c->n, rule_d, me_d, ae_d, c->stream);
    if (e == hipSuccess) e = fe::launch_gather(nnz, cptr_d, contrib_d, me_d, ae_d, F->mv_d, F->av_d, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        hip_fail(c, e, "finite-element assembly");
        return bail(MMOC_E_HIP);
    }
    cleanup();
    return MMOC_OK;
}

fe::Csr csr_of(const mmoc_ctx* c)
{
    const fe_state* F = c->fe;
    return fe::Csr{c->N, F->nrb, F->rp_d, F->ci_d, F->rb_d};
}

}  // namespace

void mmoc_fe_free_state(mmoc_ctx* c)
{
    fe_state* F = c->fe;
    if (!F) return;
    for (void* p : {(void*)F->rp_d, (void*)F->ci_d, (void*)F->rb_d, (void*)F->mv_d, (void*)F->av_d, (void*)F->ev_d,
                    (void*)F->dinv_d, (void*)F->dir_d, (void*)F->b_d, (void*)F->r_d, (void*)F->u_d, (void*)F->w_d,
                    (void*)F->p_d, (void*)F->s_d, (void*)F->part_d, (void*)F->sc_d})
        (void)hipFree(p);
    delete F;
    c->fe = nullptr;
}

// (a - a_sub)^T M (b - b_sub) with the assembled mass matrix (the measures
// of a blended mesh; arguments already checked by the caller)
mmoc_status mmoc_fe_mass_quadform(mmoc_ctx* c, const double* a, const double* a_sub, const double* b,
                                  const double* b_sub, double* out)
{
    mmoc_status st = ensure_fe(c);
    if (st != MMOC_OK) return st;
    fe_state* F = c->fe;
    // the CG partial sums double as scratch: no solve runs concurrently on a context's stream
    double* res = F->part_d + (size_t)fe::P_SLOTS * fe::kMaxRedBlocks - 1;
    HIPCHK(c, fe::launch_quadform(csr_of(c), F->mv_d, a, a_sub, b, b_sub, F->part_d, res, c->stream),
           "mass quadratic form");
    HIPCHK(c, hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, c->stream), "mass quadratic form");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mass quadratic form");
    return MMOC_OK;
}

extern "C" {

mmoc_status mmoc_fe_assemble(mmoc_ctx* c, int64_t* nnz)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = ensure_fe(c);
    if (st != MMOC_OK) return st;
    if (nnz) *nnz = c->fe->nnz;
    return MMOC_OK;
}

mmoc_status mmoc_fe_export(mmoc_ctx* c, mmoc_matrix which, int64_t* row_ptr, int32_t* cols, double* vals)
{
    if (!c) return MMOC_E_ARG;
    if (which != MMOC_MAT_MASS && which != MMOC_MAT_STIFFNESS) return fail(c, MMOC_E_ARG, "unknown matrix");
    mmoc_status st = ensure_fe(c);
    if (st != MMOC_OK) return st;
    fe_state* F = c->fe;
    std::vector<int32_t> rp(row_ptr ? (size_t)c->N + 1 : 0);
    if (row_ptr)
        HIPCHK(c, hipMemcpyAsync(rp.data(), F->rp_d, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost, c->stream),
               "export rows");
    if (cols)
        HIPCHK(c, hipMemcpyAsync(cols, F->ci_d, sizeof(int32_t) * F->nnz, hipMemcpyDeviceToHost, c->stream),
               "export columns");
    if (vals)
        HIPCHK(c, hipMemcpyAsync(vals, which == MMOC_MAT_MASS ? F->mv_d : F->av_d, sizeof(double) * F->nnz,
                                 hipMemcpyDeviceToHost, c->stream),
               "export values");
    HIPCHK(c, hipStreamSynchronize(c->stream), "export");
    for (size_t i = 0; i < rp.size(); ++i) row_ptr[i] = rp[i];
    return MMOC_OK;
}

mmoc_status mmoc_fe_apply(mmoc_ctx* c, mmoc_matrix which, const double* x, double* y)
{
    if (!c) return MMOC_E_ARG;
    if (which != MMOC_MAT_MASS && which != MMOC_MAT_STIFFNESS) return fail(c, MMOC_E_ARG, "unknown matrix");
    mmoc_status st = ensure_fe(c);
    if (st != MMOC_OK) return st;
    const size_t bytes = sizeof(double) * (size_t)c->N;
    if ((st = check_dev(c, x, bytes, 8, "x")) != MMOC_OK) return st;
    if ((st = check_dev(c, y, bytes, 8, "y")) != MMOC_OK) return st;
    if (x == y) return fail(c, MMOC_E_ARG, "x and y must not alias");
    fe_state* F = c->fe;
    HIPCHK(c, fe::launch_spmv(csr_of(c), which == MMOC_MAT_MASS ? F->mv_d : F->av_d, x, y, c->stream),
           "operator apply");
    return MMOC_OK;
}

mmoc_status mmoc_boundary_mask(mmoc_ctx* c, uint8_t* mask)
{
    if (!c) return MMOC_E_ARG;
    if (!mask) return fail(c, MMOC_E_ARG, "null mask");
    mmoc_status st = ensure_fe(c);
    if (st != MMOC_OK) return st;
    std::memcpy(mask, c->fe->bmask.data(), c->fe->bmask.size());
    return MMOC_OK;
}

mmoc_status mmoc_diffusion_step(mmoc_ctx* c, const mmoc_diffusion_args* args, const double* c_hat, double* c_out,
                                mmoc_diffusion_info* info)
{
    if (!c) return MMOC_E_ARG;
    if (!args) return fail(c, MMOC_E_ARG, "null arguments");
    const mmoc_diffusion_args& A = *args;
    if (!(A.theta >= 0.0 && A.theta <= 1.0)) return fail(c, MMOC_E_ARG, "theta must lie in [0, 1]");
    if (!(A.tau > 0.0) || !std::isfinite(A.tau)) return fail(c, MMOC_E_ARG, "tau must be positive and finite");
    if (!(A.kappa >= 0.0) || !std::isfinite(A.kappa)) return fail(c, MMOC_E_ARG, "kappa must be >= 0 and finite");
    if (A.rtol < 0.0 || !std::isfinite(A.rtol)) return fail(c, MMOC_E_ARG, "rtol must be >= 0 (0: default)");
    if (A.max_iter < 0) return fail(c, MMOC_E_ARG, "max_iter must be >= 0 (0: default)");
    if (A.precond != 0 && A.precond != 1) return fail(c, MMOC_E_ARG, "precond must be 0 or 1");
    mmoc_status st = ensure_fe(c);
    if (st != MMOC_OK) return st;
    const size_t bytes = sizeof(double) * (size_t)c->N;
    if ((st = check_dev(c, c_hat, bytes, 8, "c_hat")) != MMOC_OK) return st;
    if ((st = check_dev(c, c_out, bytes, 8, "c_out")) != MMOC_OK) return st;
    if (c_hat == c_out || A.q0 == c_out || A.q1 == c_out || A.dirichlet == c_out)
        return fail(c, MMOC_E_ARG, "c_out must not alias c_hat, q0, q1 or dirichlet");
    if (A.q0 && (st = check_dev(c, A.q0, bytes, 8, "q0")) != MMOC_OK) return st;
    if (A.q1 && (st = check_dev(c, A.q1, bytes, 8, "q1")) != MMOC_OK) return st;
    if (A.dirichlet && (st = check_dev(c, A.dirichlet, bytes, 8, "dirichlet")) != MMOC_OK) return st;
    const double rtol = A.rtol > 0.0 ? A.rtol : 1e-12;
    const int max_iter = A.max_iter > 0 ? A.max_iter : 1000;
    fe_state* F = c->fe;
    const double s1 = A.tau * A.theta * A.kappa, s2 = A.tau * (1.0 - A.theta) * A.kappa;
    const int dir = A.dirichlet ? 1 : 0;
    const uint8_t* is_dir = dir ? F->dir_d : nullptr;
    if (!(F->e_s1 == s1) || F->e_dir != dir || F->e_pre != A.precond) {
        HIPCHK(c, fe::launch_build_e(c->N, F->rp_d, F->ci_d, F->mv_d, F->av_d, s1, is_dir, A.precond, F->ev_d,
                                     F->dinv_d, c->stream),
               "system matrix");
        F->e_s1 = s1;
        F->e_dir = dir;
        F->e_pre = A.precond;
    }
    fe::RhsArgs ra{csr_of(c), F->mv_d, F->av_d, s1, s2, A.tau * (1.0 - A.theta), A.tau * A.theta,
                   c_hat, A.q0, A.q1, A.dirichlet, is_dir, F->b_d, c_out};
    HIPCHK(c, fe::launch_rhs(ra, c->stream), "right-hand side");
    fe::CgArgs ca{csr_of(c), F->ev_d, F->dinv_d, F->b_d, c_out, F->r_d, F->u_d, F->w_d, F->p_d, F->s_d,
                  F->part_d, F->sc_d, rtol * rtol};
    HIPCHK(c, fe::launch_cg_init(ca, c->stream), "CG start");
    // Iterations are enqueued in batches and the state is read back after
    // each; iterations past the stop return at once.  Successive solves of
    // a time loop take similar counts, so the first batch is the last
    // solve's count plus the iteration that detects the stop, then small
    // batches follow.
    fe::CgScalars h{};
    int launched = 0;
    int next = F->last_iters > 0 ? F->last_iters + 1 : 16;
    for (;;) {
        HIPCHK(c, hipMemcpyAsync(&h, F->sc_d, sizeof h, hipMemcpyDeviceToHost, c->stream), "CG state");
        HIPCHK(c, hipStreamSynchronize(c->stream), "CG state");
        if (h.done || launched >= max_iter) break;
        const int batch = std::min(max_iter - launched, next);
        for (int k = 0; k < batch; ++k) HIPCHK(c, fe::launch_cg_iteration(ca, launched + k, c->stream), "CG iteration");
        launched += batch;
        next = F->last_iters > 0 ? 4 : 32;
    }
    if (h.done == 1) F->last_iters = h.iters;
    if (info) {
        info->iterations = h.iters;
        info->converged = (h.done == 1 || h.done == 3) ? 1 : 0;
        info->rel_residual = h.bb > 0.0 ? std::sqrt(h.rr / h.bb) : std::sqrt(h.rr);
    }
    return MMOC_OK;
}

}  // extern "C"
