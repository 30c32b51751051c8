// mmoc_metrics.cpp -- host side of the benchmark measures (Sec. 3.1) and of
// the look-back driver (Sec. 2.3.3).
#include <math.h>

#include <algorithm>
#include <map>
#include <vector>

#include "mmoc_ctx.h"

namespace {

// Mass matrix of a unit-volume simplex from the moments of the barycentric
// coordinates: int_T lambda^alpha = |T| d! alpha! / (d + |alpha|)!.  The P2
// basis is phi_a = lambda_a (2 lambda_a - 1) at the vertices and phi_ab =
// 4 lambda_a lambda_b at the edge midpoints; the P1 basis is phi_a = lambda_a.
mmoc::MassRef mass_unit(int d, int ord)
{
    using Mono = std::vector<int>;  // exponent of each barycentric coordinate
    using Poly = std::map<Mono, double>;
    const int nv = d + 1;
    std::vector<Poly> basis;
    for (int a = 0; a < nv; ++a) {
        Poly p;
        Mono sq(nv, 0), li(nv, 0);
        sq[a] = 2;
        li[a] = 1;
        if (ord == 2) {
            p[sq] = 2.0;
            p[li] = -1.0;
        } else {
            p[li] = 1.0;
        }
        basis.push_back(p);
    }
    for (int a = 0; a < nv && ord == 2; ++a)
        for (int b = a + 1; b < nv; ++b) {
            Poly p;
            Mono e(nv, 0);
            e[a] = 1;
            e[b] = 1;
            p[e] = 4.0;
            basis.push_back(p);
        }
    auto fact = [](int k) {
        double r = 1.0;
        for (int i = 2; i <= k; ++i) r *= i;
        return r;
    };
    auto moment = [&](const Mono& e) {
        int tot = 0;
        double num = fact(d);
        for (int x : e) {
            tot += x;
            num *= fact(x);
        }
        return num / fact(d + tot);
    };
    const int nn = (int)basis.size();
    mmoc::MassRef R{};
    for (int i = 0; i < nn; ++i)
        for (int j = 0; j < nn; ++j) {
            double v = 0.0;
            for (const auto& [ei, ci] : basis[i])
                for (const auto& [ej, cj] : basis[j]) {
                    Mono e(nv);
                    for (int k = 0; k < nv; ++k) e[k] = ei[k] + ej[k];
                    v += ci * cj * moment(e);
                }
            R.m[i * nn + j] = v;
        }
    return R;
}

mmoc_status ensure_reduction(mmoc_ctx* c, int64_t count)
{
    if (c->red_cap >= count) return MMOC_OK;
    if (c->red_d) {
        HIPCHK(c, hipStreamSynchronize(c->stream), "metric buffer");
        (void)hipFree(c->red_d);
        c->red_d = nullptr;
        c->red_cap = 0;
    }
    double* p = nullptr;
    HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&p), sizeof(double) * (size_t)count), "metric buffer");
    c->red_d = p;
    c->red_cap = count;
    return MMOC_OK;
}

constexpr int64_t kRangeBlocks = 1024;

}  // namespace

extern "C" {

mmoc_status mmoc_mass_inner(mmoc_ctx* c, const double* a, const double* a_sub, const double* b,
                            const double* b_sub, double* out)
{
    if (!c || !out) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    const size_t bytes = sizeof(double) * (size_t)c->N;
    const double* ptrs[4] = {a, a_sub, b, b_sub};
    const char* names[4] = {"a_dev", "a_sub_dev", "b_dev", "b_sub_dev"};
    for (int i = 0; i < 4; ++i) {
        if (!ptrs[i]) continue;
        mmoc_status st = check_dev(c, ptrs[i], bytes, 8, names[i]);
        if (st != MMOC_OK) return st;
    }
    // blended elements are not affine: the assembled quadrature mass matrix
    if (c->blend) return mmoc_fe_mass_quadform(c, a, a_sub, b, b_sub, out);
    const int64_t nb = mmoc::mass_inner_blocks(c->dim, c->nm, c->n);
    mmoc_status st = ensure_reduction(c, std::max<int64_t>(nb, 2 * kRangeBlocks) + 2);
    if (st != MMOC_OK) return st;
    static const mmoc::MassRef R2 = mass_unit(2, 2), R3 = mass_unit(3, 2), Q2 = mass_unit(2, 1),
                               Q3 = mass_unit(3, 1);
    const int ord = c->opt.order;
    const mmoc::MassRef& R = ord == 2 ? (c->dim == 3 ? R3 : R2) : (c->dim == 3 ? Q3 : Q2);
    double* res = c->red_d + c->red_cap - 2;
    HIPCHK(c,
           mmoc::launch_mass_inner(c->dim, ord, c->geo_d, c->slot_uid_d, c->npm, c->nm, c->n, R, a, a_sub, b, b_sub,
                                   c->red_d, res, c->stream),
           "mass inner product");
    HIPCHK(c, hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, c->stream), "mass inner product");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mass inner product");
    return MMOC_OK;
}

mmoc_status mmoc_mass_inner_noalloc(mmoc_ctx* c, const double* a, const double* a_sub, const double* b,
                                    const double* b_sub, double* out_dev)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (c->blend)
        return fail(c, MMOC_E_UNSUPPORTED, "blended meshes use the assembled mass matrix (mmoc_mass_inner)");
    const size_t bytes = sizeof(double) * (size_t)c->N;
    const double* ptrs[4] = {a, a_sub, b, b_sub};
    const char* names[4] = {"a_dev", "a_sub_dev", "b_dev", "b_sub_dev"};
    mmoc_status st;
    for (int i = 0; i < 4; ++i)
        if (ptrs[i] && (st = check_dev(c, ptrs[i], bytes, 8, names[i])) != MMOC_OK) return st;
    if ((st = check_dev(c, out_dev, sizeof(double), 8, "out_dev")) != MMOC_OK) return st;
    const int64_t nb = mmoc::mass_inner_blocks(c->dim, c->nm, c->n);
    if (nb > mmoc::kNoAllocPartials)
        return fail(c, MMOC_E_ARG,
                    "mesh too large for the allocation-free path: %lld partial sums, at most %lld (use mmoc_mass_inner)",
                    (long long)nb, (long long)mmoc::kNoAllocPartials);
    if (!c->noalloc_d) return fail(c, MMOC_E_STATE, "the device scratch array has no address on this device");
    static const mmoc::MassRef R2 = mass_unit(2, 2), R3 = mass_unit(3, 2), Q2 = mass_unit(2, 1),
                               Q3 = mass_unit(3, 1);
    const int ord = c->opt.order;
    const mmoc::MassRef& R = ord == 2 ? (c->dim == 3 ? R3 : R2) : (c->dim == 3 ? Q3 : Q2);
    // every block writes its own partial sum: nothing in the array needs clearing
    HIPCHK(c,
           mmoc::launch_mass_inner(c->dim, ord, c->geo_d, c->slot_uid_d, c->npm, c->nm, c->n, R, a, a_sub, b, b_sub,
                                   c->noalloc_d, out_dev, c->stream),
           "mass inner product");
    return MMOC_OK;
}

mmoc_status mmoc_field_range(mmoc_ctx* c, const double* cf, double* min_out, double* max_out)
{
    if (!c || !min_out || !max_out) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    mmoc_status st = check_dev(c, cf, sizeof(double) * (size_t)c->N, 8, "c_dev");
    if (st != MMOC_OK) return st;
    const int64_t nb = mmoc::mass_inner_blocks(c->dim, c->nm, c->n);
    if ((st = ensure_reduction(c, std::max<int64_t>(nb, 2 * kRangeBlocks) + 2)) != MMOC_OK) return st;
    double* res = c->red_d + c->red_cap - 2;
    HIPCHK(c, mmoc::launch_range(cf, c->N, c->red_d, kRangeBlocks, res, c->stream), "field range");
    double h[2];
    HIPCHK(c, hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, c->stream), "field range");
    HIPCHK(c, hipStreamSynchronize(c->stream), "field range");
    *min_out = h[0];
    *max_out = h[1];
    return MMOC_OK;
}

mmoc_status mmoc_lookback_run(mmoc_ctx* c, double tau, int substeps, int64_t n_steps, int64_t b, double* ring,
                              int64_t ring_len, double* c_out)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (c->prec != MMOC_FP64) return fail(c, MMOC_E_UNSUPPORTED, "the look-back driver runs the float64 tracer");
    if (!c->stationary || !c->vel_set[0])
        return fail(c, MMOC_E_STATE, "the look-back driver needs a stationary velocity (set_stationary + level 0)");
    if (!(tau > 0) || !std::isfinite(tau)) return fail(c, MMOC_E_ARG, "tau must be positive and finite");
    if (n_steps < 1) return fail(c, MMOC_E_ARG, "n_steps must be at least 1");
    if (substeps < 1) return fail(c, MMOC_E_ARG, "substeps must be at least 1");
    const int64_t span = b <= 0 ? n_steps : std::min(b, n_steps);
    if (span * (int64_t)substeps > (1 << 20))
        return fail(c, MMOC_E_ARG, "look-back span x substeps exceeds 2^20 sub-steps");
    const int64_t need_ring = b <= 0 ? 1 : span + 1;
    if (ring_len < need_ring)
        return fail(c, MMOC_E_ARG, "ring_len must be at least %lld", (long long)need_ring);
    const size_t fb = sizeof(double) * (size_t)c->N;
    mmoc_status st = check_dev(c, ring, fb * (size_t)ring_len, 8, "ring_dev");
    if (st != MMOC_OK) return st;
    if ((st = check_dev(c, c_out, fb, 8, "c_out_dev")) != MMOC_OK) return st;
    if (b <= 0) {
        // b = infinity: c^{n_steps} = c^0 at the point traced back over the whole interval
        if ((st = mmoc_set_scalar(c, ring)) != MMOC_OK) return st;
        return mmoc_launch_trace(c, (double)n_steps * tau, (int)(n_steps * substeps), c_out, nullptr, nullptr, c->N);
    }
    for (int64_t n = 1; n <= n_steps; ++n) {
        const int64_t bp = std::min(b, n);
        const double* src = ring + (size_t)((n - bp) % ring_len) * c->N;
        double* dst = ring + (size_t)(n % ring_len) * c->N;
        if ((st = mmoc_set_scalar(c, src)) != MMOC_OK) return st;
        if ((st = mmoc_launch_trace(c, (double)bp * tau, (int)(bp * substeps), dst, nullptr, nullptr, c->N)) != MMOC_OK)
            return st;
    }
    if (c_out != ring + (size_t)(n_steps % ring_len) * c->N)
        HIPCHK(c,
               hipMemcpyAsync(c_out, ring + (size_t)(n_steps % ring_len) * c->N, fb, hipMemcpyDeviceToDevice,
                              c->stream),
               "look-back result");
    return MMOC_OK;
}

mmoc_status mmoc_set_rk_tableau(mmoc_ctx* c, int stages, const double* a, const double* b, const double* cn)
{
    if (!c) return MMOC_E_ARG;
    if (stages == 0) {
        c->rk = mmoc::RKTab{};
        return MMOC_OK;
    }
    if (c->prec == MMOC_FP32_MIXED)
        return fail(c, MMOC_E_UNSUPPORTED, "general RK tableaux run on the float64-arithmetic tracers only");
    if (stages < 1 || stages > mmoc::kMaxStages)
        return fail(c, MMOC_E_ARG, "stages must be in [1, %d] (0 restores RK4)", mmoc::kMaxStages);
    if (!a || !b || !cn) return fail(c, MMOC_E_ARG, "a, b and c must be host arrays");
    mmoc::RKTab t{};
    t.s = stages;
    for (int i = 0; i < stages; ++i) {
        if (!std::isfinite(b[i]) || !std::isfinite(cn[i])) return fail(c, MMOC_E_ARG, "non-finite tableau entry");
        t.b[i] = b[i];
        t.c[i] = cn[i];
        for (int l = 0; l < i; ++l) {
            const double v = a[i * stages + l];
            if (!std::isfinite(v)) return fail(c, MMOC_E_ARG, "non-finite tableau entry");
            t.a[i * mmoc::kMaxStages + l] = v;
        }
        for (int l = i; l < stages; ++l)
            if (a[i * stages + l] != 0.0)
                return fail(c, MMOC_E_ARG, "a must be strictly lower triangular (explicit method)");
    }
    if (cn[0] != 0.0) return fail(c, MMOC_E_ARG, "c[0] must be 0 (explicit method)");
    c->rk = t;
    return MMOC_OK;
}

mmoc_status mmoc_cfl_time_step(mmoc_ctx* c, double cfl, int level, double* tau, double* umax, double* hmin)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (level < 0 || level >= c->lev_cap) return fail(c, MMOC_E_ARG, "level %d is not held", level);
    if (!c->vel_set[level]) return fail(c, MMOC_E_STATE, "velocity level %d is not set", level);
    if (!(cfl > 0) || !std::isfinite(cfl)) return fail(c, MMOC_E_ARG, "cfl must be positive and finite");
    const int64_t nb = mmoc::mass_inner_blocks(c->dim, c->nm, c->n);
    mmoc_status st = ensure_reduction(c, std::max<int64_t>(nb, 2 * kRangeBlocks) + 2);
    if (st != MMOC_OK) return st;
    const int L = phys_level(c, level);
    const bool split = c->dim == 3 && c->prec == MMOC_FP64;  // (x, y) pairs + z
    const int stride = split ? 2 : (c->dim == 3 ? 3 : 2);
    const size_t elem = c->prec == MMOC_FP64 ? sizeof(double) : sizeof(float);
    const void* va = static_cast<const char*>(c->va_all) + (size_t)L * c->va_lstride * elem;
    const void* vb = split ? static_cast<const char*>(c->vb_all) + (size_t)L * c->vb_lstride * elem : nullptr;
    double* res = c->red_d + c->red_cap - 2;
    HIPCHK(c,
           mmoc::launch_speed_max(va, vb, c->zs, c->prec != MMOC_FP64, c->dim, stride, c->nslots, c->red_d, kRangeBlocks,
                                  res, c->stream),
           "largest speed");
    double u = 0.0;
    HIPCHK(c, hipMemcpyAsync(&u, res, sizeof u, hipMemcpyDeviceToHost, c->stream), "largest speed");
    HIPCHK(c, hipStreamSynchronize(c->stream), "largest speed");
    if (umax) *umax = u;
    if (hmin) *hmin = c->hmin;
    if (tau) *tau = u > 0.0 ? cfl * c->hmin / u : INFINITY;
    return MMOC_OK;
}

}  // extern "C"
