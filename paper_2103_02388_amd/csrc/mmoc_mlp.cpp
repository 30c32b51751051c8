// mmoc_mlp.cpp -- host side of the learned flow-map surrogate: parameter and
// optimizer state, training-pair buffers, the training loop and the
// surrogate step (inference, RK4 check sample, per-tile fallback).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "../../include/mmoc.h"
#include "mmoc_ctx.h"
#include "mmoc_internal.h"
#include "mmoc_mlp_internal.h"

using namespace mmoc::mlp;

struct mlp_state {
    double lo[4] = {0, 0, 0, 0}, hi[4] = {1, 1, 1, 1};
    double U = 1.0;
    float* p32 = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    __bf16* wbf = nullptr;  // w2, w3, w2t, w3t (4 x 64 x 64)
    int64_t adam_t = 0;
    // training pairs
    float* in4 = nullptr;
    float* tg3 = nullptr;
    int64_t cap = 0, count = 0;
    // training scratch
    int32_t* sel = nullptr;
    int64_t sel_n = 0;
    float* part = nullptr;
    float* scratch = nullptr;
    float* losses = nullptr;
    int64_t part_tiles = 0, losses_n = 0;
    // surrogate step scratch
    int32_t* ids = nullptr;
    unsigned long long* n_ids = nullptr;  // [2]: the check list's length (second entry unused)
    unsigned char* checked = nullptr;
    double* Xrk = nullptr;  // check points; the predictor's points while recording
    // predictor: the network learns the correction to the context's own RK4
    // trace with pred_substeps sub-steps (0: the whole displacement)
    int pred_substeps = 0;
    double corr_scale = 1.0;  // output scale of the correction
    double period = 0.0;      // > 0: the time input is t mod period
    // the check's RK4 trace runs on a second stream beside the network
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

constexpr int kTile = mmoc::kSurrogateTile;

MlpArgs args_of(mmoc_ctx* c)
{
    mlp_state* S = c->mlp;
    MlpArgs a{};
    a.geo = c->geo_d;
    a.owned = c->owned_d;
    a.n = c->N;
    a.lat_m = c->m;
    for (int i = 0; i < 4; ++i) {
        a.lo[i] = S->lo[i];
        a.hi[i] = S->hi[i];
    }
    a.p32 = S->p32;
    a.w2 = S->wbf;
    a.w3 = S->wbf + H * H;
    a.w2t = S->wbf + 2 * H * H;
    a.w3t = S->wbf + 3 * H * H;
    return a;
}

MlpState state_of(mmoc_ctx* c, float* grad)
{
    mlp_state* S = c->mlp;
    MlpState st{};
    st.p32 = S->p32;
    st.m = S->m;
    st.v = S->v;
    st.grad = grad;
    st.w2 = S->wbf;
    st.w3 = S->wbf + H * H;
    st.w2t = S->wbf + 2 * H * H;
    st.w3t = S->wbf + 3 * H * H;
    return st;
}

template <typename T>
mmoc_status alloc(mmoc_ctx* c, T** p, size_t count, const char* what)
{
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (!count) return MMOC_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(c, e, what);
    }
    return MMOC_OK;
}

// He-style initialisation, seeded
std::vector<float> init_params(uint64_t seed)
{
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<float> p(NP);
    auto fill = [&](int off, int outs, int ins) {
        for (int i = 0; i < outs * ins; ++i) p[off + i] = (float)(nd(rng) * std::sqrt(2.0 / ins));
    };
    fill(OW1, H, 4);
    fill(OW2, H, H);
    fill(OW3, H, H);
    fill(OW4, 3, H);
    for (int o = 0; o < H; ++o) p[OB1 + o] = p[OB2 + o] = p[OB3 + o] = 0.f;
    for (int o = 0; o < 3; ++o) p[OB4 + o] = 0.f;
    return p;
}

// the network's time input: t, or its phase t mod period
double time_input(const mlp_state* S, double t)
{
    return S->period > 0 ? t - S->period * std::floor(t / S->period) : t;
}

// the velocity levels of a step are set (the predictor traces through them)
mmoc_status need_velocity(mmoc_ctx* c)
{
    if (c->lev_cap < 1 || !c->vel_set[0]) return fail(c, MMOC_E_STATE, "velocity level 0 is not set");
    if (!c->stationary && !c->vel_set[1]) return fail(c, MMOC_E_STATE, "velocity level 1 is not set");
    return MMOC_OK;
}

// the predictor's departure points of every particle into X (no scalar)
mmoc_status run_predictor(mmoc_ctx* c, double dt, double* X)
{
    return mmoc_launch_trace(c, dt, c->mlp->pred_substeps, nullptr, X, nullptr, c->N);
}

mmoc_status need_aux(mmoc_ctx* c)
{
    mlp_state* S = c->mlp;
    if (S->aux) return MMOC_OK;
    HIPCHK(c, hipStreamCreateWithFlags(&S->aux, hipStreamNonBlocking), "check stream");
    HIPCHK(c, hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming), "check stream events");
    HIPCHK(c, hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming), "check stream events");
    return MMOC_OK;
}

mmoc_status need_mlp(mmoc_ctx* c)
{
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (!c->mlp) return fail(c, MMOC_E_STATE, "surrogate not configured (mmoc_mlp_configure)");
    if (c->dim != 3 || c->blend) return fail(c, MMOC_E_UNSUPPORTED, "the surrogate is built for unblended 3D meshes");
    return MMOC_OK;
}

}  // namespace

void mmoc_mlp_free_state(mmoc_ctx* c)
{
    mlp_state* S = c->mlp;
    if (!S) return;
    void* ptrs[] = {S->p32, S->m, S->v, S->grad, S->wbf, S->in4, S->tg3, S->sel, S->part, S->scratch, S->losses,
                    S->ids, S->n_ids, S->checked, S->Xrk};
    for (void* p : ptrs) (void)hipFree(p);
    if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
    if (S->ev_join) (void)hipEventDestroy(S->ev_join);
    if (S->aux) (void)hipStreamDestroy(S->aux);
    delete S;
    c->mlp = nullptr;
}

extern "C" {

int64_t mmoc_mlp_nparams(void) { return NP; }

mmoc_status mmoc_mlp_configure(mmoc_ctx* c, const double* lo, const double* hi, double U)
{
    if (!c) return MMOC_E_ARG;
    if (!lo || !hi || !(U > 0) || !std::isfinite(U)) return fail(c, MMOC_E_ARG, "need lo[4], hi[4] and U > 0");
    for (int i = 0; i < 4; ++i)
        if (!(hi[i] > lo[i])) return fail(c, MMOC_E_ARG, "input box component %d is empty", i);
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (c->dim != 3 || c->blend) return fail(c, MMOC_E_UNSUPPORTED, "the surrogate is built for unblended 3D meshes");
    const bool fresh = c->mlp == nullptr;
    if (fresh) c->mlp = new mlp_state();
    mlp_state* S = c->mlp;
    for (int i = 0; i < 4; ++i) {
        S->lo[i] = lo[i];
        S->hi[i] = hi[i];
    }
    S->U = U;
    if (!fresh) return MMOC_OK;
    mmoc_status st;
    if ((st = alloc(c, &S->p32, NP, "mlp parameters")) != MMOC_OK ||
        (st = alloc(c, &S->m, NP, "adam moments")) != MMOC_OK || (st = alloc(c, &S->v, NP, "adam moments")) != MMOC_OK ||
        (st = alloc(c, &S->grad, NP, "gradient")) != MMOC_OK ||
        (st = alloc(c, &S->wbf, 4 * H * H, "bf16 weights")) != MMOC_OK ||
        (st = alloc(c, &S->ids, (size_t)c->N, "surrogate lists")) != MMOC_OK ||
        (st = alloc(c, &S->n_ids, 2, "surrogate counts")) != MMOC_OK ||
        (st = alloc(c, &S->checked, (size_t)c->N, "surrogate flags")) != MMOC_OK ||
        (st = alloc(c, &S->Xrk, (size_t)c->N * 3, "surrogate check points")) != MMOC_OK) {
        mmoc_mlp_free_state(c);
        return st;
    }
    std::vector<float> p = init_params(0x5eedULL);
    HIPCHK(c, hipMemcpyAsync(S->p32, p.data(), sizeof(float) * NP, hipMemcpyHostToDevice, c->stream), "init weights");
    HIPCHK(c, hipMemsetAsync(S->m, 0, sizeof(float) * NP, c->stream), "init moments");
    HIPCHK(c, hipMemsetAsync(S->v, 0, sizeof(float) * NP, c->stream), "init moments");
    HIPCHK(c, launch_refresh(state_of(c, nullptr), c->stream), "init bf16 weights");
    HIPCHK(c, hipStreamSynchronize(c->stream), "init weights");
    return MMOC_OK;
}

mmoc_status mmoc_mlp_get_weights(mmoc_ctx* c, float* host, int64_t n)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (!host || n != NP) return fail(c, MMOC_E_ARG, "need a host buffer of %d floats", NP);
    HIPCHK(c, hipMemcpyAsync(host, c->mlp->p32, sizeof(float) * NP, hipMemcpyDeviceToHost, c->stream), "get weights");
    HIPCHK(c, hipStreamSynchronize(c->stream), "get weights");
    return MMOC_OK;
}

mmoc_status mmoc_mlp_set_weights(mmoc_ctx* c, const float* host, int64_t n)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (!host || n != NP) return fail(c, MMOC_E_ARG, "need a host buffer of %d floats", NP);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return fail(c, MMOC_E_ARG, "parameter %lld is not finite", (long long)i);
    mlp_state* S = c->mlp;
    HIPCHK(c, hipMemcpyAsync(S->p32, host, sizeof(float) * NP, hipMemcpyHostToDevice, c->stream), "set weights");
    HIPCHK(c, hipMemsetAsync(S->m, 0, sizeof(float) * NP, c->stream), "reset moments");
    HIPCHK(c, hipMemsetAsync(S->v, 0, sizeof(float) * NP, c->stream), "reset moments");
    S->adam_t = 0;
    HIPCHK(c, launch_refresh(state_of(c, nullptr), c->stream), "refresh bf16 weights");
    HIPCHK(c, hipStreamSynchronize(c->stream), "set weights");
    return MMOC_OK;
}

mmoc_status mmoc_mlp_record(mmoc_ctx* c, double t_np1, double dt, const double* X, int64_t capacity)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (!(dt > 0) || !std::isfinite(t_np1)) return fail(c, MMOC_E_ARG, "need dt > 0 and a finite t");
    if ((st = check_dev(c, X, sizeof(double) * 3 * c->N, 8, "X_dev")) != MMOC_OK) return st;
    mlp_state* S = c->mlp;
    if (!S->in4) {
        if (capacity < c->N || capacity > (int64_t)1 << 31) return fail(c, MMOC_E_ARG, "capacity must be in [n_unique, 2^31]");
        if ((st = alloc(c, &S->in4, (size_t)capacity * 4, "training inputs")) != MMOC_OK) return st;
        if ((st = alloc(c, &S->tg3, (size_t)capacity * 3, "training targets")) != MMOC_OK) return st;
        S->cap = capacity;
        S->count = 0;
    }
    if (S->count + c->N > S->cap) return fail(c, MMOC_E_ARG, "record buffer full (%lld pairs)", (long long)S->cap);
    MlpArgs a = args_of(c);
    const double* Xp = nullptr;
    double inv = 1.0 / (dt * S->U);
    if (S->pred_substeps > 0) {
        // the target is the correction to the predictor of the same step
        if ((st = need_velocity(c)) != MMOC_OK) return st;
        if ((st = run_predictor(c, dt, S->Xrk)) != MMOC_OK) return st;
        Xp = S->Xrk;
        inv = 1.0 / S->corr_scale;
    }
    HIPCHK(c, launch_record(a, time_input(S, t_np1), inv, X, Xp, S->in4 + S->count * 4, S->tg3 + S->count * 3,
                            c->stream),
           "record");
    S->count += c->N;
    return MMOC_OK;
}

mmoc_status mmoc_mlp_train(mmoc_ctx* c, int64_t n_samples, int epochs, int batch, float lr, unsigned long long seed,
                           double* final_loss)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    mlp_state* S = c->mlp;
    if (S->count <= 0) return fail(c, MMOC_E_STATE, "no training pairs recorded");
    if (batch <= 0 || batch % 64 || batch > (1 << 20)) return fail(c, MMOC_E_ARG, "batch must be a positive multiple of 64");
    if (n_samples < batch || n_samples > ((int64_t)1 << 31)) return fail(c, MMOC_E_ARG, "n_samples must be in [batch, 2^31]");
    if (epochs < 1 || !(lr > 0)) return fail(c, MMOC_E_ARG, "need epochs >= 1 and lr > 0");
    const int ntiles = batch / 64;
    const int64_t spe = n_samples / batch;
    if (S->sel_n != n_samples && (st = alloc(c, &S->sel, (size_t)n_samples, "sample selection")) != MMOC_OK) return st;
    S->sel_n = n_samples;
    if (S->part_tiles < ntiles) {
        if ((st = alloc(c, &S->part, (size_t)ntiles * (NP + 1), "partial gradients")) != MMOC_OK) return st;
        if ((st = alloc(c, &S->scratch, (size_t)ntiles * 5 * H * H, "training scratch")) != MMOC_OK) return st;
        S->part_tiles = ntiles;
    }
    if (S->losses_n < spe) {
        if ((st = alloc(c, &S->losses, (size_t)spe, "losses")) != MMOC_OK) return st;
        S->losses_n = spe;
    }
    // the training set: n_samples pairs drawn (with replacement) from the records
    HIPCHK(c, launch_draw(seed, n_samples, S->count, S->sel, c->stream), "draw samples");
    // each epoch walks the set in the order q -> (q P + O) mod n_samples
    static const int64_t primes[] = {1000003, 1000033, 1000037, 1000039, 1000081, 1000099, 1000117, 1000121,
                                     1000133, 1000151, 1000159, 1000171, 1000183, 1000187, 1000193, 1000199};
    std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ull);
    MlpArgs a = args_of(c);
    const int64_t total = (int64_t)epochs * spe;
    int64_t step = 0;
    for (int e = 0; e < epochs; ++e) {
        int64_t P = 1;
        for (int k = 0; k < 16; ++k) {
            const int64_t q = primes[(e + k) % 16] % n_samples;
            if (q != 0 && std::gcd(q, n_samples) == 1) {
                P = q;
                break;
            }
        }
        const int64_t O = (int64_t)(rng() % (uint64_t)n_samples);
        for (int64_t k = 0; k < spe; ++k, ++step) {
            // cosine decay from lr to lr / 100
            const double fr = (double)step / (double)(total > 1 ? total - 1 : 1);
            const float lrt = (float)(lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * fr))));
            const int64_t off = (k * (int64_t)batch % n_samples * P + O) % n_samples;
            S->adam_t += 1;
            HIPCHK(c, launch_train_step(a, state_of(c, S->grad), S->in4, S->tg3, S->sel, off, n_samples, P, batch, S->part,
                                        S->scratch, lrt, S->adam_t, S->losses + k, c->stream),
                   "train step");
        }
    }
    if (final_loss) {
        std::vector<float> l((size_t)spe);
        HIPCHK(c, hipMemcpyAsync(l.data(), S->losses, sizeof(float) * spe, hipMemcpyDeviceToHost, c->stream), "losses");
        HIPCHK(c, hipStreamSynchronize(c->stream), "train");
        double acc = 0;
        for (float v : l) acc += v;
        *final_loss = acc / (double)spe;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream), "train");
    return MMOC_OK;
}

mmoc_status mmoc_mlp_forward(mmoc_ctx* c, const float* in4, int64_t n, float* out3)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (n <= 0) return fail(c, MMOC_E_ARG, "n must be positive");
    if ((st = check_dev(c, in4, sizeof(float) * 4 * n, 4, "in_dev")) != MMOC_OK) return st;
    if ((st = check_dev(c, out3, sizeof(float) * 3 * n, 4, "out_dev")) != MMOC_OK) return st;
    HIPCHK(c, launch_forward(args_of(c), in4, n, out3, c->stream), "mlp forward");
    return MMOC_OK;
}

mmoc_status mmoc_mlp_loss_grad(mmoc_ctx* c, const float* in4, const float* tg3, int64_t n, float* grad, double* loss)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (n <= 0 || n % 64 || n > (1 << 20)) return fail(c, MMOC_E_ARG, "n must be a positive multiple of 64");
    if ((st = check_dev(c, in4, sizeof(float) * 4 * n, 4, "in_dev")) != MMOC_OK) return st;
    if ((st = check_dev(c, tg3, sizeof(float) * 3 * n, 4, "target_dev")) != MMOC_OK) return st;
    if ((st = check_dev(c, grad, sizeof(float) * NP, 4, "grad_dev")) != MMOC_OK) return st;
    mlp_state* S = c->mlp;
    const int ntiles = (int)(n / 64);
    if (S->part_tiles < ntiles) {
        if ((st = alloc(c, &S->part, (size_t)ntiles * (NP + 1), "partial gradients")) != MMOC_OK) return st;
        if ((st = alloc(c, &S->scratch, (size_t)ntiles * 5 * H * H, "training scratch")) != MMOC_OK) return st;
        S->part_tiles = ntiles;
    }
    if (S->losses_n < 1) {
        if ((st = alloc(c, &S->losses, 1, "losses")) != MMOC_OK) return st;
        S->losses_n = 1;
    }
    HIPCHK(c, launch_train_step(args_of(c), state_of(c, grad), in4, tg3, nullptr, 0, n, 1, n, S->part, S->scratch, 0.f,
                                1, S->losses, c->stream),
           "loss/gradient");
    if (loss) {
        float l;
        HIPCHK(c, hipMemcpyAsync(&l, S->losses, sizeof l, hipMemcpyDeviceToHost, c->stream), "loss");
        HIPCHK(c, hipStreamSynchronize(c->stream), "loss");
        *loss = l;
    }
    return MMOC_OK;
}

mmoc_status mmoc_mlp_infer(mmoc_ctx* c, double t_np1, double dt, double* X)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (!(dt > 0) || !std::isfinite(t_np1)) return fail(c, MMOC_E_ARG, "need dt > 0 and a finite t");
    if ((st = check_dev(c, X, sizeof(double) * 3 * c->N, 8, "X_dev")) != MMOC_OK) return st;
    mlp_state* S = c->mlp;
    if (S->pred_substeps > 0) {
        if ((st = need_velocity(c)) != MMOC_OK) return st;
        if ((st = run_predictor(c, dt, X)) != MMOC_OK) return st;
        HIPCHK(c, launch_infer(args_of(c), time_input(S, t_np1), S->corr_scale, X, 1, c->stream), "mlp inference");
    } else {
        HIPCHK(c, launch_infer(args_of(c), time_input(S, t_np1), dt * S->U, X, 0, c->stream), "mlp inference");
    }
    return MMOC_OK;
}

mmoc_status mmoc_mlp_set_predictor(mmoc_ctx* c, int substeps, double scale, double period)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (substeps < 0 || substeps > 64) return fail(c, MMOC_E_ARG, "predictor sub-steps must be in [0, 64]");
    if (substeps > 0 && !(scale > 0 && std::isfinite(scale))) return fail(c, MMOC_E_ARG, "need scale > 0");
    if (!(period >= 0 && std::isfinite(period))) return fail(c, MMOC_E_ARG, "need period >= 0");
    mlp_state* S = c->mlp;
    if (S->count > 0 && (substeps != S->pred_substeps || (substeps > 0 && scale != S->corr_scale) ||
                         period != S->period))
        return fail(c, MMOC_E_STATE, "training pairs were recorded with another predictor or time input");
    S->pred_substeps = substeps;
    S->corr_scale = substeps > 0 ? scale : 1.0;
    S->period = period;
    return MMOC_OK;
}

mmoc_status mmoc_trace_step_surrogate(mmoc_ctx* c, double t_np1, double dt, int substeps, float check_fraction,
                                      double tol, int64_t step, void* c_hat, double* X)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = need_mlp(c);
    if (st != MMOC_OK) return st;
    if (!X) return fail(c, MMOC_E_ARG, "X_dev is required by the surrogate step");
    if ((st = mmoc_check_step_args(c, dt, substeps, c_hat, X)) != MMOC_OK) return st;
    if (!(check_fraction >= 0.f && check_fraction <= 1.f)) return fail(c, MMOC_E_ARG, "check_fraction must be in [0, 1]");
    if (!(tol >= 0) || !std::isfinite(t_np1)) return fail(c, MMOC_E_ARG, "need tol >= 0 and a finite t");
    mlp_state* S = c->mlp;
    const int64_t N = c->N;
    if ((st = need_aux(c)) != MMOC_OK) return st;
    // 1. the seeded check sample (at least one per tile), selected on the
    //    context's stream before anything else: its blocks of 1,024 threads
    //    find no room beside a running trace kernel, and beside the
    //    predictor the selection took up to 3 ms instead of 0.1 ms
    HIPCHK(c, hipMemsetAsync(S->n_ids, 0, sizeof(unsigned long long), c->stream), "clear count");
    const uint64_t seed = 0x243F6A8885A308D3ull ^ ((uint64_t)step * 0x9E3779B97F4A7C15ull);
    // The list holds up to `cap` particles: twice the expected share plus one
    // per tile, so that the check trace launches a grid of that size
    // instead of one over all particles (a launch of mostly empty blocks
    // costs as much as the check itself at 1.7e7 particles).  A selection
    // beyond it is not traced and sends its tile to the fallback.
    const int64_t cap = std::min<int64_t>(
        N, 2 * (int64_t)std::ceil((double)check_fraction * (double)N) + (N + kTile - 1) / kTile + 1024);
    HIPCHK(c, launch_select_check(N, kTile, seed, check_fraction, S->ids, S->n_ids, cap, S->checked, c->stream),
           "check sample");
    // RK4 on the sample depends only on the fields and the list: it runs on
    // the auxiliary stream while the predictor and the network run on the
    // context's stream
    HIPCHK(c, hipEventRecord(S->ev_fork, c->stream), "fork");
    HIPCHK(c, hipStreamWaitEvent(S->aux, S->ev_fork, 0), "fork");
    TraceExtra on_aux;
    on_aux.stream = S->aux;
    if ((st = mmoc_launch_trace(c, dt, substeps, nullptr, S->Xrk, S->ids, cap, S->n_ids, 0, 1, &on_aux)) != MMOC_OK)
        return st;
    HIPCHK(c, hipEventRecord(S->ev_join, S->aux), "join");
    // 2. the surrogate's departure points for every particle: the network
    //    alone, or the predictor's trace plus the network's correction
    if (S->pred_substeps > 0) {
        if ((st = run_predictor(c, dt, X)) != MMOC_OK) return st;
        HIPCHK(c, launch_infer(args_of(c), time_input(S, t_np1), S->corr_scale, X, 1, c->stream), "mlp inference");
    } else {
        HIPCHK(c, launch_infer(args_of(c), time_input(S, t_np1), dt * S->U, X, 0, c->stream), "mlp inference");
    }
    HIPCHK(c, hipStreamWaitEvent(c->stream, S->ev_join, 0), "join");
    // 3. one pass over all particles, a block per tile: the tile's checked
    //    residuals |Xhat - X_rk4|_inf decide; above tol/2 the whole tile is
    //    traced by RK4 (fallback), otherwise it keeps Xhat (checked particles
    //    their RK4 result); then chat = c_h^n(X)
    TraceExtra finish;
    finish.checked = S->checked;
    finish.xcheck = S->Xrk;
    finish.tol_half = 0.5 * tol;
    return mmoc_launch_trace(c, dt, substeps, c_hat, X, nullptr, N, nullptr, 0, 1, &finish);
}

}  // extern "C"
