// mmoc_ctx.h -- the library context and host helpers shared by the
// library's translation units (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mmoc.h"
#include "mmoc_internal.h"

struct mlp_state;
struct fe_state;

struct mmoc_ctx {
    int dim = 0, level = 0, n = 0, m = 0;
    mmoc_precision prec = MMOC_FP64;
    mmoc_options opt{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;

    bool mesh_ok = false;
    int blend = 0;
    int nm = 0;
    int64_t npm = 0, nslots = 0, N = 0;
    mmoc::MacroGeo* geo_d = nullptr;
    uint64_t* owned_d = nullptr;     // unique order
    int32_t* slot_uid_d = nullptr;
    // velocity levels, a ring of lev_cap: logical level l (l = 0 the oldest
    // time) lives in physical slot (rot + l) % lev_cap; slot q of va_all
    // starts at element q * va_lstride
    void* va_all = nullptr;  // (u_x,u_y) pairs, or (u_x,u_y,u_z) triples (3D float32)
    void* vb_all = nullptr;  // u_z (3D float64)
    int64_t va_lstride = 0, vb_lstride = 0;
    // vb_all elements per slot: 2 for a two-level float64 3D ring, whose u_z
    // values are paired per slot (ring slot 0, ring slot 1; vb_lstride = 1),
    // so that a gather loads both levels' u_z at once; otherwise 1
    int zs = 1;
    int lev_cap = 2;
    int rot = 0;
    void* cs_d = nullptr;                // scalar
    // options.keep_chat: the next step's scalar written by the trace (own
    // slots) and completed from the interface slot list (owner slot, slot)
    void* cs_next = nullptr;
    int32_t* dup_d = nullptr;
    int64_t ndup = 0;
    bool chat_ready = false;
    std::vector<char> vel_set = std::vector<char>(2, 0);  // per logical level
    bool scalar_set = false;
    bool stationary = false;
    unsigned long long* stats_d = nullptr;
    double hmin = 0.0;        // shortest micro edge (computational domain)
    mmoc::RKTab rk{};         // general explicit RK tableau (s == 0: classical RK4)
    double* red_d = nullptr;  // partial sums of the metric reductions, red_cap doubles
    int64_t red_cap = 0;
    double* noalloc_d = nullptr;  // this device's allocation-free scratch (not owned)

    std::vector<mmoc::MacroGeo> geo_h;  // host copy of the geometry table

    mlp_state* mlp = nullptr;
    fe_state* fe = nullptr;
};


mmoc_status fail(mmoc_ctx* c, mmoc_status st, const char* fmt, ...);
mmoc_status hip_fail(mmoc_ctx* c, hipError_t e, const char* what);
mmoc_status check_dev(mmoc_ctx* c, const void* p, size_t bytes, size_t align, const char* name);
// validates the arguments of a trace step (fields set, dt, substeps, outputs)
mmoc_status mmoc_check_step_args(mmoc_ctx* c, double dt, int substeps, void* c_hat, double* X);
// launches the RK4 tracer on the particles order[0..n) (order null: all, lane t
// traces DoF t); n_dev (optional) is a device-side count that bounds the lanes
// Each particle is traced from logical velocity level first + n_int back to
// level first, n_int intervals of length dt with `substeps` RK sub-steps each.
// Optional launch settings: the stream (null: the context's) and the
// surrogate finish (TraceArgs::checked / xcheck / tol_half).
struct TraceExtra {
    hipStream_t stream = nullptr;
    const unsigned char* checked = nullptr;
    const double* xcheck = nullptr;
    double tol_half = 0.0;
};
mmoc_status mmoc_launch_trace(mmoc_ctx* c, double dt, int substeps, void* c_hat, double* X, const int32_t* order,
                              int64_t n, const unsigned long long* n_dev = nullptr, int first = 0, int n_int = 1,
                              const TraceExtra* ex = nullptr);
// physical ring slot of logical velocity level l
inline int phys_level(const mmoc_ctx* c, int l) { return (c->rot + l) % c->lev_cap; }
void mmoc_mlp_free_state(mmoc_ctx* c);
void mmoc_fe_free_state(mmoc_ctx* c);
// (a - a_sub)^T M (b - b_sub) with the assembled (quadrature) mass matrix
mmoc_status mmoc_fe_mass_quadform(mmoc_ctx* c, const double* a, const double* a_sub, const double* b,
                                  const double* b_sub, double* out);
// lattice node (I, J, K), m >= I >= J >= K >= 0, in lexicographic order
int64_t mmoc_lattice_index(int dim, int64_t I, int64_t J, int64_t K);

#define HIPCHK(ctx, call, what)                                \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what);  \
    } while (0)
