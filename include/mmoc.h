/*
 * mmoc.h -- C-ABI of the MI355X particle tracer for the modified method of
 * characteristics (MMOC) on block-structured P2 meshes.
 *
 * One call of mmoc_trace_step performs the Lagrangian part of one advection
 * time step (Alg. 1, departure-point and advection lines; Sec. 2.3.1 steps
 * (i)-(iii)):
 *   (i)   a particle is created at every P2 degree of freedom x_i (vertices
 *         and edge midpoints of the macro mesh refined `level` times);
 *   (ii)  it is traced backwards over [t_n, t_{n+1}] with RK4 (Sec. 3.1) in
 *         `substeps` sub-steps, the velocity being linear in time between the
 *         two levels u_h^n and u_h^{n+1} (eq. linear-interpolation), giving the
 *         departure point X_i (eq. departure-point);
 *   (iii) the scalar c_h^n is evaluated at X_i: chat_i = c_h^n(X_i)
 *         (eq. mmoc-approximation).
 * Every field evaluation locates the point first in a macro element, by a
 * walk from the macro of the previous evaluation, and then in a micro
 * element in O(1) (Sec. 2.3.2), and sums the P2 shape functions.
 *
 * Conventions
 *  - All functions return an mmoc_status; MMOC_OK == 0, errors are negative.
 *    On error nothing has been enqueued on the stream and mmoc_last_error()
 *    holds a one-line reason.  No C++ exception crosses this interface.
 *  - Device pointers ("_dev") must be device memory of the context's GPU,
 *    8-byte aligned for double and 4-byte aligned for float; the library
 *    checks both (hipPointerGetAttributes) and never frees caller memory.
 *  - All device work is enqueued on the stream given at creation (or by
 *    mmoc_set_stream); calls return before the work has finished.  Outputs
 *    are valid once that stream is synchronised.  mmoc_get_stats
 *    synchronises the stream.
 *  - A context is not thread-safe; use one context per host thread.
 *  - Unique DoF order ("unique layout"): macro-major, each DoF at its first
 *    occurrence; inside a macro, lattice nodes (I, J, K), m >= I >= J >= K
 *    >= 0, in lexicographic order, with m = 2^(level+1) for P2 and m =
 *    2^level for P1 (options.order).  A DoF on an interface
 *    belongs to the lowest-index macro that contains it (the paper leaves the
 *    choice open, Sec. 2.3.1 step (i)).  mmoc_dof_coords returns positions in
 *    this order.
 *  - Vector fields are structure-of-arrays [dim][n_unique] float64.
 */
#ifndef MMOC_H
#define MMOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mmoc_ctx mmoc_ctx; /* opaque; owned by the library */

typedef enum {
    MMOC_OK = 0,
    MMOC_E_ARG = -1,         /* invalid argument (null/misaligned/host pointer, size, value) */
    MMOC_E_MESH = -2,        /* invalid mesh (degenerate, non-manifold, non-conforming order) */
    MMOC_E_STATE = -3,       /* call out of order (e.g. trace before fields are set) */
    MMOC_E_HIP = -4,         /* HIP runtime error */
    MMOC_E_NOMEM = -5,       /* device allocation failed */
    MMOC_E_UNSUPPORTED = -6  /* combination not built (e.g. P1 on a blended mesh) */
} mmoc_status;

typedef enum {
    MMOC_FP64 = 0,        /* every stage in float64 */
    MMOC_FP32_MIXED = 1,  /* stages, location and interpolation in float32 on float32 field
                             copies; location decisions within eps of a macro or micro face
                             re-taken in float64; departure points accumulated in float64 */
    MMOC_FP32_FIELDS = 2  /* float32 field records (half the gather bytes of MMOC_FP64),
                             every operation in float64; chat is written as float32.  The
                             only error against float64 is the rounding of the stored
                             nodal values. */
} mmoc_precision;

typedef enum {
    MMOC_BLEND_NONE = 0,         /* physical domain = computational domain */
    MMOC_BLEND_SHELL_RADIAL = 1  /* radial blending of a spherical shell (3D) or an annulus
                                    (2D): each macro's column (the tips of its d unit
                                    directions span a plane, in 2D a line, n.x = c) is
                                    mapped radially, Phi(x) = x (n.x)/(c|x|) (Sec. 2.1
                                    blending function; Sec. 4 annulus) */
} mmoc_blend;

typedef struct {
    double eps_in;     /* macro acceptance: min barycentric >= -eps_in (default 1e-12) */
    float eps32_macro; /* FP32 path: macro decisions with |min lambda| < eps redone in FP64 (4e-6) */
    float eps32_micro; /* FP32 path: micro decisions with a sorted-coordinate gap < eps*n
                          redone in FP64 (default 2^-18: float32 rounding of the
                          lattice coordinates is about n * 1e-6).  0 turns the micro
                          band off: the P2 field is continuous across micro faces, so
                          a micro tie changes the value only by rounding, and
                          particles of a slow flow, which sit within float32 rounding
                          of a lattice node at every stage, are then not re-decided */
    int max_hops;      /* walk hops before brute-force location (default 64) */
    int order;         /* element order of the fields and DoFs: 2 = P2 (default; 0 also
                          means 2), 1 = P1, the micro vertices (Sec. 3.1: P1 and P2
                          Lagrange elements).  P1 is not built for blended meshes. */
    int elem_cache;    /* 1 (default): each lane keeps the nodal velocities of its last
                          micro element in LDS and gathers only when the element changes
                          (3D P2 RK4 traces over one interval: a stationary level, two
                          float32 levels, or the earlier of two float64 levels, whose
                          later level is gathered at every stage); 0: gather at every
                          stage.  Results are bitwise the same either way. */
    int keep_chat;     /* 1: every trace call that writes chat for all particles also
                          writes it into a second block-layout scalar array of the
                          library, which mmoc_use_last_chat then makes the scalar of
                          the next step (a time-stepping run then ingests no scalar;
                          allocates one more scalar array and the interface slot list
                          at mmoc_upload_mesh).  0 (default): off. */
    int reserved;
} mmoc_options;

typedef struct {
    int64_t n_particles;   /* particles traced since the last reset */
    int64_t n_outside;     /* particles with at least one evaluation outside the domain
                              (extrapolated from the boundary element) */
    int64_t n_multi_hop;   /* particles whose walk needed more than one hop at least once */
    int64_t n_bruteforce;  /* particles located by brute force at least once */
    int64_t n_tieband;     /* FP32 path: particles with at least one FP64 tie-break */
    int64_t n_nan;         /* particles with a NaN departure point or value */
    int64_t n_checked;     /* surrogate: particles re-traced by RK4 as the check sample */
    int64_t n_fallback;    /* surrogate: particles whose result came from the RK4 fallback */
    double max_check_residual; /* surrogate: largest |Xhat - X_rk4|_inf over the check sample */
    int64_t n_cache_lookups;   /* stage evaluations through the element cache */
    int64_t n_cache_hits;      /* ... of which found their element's values in it */
} mmoc_stats;

/* Fills *opt with the defaults listed above. */
void mmoc_default_options(mmoc_options* opt);

/* Creates a context for a mesh of dimension dim (2: triangles, 3: tetrahedra)
 * whose macros are refined `level` times (0..10 in 2D, 0..9 in 3D).  opt may be NULL
 * (defaults).  hip_stream is a hipStream_t (NULL: the null stream).  Selects
 * the current HIP device.  *out is NULL on failure. */
mmoc_status mmoc_create(mmoc_ctx** out, int dim, int level, mmoc_precision prec,
                        const mmoc_options* opt, void* hip_stream);

/* Changes the stream used by later calls. */
mmoc_status mmoc_set_stream(mmoc_ctx* ctx, void* hip_stream);

/* Uploads the coarse mesh (Sec. 2.1: the macro elements that are refined
 * uniformly; Sec. 2.3.1 grid data structure).  vertex_xyz: host [n_vertices][dim]
 * computational-domain coordinates; macro_vertices: host [n_macros][dim+1]
 * vertex ids.  Macros sharing a face must list the face's vertices in the same
 * relative order (this makes the refined meshes conform; ascending ids always
 * do).  Derives face neighbours, the unique DoF numbering and the per-macro
 * block layout, and uploads them.  May be called once per context.
 * Errors: MMOC_E_MESH for degenerate or non-manifold meshes or non-conforming
 * vertex orders or a blended macro that does not span exactly dim radial
 * directions, MMOC_E_UNSUPPORTED for P1 elements on a blended mesh. */
mmoc_status mmoc_upload_mesh(mmoc_ctx* ctx, int n_vertices, const double* vertex_xyz,
                             int n_macros, const int32_t* macro_vertices, mmoc_blend blend);

/* Number of unique DoFs (= particles) and of block-layout slots (duplicated
 * interface nodes included). */
mmoc_status mmoc_num_dofs(const mmoc_ctx* ctx, int64_t* n_unique, int64_t* n_block);

/* Writes the physical DoF positions x_i, SoA [dim][n_unique] float64, device
 * memory owned by the caller (Sec. 2.3.1 step (i)). */
mmoc_status mmoc_dof_coords(mmoc_ctx* ctx, double* xyz_dev);

/* Sets velocity level `level` from a unique-layout SoA [dim][n_unique]
 * float64 device array (eq. linear-interpolation).  With the default two
 * levels, level 0 is u_h^n at t_n and level 1 u_h^{n+1} at t_{n+1};
 * mmoc_set_level_count holds more (levels l at equally spaced times, l = 0
 * the oldest).  The values are copied into the library's block layout
 * (float32 for MMOC_FP32_MIXED and MMOC_FP32_FIELDS); the caller may free
 * u_dev once the stream has passed this call. */
mmoc_status mmoc_set_velocity(mmoc_ctx* ctx, int level, const double* u_dev);

/* on != 0: the velocity is stationary; only level 0 is used (setting level 1
 * is an MMOC_E_STATE error) and each stage evaluates one field.  Switching
 * back to two levels requires level 1 to be set again. */
mmoc_status mmoc_set_stationary(mmoc_ctx* ctx, int on);

/* Makes level l + 1 the new level l for every l (u^{n+1} becomes u^n for the
 * next step; the levels form a ring, nothing is copied).  The last level
 * must be set again before it is used; the scalar keeps its value until
 * mmoc_set_scalar is called. */
mmoc_status mmoc_swap_velocity_levels(mmoc_ctx* ctx);

/* Sets the scalar c_h^n from a unique-layout [n_unique] float64 device array
 * (copied into the block layout). */
mmoc_status mmoc_set_scalar(mmoc_ctx* ctx, const double* c_dev);

/* The scalar of the next step is the chat of the last trace call that wrote
 * chat for all particles (options.keep_chat = 1): the same block-layout
 * values mmoc_set_scalar(chat) would ingest, without the ingestion.  The
 * scalar array of the step before becomes the one the next trace writes.
 * MMOC_E_STATE if keep_chat is off or no such trace call ran since the last
 * mmoc_use_last_chat. */
mmoc_status mmoc_use_last_chat(mmoc_ctx* ctx);

/* mmoc_set_velocity(ctx, level, u_dev) and mmoc_set_scalar(ctx, c_dev) in
 * one pass over the block layout: the field ingestion of a time step
 * (Alg. 1: the new velocity level and the current scalar).  Same arguments,
 * layouts and errors as the two calls. */
mmoc_status mmoc_set_fields(mmoc_ctx* ctx, int level, const double* u_dev, const double* c_dev);

/* One MMOC advection step of length dt > 0 with substeps >= 1 RK4 sub-steps
 * (Alg. 1 departure-point and advection lines).  c_hat_dev receives
 * chat_i = c_h^n(X_i) in unique order: double* [n_unique] for MMOC_FP64,
 * float* [n_unique] for MMOC_FP32_MIXED and MMOC_FP32_FIELDS.  X_dev (may be
 * NULL) receives the departure points, SoA [dim][n_unique] float64 (physical coordinates).
 * Points that leave the domain are evaluated by extrapolating the boundary
 * element reached by the walk (counted in n_outside). */
mmoc_status mmoc_trace_step(mmoc_ctx* ctx, double dt, int substeps, void* c_hat_dev, double* X_dev);

/* Holds `levels` velocity levels (2..65536; default 2) for traces across
 * several time steps (look-back b > 1 with a time-dependent velocity,
 * Sec. 2.3.3).  Reallocates the levels: every level must be set again. */
mmoc_status mmoc_set_level_count(mmoc_ctx* ctx, int levels);

/* A trace across n_int >= 1 time steps of length dt (look-back, Sec.
 * 2.3.3): from the DoFs at the time of level first + n_int back to the time
 * of level `first`, with `substeps` RK sub-steps per step; the velocity is
 * linear in time between consecutive levels.  The scalar set by
 * mmoc_set_scalar is the field at the time of level `first`.  Levels
 * first .. first + n_int must be set.  Outputs as in mmoc_trace_step.  With
 * a stationary velocity (first must be 0) this is one trace of length
 * n_int * dt.  mmoc_trace_step(dt, S) is mmoc_trace_span(0, 1, dt, S). */
mmoc_status mmoc_trace_span(mmoc_ctx* ctx, int first, int n_int, double dt, int substeps, void* c_hat_dev,
                            double* X_dev);

/* Statistics accumulated since creation or the last reset; synchronises. */
mmoc_status mmoc_get_stats(mmoc_ctx* ctx, mmoc_stats* out);
mmoc_status mmoc_reset_stats(mmoc_ctx* ctx);

/* ---------------- integrator and time step (Sec. 3.1, Alg. 1) ------------- */

/* Selects a general explicit Runge-Kutta method for the trace (the paper
 * uses the classical RK4 and notes that any explicit RK method applies,
 * Sec. 3.1).  Host arrays: a [stages][stages] row-major (strictly lower
 * triangular, else MMOC_E_ARG), b [stages], c [stages] with c[0] == 0.
 * Sub-step j of S computes, backwards in time, y_i = Y - h sum_{l<i} a_il k_l,
 * k_i = u~(y_i) at theta_i = 1 - (j + c_i)/S (eq. linear-interpolation), and
 * Y <- Y - h sum_i b_i k_i.  1 <= stages <= 7; stages = 0 restores the
 * built-in classical RK4 (the fastest path).  MMOC_FP64 and MMOC_FP32_FIELDS
 * contexts only (MMOC_E_UNSUPPORTED for MMOC_FP32_MIXED). */
mmoc_status mmoc_set_rk_tableau(mmoc_ctx* ctx, int stages, const double* a, const double* b, const double* c);

/* CFL time step of Alg. 1: *tau = cfl * h_min / max_i |u_i|, with the
 * maximum over the nodal values of velocity level `level` (0 or 1) and
 * h_min the shortest micro edge of the refined mesh (in the computational
 * domain).  *umax and *hmin (each may be NULL) receive the two factors;
 * *tau is +inf for a zero field.  Synchronises the stream. */
mmoc_status mmoc_cfl_time_step(mmoc_ctx* ctx, double cfl, int level, double* tau, double* umax, double* hmin);

/* ---------------- benchmark measures and look-back (Sec. 2.3.3, 3.1) ------ */

/* Discrete H0 inner product with the P2 mass matrix M of the refined mesh
 * (the matrix of the H0 error norm and of the mass m(t) = 1^T M c, Sec. 3.1):
 * *out = (a - a_sub)^T M (b - b_sub).  All arrays are unique-layout
 * [n_unique] float64 device arrays; a or b = NULL stands for the vector of
 * ones, a_sub / b_sub = NULL for zero.  Exact for P2 functions on affine elements;
 * on a blended mesh M is the assembled quadrature mass matrix of
 * mmoc_fe_assemble (assembled at the first call).  Deterministic (fixed
 * summation order); synchronises the stream. */
mmoc_status mmoc_mass_inner(mmoc_ctx* ctx, const double* a_dev, const double* a_sub_dev, const double* b_dev,
                            const double* b_sub_dev, double* out);

/* mmoc_mass_inner for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, but the
 * partial sums live in a file-scope device array of the library (512 KiB per
 * GPU, held until the process ends) and the result goes to out_dev, one
 * float64 of caller-owned device memory.  Asynchronous on the context's
 * stream; allocates nothing, copies nothing to the host and does not
 * synchronise.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other contexts, other host threads)
 * race.  Errors: MMOC_E_UNSUPPORTED on blended meshes (their mass matrix is
 * the assembled one); MMOC_E_ARG for a mesh needing more than 65,536
 * partial sums (one per 256 micro cubes: the 6-tetrahedron cube up to level
 * 7) or bad buffers; MMOC_E_STATE before a mesh is uploaded. */
mmoc_status mmoc_mass_inner_noalloc(mmoc_ctx* ctx, const double* a_dev, const double* a_sub_dev,
                                    const double* b_dev, const double* b_sub_dev, double* out_dev);

/* Smallest and largest nodal value of a unique-layout [n_unique] float64
 * device array (var = max - min and the peak ratio of Sec. 3.1); NaNs are
 * skipped.  Synchronises the stream. */
mmoc_status mmoc_field_range(mmoc_ctx* ctx, const double* c_dev, double* min_out, double* max_out);

/* n_steps MMOC steps of length tau with look-back distance b (Sec. 2.3.3),
 * for a stationary velocity (mmoc_set_stationary(ctx, 1) and level 0 set)
 * and a float64 context.  Step n (1..n_steps) computes
 *   c^n = c^{n-b'}(X),  b' = min(b, n),
 * with X traced back over b' tau in b' * substeps RK4 sub-steps (substeps
 * per time step; 1 is one RK4 step per tau).  b <= 0 stands for b = infinity:
 * c^{n_steps} = c^0 at the point traced back over the whole interval, one
 * trace.  ring_dev: caller-owned float64 device array [ring_len][n_unique];
 * slot 0 holds c^0 on entry, c^j is kept in slot j % ring_len, and ring_len
 * must be at least min(b, n_steps) + 1 (1 for b = infinity).  c_out_dev
 * ([n_unique] float64, must not overlap other ring slots) receives
 * c^{n_steps}.  The scalar set on ctx is overwritten.  Asynchronous on the
 * context's stream. */
mmoc_status mmoc_lookback_run(mmoc_ctx* ctx, double tau, int substeps, int64_t n_steps, int64_t b,
                              double* ring_dev, int64_t ring_len, double* c_out_dev);

/* ---------------- learned flow-map surrogate (not part of the paper) -------
 * An MLP (x, t) -> scaled displacement, 4 -> 64 -> 64 -> 64 -> 3 with
 * tanh-form GELU (Hendrycks & Gimpel 2016), bf16 weights and activations,
 * fp32 accumulation on the matrix cores.  Inputs are affinely scaled to
 * [-1,1] (box [lo, hi] per input).  Without a predictor the output is the
 * whole displacement (X - x) / (dt * U); with a predictor
 * (mmoc_mlp_set_predictor) it is the correction (X - X_p) / scale to the
 * departure point X_p of the context's own RK4 tracer with fewer sub-steps.
 * Parameters are a flat float32 vector of mmoc_mlp_nparams() entries, layer
 * by layer: W1 [64][4], b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64],
 * W4 [3][64], b4 [3] (W[out][in]).  The surrogate is built for unblended 3D
 * meshes (MMOC_E_UNSUPPORTED otherwise). */

int64_t mmoc_mlp_nparams(void);

/* Input box: lo[4], hi[4] for (x, y, z, t); output scale U > 0 of the
 * whole-displacement form.  Allocates the surrogate's state (parameters
 * seeded, Adam moments zero) on the first call. */
mmoc_status mmoc_mlp_configure(mmoc_ctx* ctx, const double* lo, const double* hi, double U);

/* The predictor the network corrects and its time input.  substeps in
 * [1, 64]: X_p is the context's RK4 trace of the step with that many
 * sub-steps (the fields of the step must be set when recording, inferring
 * and stepping), and the network's output is (X - X_p) / scale, scale > 0
 * (a length).  substeps 0: no predictor (the default; scale is ignored).
 * period > 0: the time input is the phase t mod period (a velocity periodic
 * in time); 0: t itself (the default).  Must be set before the first pair
 * is recorded (MMOC_E_STATE if pairs were recorded with another setting). */
mmoc_status mmoc_mlp_set_predictor(mmoc_ctx* ctx, int substeps, double scale, double period);

/* Appends training pairs for the step just traced: the DoF positions with
 * time t_np1 as inputs and X_dev (SoA [dim][n_unique] float64, the step's
 * departure points, a step of length dt) as targets, expressed as the
 * network's output (with a predictor, the predictor is traced through the
 * context's current fields to form the correction).  Buffers up to
 * `capacity` pairs (set by the first call; library owned device memory). */
mmoc_status mmoc_mlp_record(mmoc_ctx* ctx, double t_np1, double dt, const double* X_dev,
                            int64_t capacity);

/* Trains on `n_samples` pairs drawn (seeded, with replacement) from the
 * recorded ones: `epochs` passes of n_samples/batch Adam steps (beta 0.9,
 * 0.999, eps 1e-8), learning rate cosine-decayed from lr to lr/100, MSE
 * loss.  Forward and backward run on the GPU (bf16 matrix cores, fp32
 * master weights and moments).  *final_loss receives the mean loss of the
 * last epoch (may be NULL); synchronises. */
mmoc_status mmoc_mlp_train(mmoc_ctx* ctx, int64_t n_samples, int epochs, int batch, float lr,
                           unsigned long long seed, double* final_loss);

/* The raw network on caller data: out_dev[n][3] = MLP(in_dev[n][4]) (inputs
 * already scaled), float32 device arrays. */
mmoc_status mmoc_mlp_forward(mmoc_ctx* ctx, const float* in_dev, int64_t n, float* out_dev);

/* Loss 1/(3n) sum |MLP(in) - target|^2 and its gradient with respect to the
 * parameters (grad_dev: float32 device array of mmoc_mlp_nparams() entries),
 * computed by the training kernels (n a multiple of 64); *loss may be NULL.
 * Synchronises. */
mmoc_status mmoc_mlp_loss_grad(mmoc_ctx* ctx, const float* in_dev, const float* target_dev, int64_t n,
                               float* grad_dev, double* loss);

/* Host float32 copies of the master parameters (set also clears the Adam
 * moments). */
mmoc_status mmoc_mlp_get_weights(mmoc_ctx* ctx, float* host_params, int64_t n);
mmoc_status mmoc_mlp_set_weights(mmoc_ctx* ctx, const float* host_params, int64_t n);

/* Surrogate departure points for all particles, written to X_dev (SoA
 * [dim][n_unique] float64): Xhat_i = x_i + dt U MLP(x_i, t_np1), or with a
 * predictor Xhat_i = X_p,i + scale MLP(x_i, t_np1). */
mmoc_status mmoc_mlp_infer(mmoc_ctx* ctx, double t_np1, double dt, double* X_dev);

/* Surrogate step.  The departure points of all particles come from the
 * network (mmoc_mlp_infer).  A seeded sample of about check_fraction of the
 * particles (a 32-bit hash of (step, i) below check_fraction * 2^32, with
 * at least one per tile of 128 consecutive particles) is re-traced by RK4
 * with `substeps` sub-steps by the context's own tracer and precision, on
 * the same fields (on a second stream, beside the network).  The sample
 * list holds 2 check_fraction n_unique + n_unique/128 + 1024 entries; a
 * selected particle beyond it is not traced and its tile falls back.
 * Every checked particle keeps
 * its RK4 result; every particle of a tile in which some checked residual
 * |Xhat - X_rk4|_inf exceeds tol/2 is re-traced by RK4 (fallback).  Then
 * chat = c_h^n(X) as in mmoc_trace_step.  c_hat_dev: double* for MMOC_FP64
 * contexts, float* otherwise.  step seeds the sample.  Statistics:
 * n_checked, n_fallback (unchecked particles of fallback tiles) and
 * max_check_residual; n_particles counts traced and evaluated lanes. */
mmoc_status mmoc_trace_step_surrogate(mmoc_ctx* ctx, double t_np1, double dt, int substeps,
                                      float check_fraction, double tol, int64_t step,
                                      void* c_hat_dev, double* X_dev);

/* Reason of the last failed call on ctx (valid until the next call). */
const char* mmoc_last_error(const mmoc_ctx* ctx);

/* Frees the context and all library-owned device memory (synchronises). */
void mmoc_destroy(mmoc_ctx* ctx);

/* ----------------------------------------------------------------------
 * Diffusion: the Theta-method step of Sec. 2.2 (eq. linear-system), the
 * diffusion line of Alg. 1.  Alg. 2 (Strang splitting) is two calls with
 * tau / 2 around the advection step.
 *
 * The Galerkin matrices M_ij = (phi_j, phi_i) and A_ij = (grad phi_j,
 * grad phi_i) over the physical domain are assembled on the device at the
 * first call that needs them (P2, or P1 for an order-1 context), in CSR form
 * over the unique DoFs.  Integrals are taken through the element map
 * Phi(affine micro simplex) with the collapsed Gauss rule of 4 points per
 * direction on the reference simplex: exact for the unblended P2 matrices,
 * and a quadrature of the smooth blended integrands otherwise.  The sums are
 * taken in a fixed order, so the matrices are bitwise reproducible.  All
 * vectors are float64 device arrays of N entries in the unique DoF order,
 * whatever the context's precision.
 * ---------------------------------------------------------------------- */
typedef enum { MMOC_MAT_MASS = 0, MMOC_MAT_STIFFNESS = 1 } mmoc_matrix;

/* Assembles M and A now (otherwise done by the first call below that needs
 * them); *nnz (optional) receives the number of stored entries per matrix.
 * Synchronises the stream.  Errors: MMOC_E_STATE before a mesh is uploaded,
 * MMOC_E_UNSUPPORTED for meshes beyond 32-bit CSR indices. */
mmoc_status mmoc_fe_assemble(mmoc_ctx* ctx, int64_t* nnz);

/* Copies one matrix to host memory: row_ptr [N+1] (int64), cols [nnz]
 * (ascending within each row) and vals [nnz]; each pointer may be NULL to
 * skip it.  Synchronises the stream. */
mmoc_status mmoc_fe_export(mmoc_ctx* ctx, mmoc_matrix which, int64_t* row_ptr, int32_t* cols, double* vals);

/* y = M x or y = A x (device float64 [N]; x and y must not alias).
 * Enqueued on the context's stream. */
mmoc_status mmoc_fe_apply(mmoc_ctx* ctx, mmoc_matrix which, const double* x, double* y);

/* Host uint8 [N]: 1 for DoFs on the domain boundary (lattice nodes of macro
 * faces without a neighbour), 0 elsewhere.  This is the Dirichlet set of
 * mmoc_diffusion_step (Sec. 2.2: V_h^D). */
mmoc_status mmoc_boundary_mask(mmoc_ctx* ctx, uint8_t* mask);

typedef struct {
    double theta;             /* Theta in [0, 1]: 1 implicit Euler, 0.5 Crank-Nicolson */
    double tau;               /* time step > 0 */
    double kappa;             /* diffusivity >= 0 */
    const double* q0;         /* device [N] load vector (q(t_n), phi_i), or NULL: zero */
    const double* q1;         /* device [N] load vector (q(t_{n+1}), phi_i), or NULL: zero */
    const double* dirichlet;  /* device [N]: values c_Gamma(t_{n+1}) at the boundary DoFs (other
                                 entries are not read), or NULL: homogeneous Neumann everywhere */
    double rtol;              /* CG stops at ||r||_2 <= rtol ||b||_2 (0: 1e-12) */
    int max_iter;             /* CG iteration limit (0: 1000) */
    int precond;              /* 0: plain CG, 1: Jacobi (diagonal) preconditioned CG */
} mmoc_diffusion_args;

typedef struct {
    int iterations;       /* CG iterations taken */
    int converged;        /* 1 when the tolerance was met (or the right-hand side is zero) */
    double rel_residual;  /* ||r||_2 / ||b||_2 of the last iterate (recursive residual) */
} mmoc_diffusion_info;

/* One diffusion step (Sec. 2.2, eq. linear-system): solves
 *   (M + tau Theta kappa A) c = (M - tau (1 - Theta) kappa A) c_hat
 *                               + tau (Theta q1 + (1 - Theta) q0)
 * for c_out by conjugate gradients (the matrix is symmetric positive
 * definite), starting from c_hat.  With `dirichlet` given, the boundary DoFs
 * take those values, their rows become identity rows and their known values
 * move to the right-hand side of the other rows.  c_hat and c_out: device
 * float64 [N]; c_out must not alias any input.  The call synchronises the stream once per batch
 * of iterations to read the convergence state; not converging within
 * max_iter is reported in *info (optional), not as an error.
 * Errors: MMOC_E_ARG for theta outside [0, 1], tau <= 0, kappa < 0,
 * non-finite values or bad buffers; MMOC_E_STATE before a mesh. */
mmoc_status mmoc_diffusion_step(mmoc_ctx* ctx, const mmoc_diffusion_args* args, const double* c_hat,
                                double* c_out, mmoc_diffusion_info* info);

#ifdef __cplusplus
}
#endif

#endif /* MMOC_H */
