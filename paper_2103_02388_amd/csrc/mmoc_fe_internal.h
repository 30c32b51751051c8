// mmoc_fe_internal.h -- layouts shared by the host code and the kernels of
// the finite-element operators and the diffusion solve (not part of the
// public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mmoc_internal.h"

namespace mmoc {
namespace fe {

// quadrature rule on the reference simplex {xi >= 0, sum xi <= 1}
constexpr int kMaxQ = 64;
struct QRule {
    int nq;
    double pt[kMaxQ][3];
    double w[kMaxQ];
};

// micro simplex: its macro and the n-lattice coordinates (I, J, K) of its
// d + 1 vertices (Kuhn coordinates of the macro, n >= I >= J >= K >= 0)
struct alignas(8) Elem {
    int32_t macro;
    int16_t v[4][3];
};

// scalars of one conjugate-gradient solve, on the device (written by the
// first block of the reducing kernels, for the host)
struct CgScalars {
    double alpha[2];  // step length of the last two iterations (by parity)
    double beta;
    double rr;        // r . r of the last tested iterate
    double bb;        // b . b
    double thresh;    // stop when rr <= thresh
    int iters;        // updates applied to x
    int done;         // 1: converged, 2: breakdown (step not positive), 3: zero right-hand side
};

// element matrices: thread per (element, local row i); writes rows of the
// nb x nb mass and stiffness matrices of every element
hipError_t launch_element_matrices(int dim, int order, int blend, const MacroGeo* geo, const Elem* el, int64_t nel,
                                   int n, const QRule* rule, double* me, double* ae, hipStream_t s);
// CSR values: slot k sums elem[contrib[j]] for j in [cptr[k], cptr[k+1]) in order
hipError_t launch_gather(int64_t nnz, const int64_t* cptr, const int32_t* contrib, const double* me,
                         const double* ae, double* mv, double* av, hipStream_t s);
// CSR matrix with its row blocks: block b holds rows [rb[b], rb[b+1]), at
// most kRowsPerBlock rows whose entries fit the kLds staging buffer
constexpr int kRowsPerBlock = 256;
constexpr int kLds = 4096;
constexpr int kMaxRedBlocks = 1024;  // grid of the reducing kernels (row blocks strided over it)
struct Csr {
    int64_t N;
    int64_t nrb;     // row blocks
    const int32_t* rp;
    const int32_t* ci;
    const int4* rb;  // per row block: first row, end row, first entry, end entry
};

// E = M + s1 A with Dirichlet rows (is_dir) replaced by identity rows and
// Dirichlet columns of the other rows by zeros; dinv = 1 / diag(E) (or 1)
hipError_t launch_build_e(int64_t N, const int32_t* rp, const int32_t* ci, const double* mv, const double* av,
                          double s1, const uint8_t* is_dir, int precond, double* ev, double* dinv, hipStream_t s);
// y = V x for the CSR values V
hipError_t launch_spmv(const Csr& A, const double* v, const double* x, double* y, hipStream_t s);

struct RhsArgs {
    Csr A;
    const double* mv;
    const double* av;
    double s1, s2;      // tau Theta kappa, tau (1 - Theta) kappa
    double w0, w1;      // tau (1 - Theta), tau Theta: weights of q0, q1
    const double* chat;
    const double* q0;   // or null
    const double* q1;   // or null
    const double* g;    // Dirichlet values, or null
    const uint8_t* is_dir;
    double* b;
    double* x;
};
// right-hand side b (Dirichlet values lifted) and the initial iterate x
hipError_t launch_rhs(const RhsArgs& a, hipStream_t s);

// (a - a_sub)^T V (b - b_sub) for the CSR values V (a, b null: ones; a_sub,
// b_sub null: zero): per-block partials into part[0..G), then their sum in
// block order into *out
hipError_t launch_quadform(const Csr& A, const double* v, const double* a, const double* a_sub, const double* b,
                           const double* b_sub, double* part, double* out, hipStream_t s);

// partial sums, part[slot * kMaxRedBlocks + block]: gamma = r.u by
// iteration parity, delta = w.u, r.r, b.b
enum { P_G0 = 0, P_G1 = 1, P_DE = 2, P_RR = 3, P_BB = 4, P_SLOTS = 5 };
struct CgArgs {
    Csr A;
    const double* ev;
    const double* dinv;
    const double* b;
    double* x;
    double* r;
    double* u;  // D^-1 r
    double* w;  // E u
    double* p;
    double* s;  // E p
    double* part;  // P_SLOTS * kMaxRedBlocks
    CgScalars* sc;
    double rtol2;
};
// r = b - E x, u = D^-1 r; r.r, b.b; then the stop threshold
hipError_t launch_cg_init(const CgArgs& a, hipStream_t s);
// iteration k of CG as two kernels (w = E u with the inner products; the
// stop test, the step scalars and the vector updates), each returning at
// once when the solve has stopped.  Every block sums the partials of the
// kernel before it in the same fixed order, so no atomics are needed and
// every block takes the same decisions.
hipError_t launch_cg_iteration(const CgArgs& a, int k, hipStream_t s);

}  // namespace fe
}  // namespace mmoc
