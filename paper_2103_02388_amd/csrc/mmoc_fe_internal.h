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

// scalars of one conjugate-gradient solve, on the device
struct CgScalars {
    double rz;      // r . z (z = D^-1 r, or r without preconditioner)
    double pq;      // p . A p
    double alpha, beta;
    double rr;      // r . r
    double bb;      // b . b
    double thresh;  // stop when rr <= thresh
    int iters;
    int done;       // 1: converged, 2: breakdown (p . A p <= 0), 3: zero right-hand side
};

// element matrices: thread per (element, local row i); writes rows of the
// nb x nb mass and stiffness matrices of every element
hipError_t launch_element_matrices(int dim, int order, int blend, const MacroGeo* geo, const Elem* el, int64_t nel,
                                   int n, const QRule* rule, double* me, double* ae, hipStream_t s);
// CSR values: slot k sums elem[contrib[j]] for j in [cptr[k], cptr[k+1]) in order
hipError_t launch_gather(int64_t nnz, const int64_t* cptr, const int32_t* contrib, const double* me,
                         const double* ae, double* mv, double* av, hipStream_t s);
// E = M + s1 A with Dirichlet rows (is_dir) replaced by identity rows and
// Dirichlet columns of the other rows by zeros; dinv = 1 / diag(E) (or 1)
hipError_t launch_build_e(int64_t N, const int32_t* rp, const int32_t* ci, const double* mv, const double* av,
                          double s1, const uint8_t* is_dir, int precond, double* ev, double* dinv, hipStream_t s);
// y = V x for the CSR values V
hipError_t launch_spmv(int64_t N, const int32_t* rp, const int32_t* ci, const double* v, const double* x, double* y,
                       hipStream_t s);

struct RhsArgs {
    int64_t N;
    const int32_t* rp;
    const int32_t* ci;
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

struct CgArgs {
    int64_t N;
    const int32_t* rp;
    const int32_t* ci;
    const double* ev;
    const double* dinv;
    const double* b;
    double* x;
    double* r;
    double* p;
    double* q;
    double* part;            // 2 * kRedBlocks partial sums
    unsigned* ticket;        // block counter of the last-block reductions (0 between launches)
    CgScalars* sc;
    double rtol2;
    int max_iter;
};
constexpr int kRedBlocks = 1024;  // grid of the reducing kernels (grid-stride)
// r = b - E x, z = D^-1 r, p = z; rz, rr, bb; done when converged at start
hipError_t launch_cg_init(const CgArgs& a, hipStream_t s);
// one CG iteration as three kernels; each returns at once when sc->done
hipError_t launch_cg_iteration(const CgArgs& a, hipStream_t s);

}  // namespace fe
}  // namespace mmoc
