// mmoc_internal.h -- data layouts shared by the host side of the library and
// its HIP kernels.  Nothing here is part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmoc {

// Geometry of one macro element, 256 bytes, read by the kernels from an
// L2-resident table.  x = v0 + B s (computational domain), s = Binv (x - v0).
// For the radially blended shell, (pn, pc) is the plane n.x = c through the
// macro's three unit directions.  nbr[k]: macro across the face opposite
// local vertex k, -1 on the domain boundary.
struct alignas(16) MacroGeo {
    double v0[3];
    double binv[9];   // row-major
    double B[9];      // row-major
    double pn[3];
    double pc;
    int32_t nbr[4];
    float binvf[9];   // float copy of binv for the mixed-precision tracer
    float pad;
};
static_assert(sizeof(MacroGeo) == 256, "MacroGeo must stay 256 bytes");

// Particle table entry: owner macro and lattice coordinates of the DoF a
// thread traces.  bits 0-11 K, 12-23 J, 24-35 I, 36-63 macro.
__host__ __device__ inline uint64_t pack_owned(uint32_t M, uint32_t I, uint32_t J, uint32_t K)
{
    return ((uint64_t)M << 36) | ((uint64_t)I << 24) | ((uint64_t)J << 12) | (uint64_t)K;
}

// Statistic counters kept in device memory.  Each counter is a row of
// kStatSpread uint64 words; a block adds into word blockIdx % kStatSpread of
// the row, so that the per-wave atomics of thousands of waves finishing
// together do not queue on one address.  The host sums a row (max for
// ST_MAXRES_BITS) when it reads the statistics.
constexpr int kStatSpread = 64;
enum StatSlot {
    ST_PARTICLES = 0,
    ST_OUTSIDE,
    ST_MULTIHOP,
    ST_BRUTE,
    ST_TIEBAND,
    ST_NAN,
    ST_CHECKED,
    ST_FALLBACK,
    ST_MAXRES_BITS,  // max check residual, stored as the bits of a non-negative double
    ST_CACHE_LOOKUPS,  // stage evaluations that went through the element cache
    ST_CACHE_HITS,     // ... and found their element in it
    ST_COUNT
};

// Tile of the surrogate's check and fallback: 128 consecutive particles in
// unique order, which is one block of the trace kernels (the finish pass
// branches per block).
constexpr int kSurrogateTile = 128;

enum LaneFlag : unsigned {
    LF_OUTSIDE = 1u,
    LF_MULTIHOP = 2u,
    LF_BRUTE = 4u,
    LF_TIEBAND = 8u,
    LF_NAN = 16u,
    LF_FALLBACK = 32u,  // surrogate finish: re-traced because its tile failed the check
};

// Arguments of the trace kernels.  Fields live in per-component arrays over
// the block slots (slot = macro * npm + lattice index, macro-major, lattice
// nodes of a macro in lexicographic order), one set per velocity level (a
// ring of lev_cap levels, equally spaced in time; the stage times select the
// two levels around them):
//   3D float64: va = (u_x, u_y) pairs (16 B), vb = u_z (8 B)
//   3D float32: va = (u_x, u_y, u_z) triples (12 B), vb unused
//   2D        : va = (u_x, u_y) pairs, vb unused
//   cs        : the scalar c at t_n
// Small records keep the number of distinct cache lines per wave-level load
// low, which is what the gather throughput depends on.
// Butcher tableau of a general explicit Runge-Kutta method (s > 0), or the
// classical RK4 of the specialised path (s == 0).  a is row-major
// [kMaxStages][kMaxStages], strictly lower triangular.
constexpr int kMaxStages = 7;
struct RKTab {
    int s;
    double a[kMaxStages * kMaxStages];
    double b[kMaxStages];
    double c[kMaxStages];
};

template <typename T>
struct TraceArgs {
    const MacroGeo* geo;
    const uint64_t* owned;   // [n_unique] (macro, I, J, K) per DoF, unique order
    const int32_t* order;    // [n] unique ids in lane order, or null: lane t traces DoF t
    const unsigned long long* n_dev;  // if set: lanes t >= *n_dev do nothing (device-side count)
    const T* va;             // velocity ring, physical slot 0 (see lev_cap / rot / lsa / lsb)
    const T* vb;
    const T* cs;
    int64_t lsa, lsb;        // elements per velocity level in va / vb
    int zs;                  // vb elements per slot: 1, or 2 when the u_z of a two-level
                             // float64 ring are paired per slot (ring slot 0 first; lsb = 1)
    int lev_cap, rot;        // ring size and physical slot of logical level 0
    int first, n_int;        // trace from logical level first + n_int back to first
    int64_t n;               // particles traced by this launch (lanes)
    int64_t xstride;         // n_unique: stride of X and extent of c_hat
    int nm;                  // macros
    int npm;                 // lattice nodes per macro
    int nlev;                // 1 (stationary) or 2
    int level_n;             // micro edges per macro edge, 2^level
    int ord;                 // element order: 2 (P2) or 1 (P1)
    int lat_m;               // DoF lattice resolution, order * level_n
    int substeps;            // RK sub-steps per interval (dt = interval length)
    int max_hops;
    int xcd_log2;            // set by the launcher: log2 of the XCD run length in blocks, -1 contiguous eighths
    double dt;
    double eps_in;
    float eps32_macro;
    float eps32_micro;
    int elem_cache;          // 1: keep the last element's nodal velocities per lane in LDS
    // Surrogate finish (order must be null; a block is a tile of
    // kSurrogateTile particles): X holds the surrogate's departure points,
    // xcheck the RK4 ones of the particles with checked[pid] set.  A tile in
    // which some checked residual |X - xcheck|_inf exceeds tol_half is
    // traced (fallback); the others keep X (checked particles take xcheck)
    // and only get the scalar.
    const unsigned char* checked;
    const double* xcheck;
    double tol_half;
    T* c_hat;                // [n_unique] or null
    T* c_next;               // block-layout scalar of the next step: chat at each DoF's own slot, or null
    double* X;               // [dim][n_unique] or null
    unsigned long long* stats;
    RKTab rk;                // float64-arithmetic kernels only
};

// Launchers (kernels in mmoc_kernels.hip).  Each validates nothing: the host
// side checks every argument before calling them.
hipError_t launch_trace_fp64(int dim, int blend, const TraceArgs<double>& a, hipStream_t s);
// v[dup[2i + 1]] = v[dup[2i]] for i < ndup (interface slots from their owner's slot)
hipError_t launch_dup_fill(void* v, int fp32, const int32_t* dup, int64_t ndup, hipStream_t s);
hipError_t launch_trace_fp32(int dim, int blend, const TraceArgs<float>& a, hipStream_t s);
// float32 records, float64 arithmetic (MMOC_FP32_FIELDS)
hipError_t launch_trace_fp32_fields(int dim, int blend, const TraceArgs<float>& a, hipStream_t s);
// chat = c_h^n(X) for every particle, X given ([dim][n]); the walk starts in
// the particle's own macro (uses geo, owned, cs, n, nm, npm, level_n,
// max_hops, eps_in, eps32_*, c_hat, X (read), stats)
hipError_t launch_scalar_eval_fp64(int dim, int blend, const TraceArgs<double>& a, hipStream_t s);
hipError_t launch_scalar_eval_fp32(int dim, int blend, const TraceArgs<float>& a, hipStream_t s);
hipError_t launch_scalar_eval_fp32_fields(int dim, int blend, const TraceArgs<float>& a, hipStream_t s);
hipError_t launch_dof_coords(int dim, int blend, const MacroGeo* geo, const uint64_t* owned,
                             int64_t n, int lat_m, double* out, hipStream_t s);
// Copy of a unique-layout field into block slots: component i of DoF
// slot_uid[slot] goes to dst[i][slot * stride[i] + off[i]] (i < ncomp).
// Field ingestion: component i of the unique array src[i] (n_unique values)
// goes to record element dst[i][slot * stride[i] + off[i]] of every slot.
struct ScatterDst {
    const double* src[4];
    void* dst[4];
    int stride[4];
    int off[4];
};
hipError_t launch_scatter(int ncomp, const int32_t* slot_uid, int64_t nslots, int64_t n_unique, const ScatterDst& d,
                          int fp32, hipStream_t s);

// P2 mass matrix of a simplex of unit volume, nodes ordered as vertices
// 0..d then edges (a, b), a < b, lexicographic; entry (i, j) at m[i * NN + j]
struct MassRef {
    double m[100];
};
// blocks (partial sums) of one a^T M b launch
int64_t mass_inner_blocks(int dim, int nm, int n);
// The allocation-free mass inner product keeps its partial sums in a
// file-scope device array of this many doubles (512 KiB per GPU).
constexpr int64_t kNoAllocPartials = (int64_t)1 << 16;
// device address of that array on `device` (the current device)
hipError_t noalloc_scratch(int device, double** out);
// out[0] = (a - a_sub)^T M (b - b_sub) over the whole refined mesh (a null:
// ones; a_sub, b_sub null: zero); partial holds mass_inner_blocks doubles
hipError_t launch_mass_inner(int dim, int ord, const MacroGeo* geo, const int32_t* slot_uid, int64_t npm, int nm,
                             int n, const MassRef& R, const double* a, const double* a_sub, const double* b,
                             const double* b_sub, double* partial, double* out, hipStream_t s);
// out[0] = min c, out[1] = max c (NaNs skipped); partial holds 2 nblocks doubles
hipError_t launch_range(const double* c, int64_t n, double* partial, int64_t nblocks, double* out, hipStream_t s);
// out[0] = largest nodal speed of one velocity level in block slots (va
// records of `stride` components, the last component in vb, zs elements per
// slot, when vb is set); partial holds nblocks doubles
hipError_t launch_speed_max(const void* va, const void* vb, int zs, int fp32, int dim, int stride, int64_t nslots,
                            double* partial, int64_t nblocks, double* out, hipStream_t s);

}  // namespace mmoc
