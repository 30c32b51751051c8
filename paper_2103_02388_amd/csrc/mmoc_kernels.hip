// mmoc_kernels.hip -- helper kernels of the MMOC tracer: DoF positions and
// the copy of unique-layout fields into the per-macro block records.
#include "mmoc_internal.h"

#include <math.h>

namespace mmoc {
namespace {

constexpr int kBlock = 256;

// physical position of lattice node (I, J, K) of macro M: Phi(v0 + B s),
// s = (I - J, J - K, K) / m (Sec. 2.3.1 step (i))
template <int DIM, int BLEND>
__global__ __launch_bounds__(kBlock) void dof_coords_kernel(const MacroGeo* __restrict__ geo,
                                                            const uint64_t* __restrict__ owned, int64_t n,
                                                            int lat_m, double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const uint64_t e = owned[t];
    const int M = (int)(e >> 36);
    const int I = (int)((e >> 24) & 0xfffu), J = (int)((e >> 12) & 0xfffu), K = (int)(e & 0xfffu);
    const double invm = 1.0 / (double)lat_m;
    double s[3];
    if constexpr (DIM == 2) {
        s[0] = (double)(I - J) * invm;
        s[1] = (double)J * invm;
    } else {
        s[0] = (double)(I - J) * invm;
        s[1] = (double)(J - K) * invm;
        s[2] = (double)K * invm;
    }
    const MacroGeo& G = geo[M];
    double p[3];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        double acc = G.v0[i];
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc = fma(G.B[i * 3 + a], s[a], acc);
        p[i] = acc;
    }
    double f = 1.0;
    if constexpr (BLEND) {
        double nx = G.pn[0] * p[0] + G.pn[1] * p[1], r2 = p[0] * p[0] + p[1] * p[1];
        if constexpr (DIM == 3) {
            nx += G.pn[2] * p[2];
            r2 += p[2] * p[2];
        }
        f = nx / (G.pc * sqrt(r2));
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) out[(int64_t)i * n + t] = BLEND ? p[i] * f : p[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scatter_kernel(int ncomp, const int32_t* __restrict__ slot_uid,
                                                         int64_t nslots, int64_t nu, ScatterDst d)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= nslots) return;
    const int64_t q = slot_uid[t];
    for (int i = 0; i < ncomp; ++i) static_cast<T*>(d.dst[i])[t * d.stride[i] + d.off[i]] = (T)d.src[i][q];
    (void)nu;
}

// interface slots of the next step's scalar from their owners' slots
template <typename T>
__global__ __launch_bounds__(kBlock) void dup_fill_kernel(T* __restrict__ v, const int2* __restrict__ dup, int64_t ndup)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= ndup) return;
    const int2 p = dup[t];
    v[p.y] = v[p.x];
}

inline unsigned grid_plain(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_dof_coords(int dim, int blend, const MacroGeo* geo, const uint64_t* owned, int64_t n,
                             int lat_m, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const dim3 grid(grid_plain(n)), block(kBlock);
    if (dim == 2 && !blend) dof_coords_kernel<2, 0><<<grid, block, 0, s>>>(geo, owned, n, lat_m, out);
    else if (dim == 2) dof_coords_kernel<2, 1><<<grid, block, 0, s>>>(geo, owned, n, lat_m, out);
    else if (!blend) dof_coords_kernel<3, 0><<<grid, block, 0, s>>>(geo, owned, n, lat_m, out);
    else dof_coords_kernel<3, 1><<<grid, block, 0, s>>>(geo, owned, n, lat_m, out);
    return hipGetLastError();
}

hipError_t launch_dup_fill(void* v, int fp32, const int32_t* dup, int64_t ndup, hipStream_t s)
{
    if (ndup <= 0) return hipSuccess;
    const int2* p = reinterpret_cast<const int2*>(dup);
    if (fp32) dup_fill_kernel<float><<<grid_plain(ndup), kBlock, 0, s>>>(static_cast<float*>(v), p, ndup);
    else dup_fill_kernel<double><<<grid_plain(ndup), kBlock, 0, s>>>(static_cast<double*>(v), p, ndup);
    return hipGetLastError();
}

hipError_t launch_scatter(int ncomp, const int32_t* slot_uid, int64_t nslots, int64_t n_unique, const ScatterDst& d,
                          int fp32, hipStream_t s)
{
    if (nslots <= 0) return hipSuccess;
    if (ncomp < 1 || ncomp > 4) return hipErrorInvalidValue;
    const dim3 grid(grid_plain(nslots)), block(kBlock);
    if (fp32) scatter_kernel<float><<<grid, block, 0, s>>>(ncomp, slot_uid, nslots, n_unique, d);
    else scatter_kernel<double><<<grid, block, 0, s>>>(ncomp, slot_uid, nslots, n_unique, d);
    return hipGetLastError();
}

}  // namespace mmoc
