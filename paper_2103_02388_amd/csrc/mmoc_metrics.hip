// mmoc_metrics.hip -- the accuracy measures of the paper's benchmarks
// (Sec. 3.1) on the GPU: the discrete H0 inner product a^T M b with the P2
// (or P1) mass matrix M of the refined mesh, and the range (min, max) of a
// nodal field.  Both reduce in two passes with a fixed summation order, so a result
// does not depend on the schedule.
//
// The mass matrix is assembled on the fly, one micro simplex at a time: a
// thread takes one cube k (n-1 >= k1 >= k2 >= k3 >= 0) of a macro's Kuhn
// lattice and visits the Freudenthal simplices of that cube that lie inside
// the macro (vertices V_0 = k, V_a = V_{a-1} + e_{pi(a)}, all with
// n >= V_1 >= V_2 >= V_3 >= 0).  Together they tile the macro with n^d
// simplices of volume |det B| / (d! n^d).  Nodal values are read from the
// caller's unique arrays through the slot -> unique-id table.
#include "mmoc_internal.h"

#include <math.h>

#include <mutex>

// Partial sums of the allocation-free mass inner product
// (mmoc_mass_inner_noalloc): one array per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel (in host code it
// is a stand-in, not a device address): it uses the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
static __device__ __align__(256) double scratch[mmoc::kNoAllocPartials];

namespace mmoc {
namespace {

constexpr int kMB = 256;

__device__ __forceinline__ int64_t tri64(int64_t x) { return x * (x + 1) / 2; }
__device__ __forceinline__ int64_t tet64(int64_t x) { return x * (x + 1) * (x + 2) / 6; }

// q -> (k1 >= k2 >= k3 >= 0) with q = tet(k1) + tri(k2) + k3
__device__ __forceinline__ void decode3(int64_t q, int* k)
{
    int64_t a = (int64_t)cbrt(6.0 * (double)q);
    while (a > 0 && tet64(a) > q) --a;
    while (tet64(a + 1) <= q) ++a;
    const int64_t r = q - tet64(a);
    int64_t b = (int64_t)((sqrt(8.0 * (double)r + 1.0) - 1.0) * 0.5);
    while (b > 0 && tri64(b) > r) --b;
    while (tri64(b + 1) <= r) ++b;
    k[0] = (int)a;
    k[1] = (int)b;
    k[2] = (int)(r - tri64(b));
}

// q -> (k1 >= k2 >= 0) with q = tri(k1) + k2
__device__ __forceinline__ void decode2(int64_t q, int* k)
{
    int64_t a = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    while (a > 0 && tri64(a) > q) --a;
    while (tri64(a + 1) <= q) ++a;
    k[0] = (int)a;
    k[1] = (int)(q - tri64(a));
    k[2] = 0;
}

__device__ __forceinline__ double nodal(const double* __restrict__ a, const double* __restrict__ a_sub, int64_t u)
{
    const double v = a ? a[u] : 1.0;
    return a_sub ? v - a_sub[u] : v;
}

// sum over the wave, then over the waves of the block, in a fixed order
__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

template <int DIM, int ORD>
__global__ __launch_bounds__(kMB) void mass_inner_kernel(const MacroGeo* __restrict__ geo,
                                                         const int32_t* __restrict__ slot_uid, int64_t npm, int n,
                                                         int64_t cubes_per_macro, int64_t total, MassRef R,
                                                         const double* __restrict__ a, const double* __restrict__ a_sub,
                                                         const double* __restrict__ b, const double* __restrict__ b_sub,
                                                         double* __restrict__ partial)
{
    constexpr int NV = DIM + 1;
    constexpr int NN = ORD == 2 ? (DIM + 1) * (DIM + 2) / 2 : DIM + 1;
    __shared__ double sh[kMB / 64];
    const int64_t t = (int64_t)blockIdx.x * kMB + threadIdx.x;
    double acc = 0.0;
    if (t < total) {
        const int M = (int)(t / cubes_per_macro);
        const int64_t q = t - (int64_t)M * cubes_per_macro;
        int k[3];
        if constexpr (DIM == 3) decode3(q, k);
        else decode2(q, k);
        const MacroGeo& G = geo[M];
        double det;
        if constexpr (DIM == 3) {
            const double* B = G.B;
            det = B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
                  B[2] * (B[3] * B[7] - B[4] * B[6]);
        } else {
            det = G.B[0] * G.B[4] - G.B[1] * G.B[3];
        }
        double vol = fabs(det);
        for (int i = 0; i < DIM; ++i) vol /= (double)((i + 1) * n);
        const int64_t base = (int64_t)M * npm;
        // the d! axis orders of the cube
        constexpr int NP = DIM == 3 ? 6 : 2;
        const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        for (int p = 0; p < NP; ++p) {
            int V[NV][3];
            for (int i = 0; i < 3; ++i) V[0][i] = k[i];
            bool ok = true;
            for (int s = 1; s < NV; ++s) {
                for (int i = 0; i < 3; ++i) V[s][i] = V[s - 1][i];
                V[s][DIM == 3 ? perm3[p][s - 1] : (p == 0 ? s - 1 : 2 - s)] += 1;
                ok &= V[s][0] <= n && V[s][0] >= V[s][1];
                if constexpr (DIM == 3) ok &= V[s][1] >= V[s][2];
            }
            if (!ok) continue;
            double av[NN], bv[NN];
            int c = 0;
            // P2 nodes V_a + V_b on the 2n-lattice; P1 nodes V_a on the n-lattice
            auto load = [&](int A, int Bn) {
                const int I = ORD == 2 ? V[A][0] + V[Bn][0] : V[A][0];
                const int J = ORD == 2 ? V[A][1] + V[Bn][1] : V[A][1];
                const int K = ORD == 2 ? V[A][2] + V[Bn][2] : V[A][2];
                const int64_t idx = DIM == 3 ? tet64(I) + tri64(J) + K : tri64(I) + J;
                const int64_t u = slot_uid[base + idx];
                av[c] = nodal(a, a_sub, u);
                bv[c] = nodal(b, b_sub, u);
                ++c;
            };
            for (int s = 0; s < NV; ++s) load(s, s);
            if constexpr (ORD == 2)
                for (int s = 0; s < NV; ++s)
                    for (int r = s + 1; r < NV; ++r) load(s, r);
            double quad = 0.0;
            for (int i = 0; i < NN; ++i) {
                double row = 0.0;
                for (int j = 0; j < NN; ++j) row = fma(R.m[i * NN + j], bv[j], row);
                quad = fma(av[i], row, quad);
            }
            acc = fma(vol, quad, acc);
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// fixed-order sum of count partials into out[0]
__global__ __launch_bounds__(kMB) void sum_partials_kernel(const double* __restrict__ partial, int64_t count,
                                                           double* __restrict__ out)
{
    __shared__ double sh[kMB / 64];
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kMB) v += partial[i];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) out[0] = s;
}

// per-block min and max of c (grid-stride); NaNs are skipped
__global__ __launch_bounds__(kMB) void range_kernel(const double* __restrict__ c, int64_t n,
                                                    double* __restrict__ pmin, double* __restrict__ pmax)
{
    __shared__ double smin[kMB / 64], smax[kMB / 64];
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * kMB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kMB) {
        const double v = c[i];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_down(lo, off, 64));
        hi = fmax(hi, __shfl_down(hi, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[w] = lo;
        smax[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kMB / 64; ++i) {
            lo = fmin(lo, smin[i]);
            hi = fmax(hi, smax[i]);
        }
        pmin[blockIdx.x] = lo;
        pmax[blockIdx.x] = hi;
    }
}

__global__ __launch_bounds__(64) void range_final_kernel(const double* __restrict__ pmin,
                                                         const double* __restrict__ pmax, int64_t count,
                                                         double* __restrict__ out)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = threadIdx.x; i < count; i += 64) {
        lo = fmin(lo, pmin[i]);
        hi = fmax(hi, pmax[i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_down(lo, off, 64));
        hi = fmax(hi, __shfl_down(hi, off, 64));
    }
    if (threadIdx.x == 0) {
        out[0] = lo;
        out[1] = hi;
    }
}

// per-block largest nodal speed |u| of one velocity level stored in block
// slots: (x, y) pairs in va (stride 2) with z in vb (zs elements per slot),
// or (x, y, z) triples in va (stride 3) with vb null
template <typename T>
__global__ __launch_bounds__(kMB) void speed_max_kernel(const T* __restrict__ va, const T* __restrict__ vb, int zs,
                                                        int dim, int stride, int64_t nslots,
                                                        double* __restrict__ pmax)
{
    __shared__ double sh[kMB / 64];
    double hi = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kMB + threadIdx.x; q < nslots; q += (int64_t)gridDim.x * kMB) {
        double s2 = 0.0;
        for (int i = 0; i < (vb ? 2 : dim); ++i) {
            const double v = (double)va[q * stride + i];
            s2 += v * v;
        }
        if (vb) {
            const double v = (double)vb[q * zs];
            s2 += v * v;
        }
        hi = fmax(hi, s2);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) hi = fmax(hi, __shfl_down(hi, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kMB / 64; ++i) hi = fmax(hi, sh[i]);
        pmax[blockIdx.x] = hi;
    }
}

__global__ __launch_bounds__(64) void max_final_kernel(const double* __restrict__ p, int64_t count,
                                                       double* __restrict__ out)
{
    double hi = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 64) hi = fmax(hi, p[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) hi = fmax(hi, __shfl_down(hi, off, 64));
    if (threadIdx.x == 0) out[0] = sqrt(hi);
}

}  // namespace

hipError_t launch_speed_max(const void* va, const void* vb, int zs, int fp32, int dim, int stride, int64_t nslots,
                            double* partial, int64_t nblocks, double* out, hipStream_t s)
{
    if (fp32)
        speed_max_kernel<float><<<(unsigned)nblocks, kMB, 0, s>>>((const float*)va, (const float*)vb, zs, dim,
                                                                  stride, nslots, partial);
    else
        speed_max_kernel<double><<<(unsigned)nblocks, kMB, 0, s>>>((const double*)va, (const double*)vb, zs, dim,
                                                                   stride, nslots, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    max_final_kernel<<<1, 64, 0, s>>>(partial, nblocks, out);
    return hipGetLastError();
}

int64_t mass_inner_blocks(int dim, int nm, int n)
{
    const int64_t cubes = dim == 3 ? (int64_t)n * (n + 1) * (n + 2) / 6 : (int64_t)n * (n + 1) / 2;
    return ((int64_t)nm * cubes + kMB - 1) / kMB;
}

hipError_t launch_mass_inner(int dim, int ord, const MacroGeo* geo, const int32_t* slot_uid, int64_t npm, int nm,
                             int n, const MassRef& R, const double* a, const double* a_sub, const double* b,
                             const double* b_sub, double* partial, double* out, hipStream_t s)
{
    const int64_t cubes = dim == 3 ? (int64_t)n * (n + 1) * (n + 2) / 6 : (int64_t)n * (n + 1) / 2;
    const int64_t total = (int64_t)nm * cubes;
    const int64_t nb = mass_inner_blocks(dim, nm, n);
    if (dim == 3 && ord == 2)
        mass_inner_kernel<3, 2><<<(unsigned)nb, kMB, 0, s>>>(geo, slot_uid, npm, n, cubes, total, R, a, a_sub, b,
                                                             b_sub, partial);
    else if (dim == 3)
        mass_inner_kernel<3, 1><<<(unsigned)nb, kMB, 0, s>>>(geo, slot_uid, npm, n, cubes, total, R, a, a_sub, b,
                                                             b_sub, partial);
    else if (ord == 2)
        mass_inner_kernel<2, 2><<<(unsigned)nb, kMB, 0, s>>>(geo, slot_uid, npm, n, cubes, total, R, a, a_sub, b,
                                                             b_sub, partial);
    else
        mass_inner_kernel<2, 1><<<(unsigned)nb, kMB, 0, s>>>(geo, slot_uid, npm, n, cubes, total, R, a, a_sub, b,
                                                             b_sub, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_partials_kernel<<<1, kMB, 0, s>>>(partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_range(const double* c, int64_t n, double* partial, int64_t nblocks, double* out, hipStream_t s)
{
    range_kernel<<<(unsigned)nblocks, kMB, 0, s>>>(c, n, partial, partial + nblocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    range_final_kernel<<<1, 64, 0, s>>>(partial, partial + nblocks, nblocks, out);
    return hipGetLastError();
}

// Device address of `scratch` on `device`, which must be the current
// device: taken once per device with hipGetSymbolAddress and kept.
hipError_t noalloc_scratch(int device, double** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace mmoc
