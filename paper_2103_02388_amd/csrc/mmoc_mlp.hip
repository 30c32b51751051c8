// mmoc_mlp.hip -- kernels of the learned flow-map surrogate (not part of the
// paper's method: a network (x, t_{n+1}) -> departure point, trained on the
// tracer's own departure points, that the RK4 tracer checks and replaces
// where it is not accurate enough).
//
// Network 4 -> 64 -> 64 -> 64 -> 3, tanh-form GELU (Hendrycks & Gimpel
// 2016).  The two 64 x 64 layers run on the matrix cores
// (v_mfma_f32_16x16x32_bf16: bf16 operands, fp32 accumulation) over tiles of
// 64 samples, one wave per tile; the 4 -> 64 input layer and the 64 -> 3
// output layer run on the vector ALU in fp32 (the output layer keeps fp32
// activations: the departure point needs more than bf16's 8 bits).
//
// Matrix-core fragments (16 x 16 output tile, K = 32): lane l holds
// A[row l%16][k 8(l/16) .. +7], B[k 8(l/16) .. +7][col l%16] and the
// accumulator D[row 4(l/16) + i][col l%16], i = 0..3.  Operands are kept in
// LDS as row-major [m][k] (A) and [n][k] (B), so every fragment is one
// 16-byte read.  A 64 x 64 product is 4 x 4 tiles x 2 k-steps = 32 MFMAs.
#include "mmoc_internal.h"
#include "mmoc_mlp_internal.h"

#include <math.h>

namespace mmoc {
namespace mlp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;

constexpr int LDA = 72;  // padded bf16 row stride of LDS operand tiles (144 B)
constexpr int LDF = 65;  // padded fp32 row stride

// The tanh form u/2 (1 + tanh(v)), v = sqrt(2/pi) (u + 0.044715 u^3), is
// evaluated as u s with s = 1/(1 + e^(-2v)) (1 + tanh(v) = 2 s): one
// hardware exp2 and one hardware reciprocal, no division.  e^(-2v) =
// 2^(kk w) with w = u + 0.044715 u^3 and kk = -2 sqrt(2/pi) log2(e); for
// very negative u it overflows to +inf and s to 0, as it should.
constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2/pi)
constexpr float kGeluK = -2.3022082f;           // -2 sqrt(2/pi) / ln 2

__device__ __forceinline__ float gelu_sig(float u)
{
    const float w = fmaf(0.044715f * u, u * u, u);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(kGeluK * w));
}

__device__ __forceinline__ float gelu(float u) { return u * gelu_sig(u); }

// d/du: with 1 - tanh(v)^2 = 4 s (1 - s), gelu'(u) = s + 2 u s (1 - s) v'
__device__ __forceinline__ float gelu_d(float u)
{
    const float s = gelu_sig(u);
    const float dv = kGeluC * fmaf(3.0f * 0.044715f, u * u, 1.0f);
    return fmaf(2.0f * u * s * (1.0f - s), dv, s);
}

// acc[mt][nt] += A[64 x 64] * B where A is in LDS [m][k] (stride LDA) and B
// is given as [n][k] (stride ldb) in LDS or global memory.
template <typename BP>
__device__ __forceinline__ void mfma64(const __bf16* A, BP B, int ldb, floatx4 (&acc)[4][4])
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < 64; kk += 32) {
        bf16x8 a[4], b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[t] = *reinterpret_cast<const bf16x8*>(A + (t * 16 + r) * LDA + kk + 8 * g);
            b[t] = *reinterpret_cast<const bf16x8*>(B + (t * 16 + r) * ldb + kk + 8 * g);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
    }
}

__device__ __forceinline__ void zero(floatx4 (&acc)[4][4])
{
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// row / column of accumulator element (mt, nt, i) held by this lane
__device__ __forceinline__ int acc_row(int mt, int i) { return mt * 16 + 4 * ((threadIdx.x & 63) >> 4) + i; }
__device__ __forceinline__ int acc_col(int nt) { return nt * 16 + (threadIdx.x & 15); }

// Forward pass of one wave's 64 samples (lane = sample, inputs xin).  On
// return sA3 (fp32 [s][f], stride LDF) holds the last hidden activations and
// y the outputs.  With `keep`, z1..z3 ([s][f], fp32, global scratch gz) and
// the bf16 operands a1, a2 transposed ([f][s], sA1T / sA2T) are kept for the
// backward pass.
__device__ void forward_tile(const float* __restrict__ p32, const __bf16* __restrict__ w2, const __bf16* __restrict__ w3,
                             const float xin[4], __bf16* sA, float* sA3, float y[3], bool keep, float* gz,
                             __bf16* sA1T, __bf16* sA2T)
{
    const int lane = threadIdx.x & 63;
    // layer 1 on the vector ALU
    for (int f = 0; f < H; ++f) {
        float z = p32[OB1 + f];
#pragma unroll
        for (int i = 0; i < 4; ++i) z = fmaf(p32[OW1 + f * 4 + i], xin[i], z);
        const __bf16 a = (__bf16)gelu(z);
        sA[lane * LDA + f] = a;
        if (keep) {
            gz[0 * H * H + lane * H + f] = z;
            sA1T[f * LDA + lane] = a;
        }
    }
    __syncthreads();
    floatx4 acc[4][4];
    // layer 2
    zero(acc);
    mfma64(sA, w2, H, acc);
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int s = acc_row(mt, i), f = acc_col(nt);
                const float z = acc[mt][nt][i] + p32[OB2 + f];
                const __bf16 a = (__bf16)gelu(z);
                sA[s * LDA + f] = a;
                if (keep) {
                    gz[1 * H * H + s * H + f] = z;
                    sA2T[f * LDA + s] = a;
                }
            }
    __syncthreads();
    // layer 3
    zero(acc);
    mfma64(sA, w3, H, acc);
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int s = acc_row(mt, i), f = acc_col(nt);
                const float z = acc[mt][nt][i] + p32[OB3 + f];
                sA3[s * LDF + f] = gelu(z);
                if (keep) gz[2 * H * H + s * H + f] = z;
            }
    __syncthreads();
    // layer 4 on the vector ALU, fp32
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        float acc4 = p32[OB4 + o];
        for (int f = 0; f < H; ++f) acc4 = fmaf(p32[OW4 + o * H + f], sA3[lane * LDF + f], acc4);
        y[o] = acc4;
    }
}

__device__ __forceinline__ void scale_inputs(const MlpArgs& A, const double* x, double t, float in[4])
{
    for (int i = 0; i < 3; ++i) in[i] = (float)(2.0 * (x[i] - A.lo[i]) / (A.hi[i] - A.lo[i]) - 1.0);
    in[3] = (float)(2.0 * (t - A.lo[3]) / (A.hi[3] - A.lo[3]) - 1.0);
}

// position of DoF e: x = v0 + B s (blended shells are not supported here)
__device__ __forceinline__ void dof_pos(const MacroGeo* __restrict__ geo, uint64_t e, int lat_m, double* x)
{
    const int M = (int)(e >> 36);
    const int I = (int)((e >> 24) & 0xfffu), J = (int)((e >> 12) & 0xfffu), K = (int)(e & 0xfffu);
    const double invm = 1.0 / (double)lat_m;
    const double s[3] = {(double)(I - J) * invm, (double)(J - K) * invm, (double)K * invm};
    const MacroGeo& G = geo[M];
    for (int i = 0; i < 3; ++i) {
        double acc = G.v0[i];
        for (int a = 0; a < 3; ++a) acc = fma(G.B[i * 3 + a], s[a], acc);
        x[i] = acc;
    }
}

// ------------------------------------------------------------- inference

// Forward pass for inference, one wave per tile of 64 samples, one block per
// wave.  The hidden layers are computed transposed, D^T = W A^T: the weights
// are the matrix-core A operand ([out][in], read from L1/L2) and the
// activations the B operand ([sample][feature] in LDS), so an accumulator
// lane holds four consecutive features of one sample and writes them to LDS
// as one 8-byte store.  The last hidden layer stays in registers (fp32); the
// output layer sums each lane's 16 features per sample and reduces over the
// four lanes that share the sample.  Same bf16 rounding points as
// forward_tile; only the fp32 order of the output sums differs.
// One transposed hidden layer, n-tile by n-tile (16 samples at a time, so
// that only 16 accumulators are live): epi(nt, acc) receives
// acc[mt][i] = (W a + b)[feature mt*16 + 4g + i][sample nt*16 + r].
template <typename Epi>
__device__ __forceinline__ void hidden_t(const __bf16* __restrict__ W, const float* __restrict__ bias,
                                         const __bf16* sA, Epi epi)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    bf16x8 a[2][4];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            a[k][t] = *reinterpret_cast<const bf16x8*>(W + (t * 16 + r) * H + 32 * k + 8 * g);
    float bv[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[mt][i] = bias[mt * 16 + 4 * g + i];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        floatx4 acc[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt] = floatx4{bv[mt][0], bv[mt][1], bv[mt][2], bv[mt][3]};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(sA + (nt * 16 + r) * LDA + 32 * k + 8 * g);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[k][mt], b, acc[mt], 0, 0, 0);
        }
        epi(nt, acc);
    }
}

__device__ void forward_infer(const float* __restrict__ p32, const __bf16* __restrict__ w2,
                              const __bf16* __restrict__ w3, const float xin[4], __bf16* sA, float y[3])
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    // layer 1 on the vector ALU: four features at a time, one 8-byte store
#pragma unroll 4
    for (int f = 0; f < H; f += 4) {
        __bf16 a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float z = p32[OB1 + f + j];
#pragma unroll
            for (int i = 0; i < 4; ++i) z = fmaf(p32[OW1 + (f + j) * 4 + i], xin[i], z);
            a[j] = (__bf16)gelu(z);
        }
        *reinterpret_cast<uint2*>(sA + lane * LDA + f) = *reinterpret_cast<const uint2*>(a);
    }
    __syncthreads();
    // layer 2: a2 = gelu(W2 a1 + b2), written over a1 row block by row block
    // (an n-tile reads and writes only its own 16 sample rows; the block is
    // one wave, whose LDS operations complete in order)
    hidden_t(w2, p32 + OB2, sA, [&](int nt, const floatx4 (&acc)[4]) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            __bf16 v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = (__bf16)gelu(acc[mt][i]);
            *reinterpret_cast<uint2*>(sA + (nt * 16 + r) * LDA + mt * 16 + 4 * g) = *reinterpret_cast<const uint2*>(v);
        }
    });
    __syncthreads();
    // layer 3 (fp32 activations in registers) and the output layer: each lane
    // sums its 16 features of a sample, the four lanes of the sample
    // (r, r + 16, r + 32, r + 48) reduce, and lane l keeps sample l = 16 g + r
    const float* w4 = p32 + OW4 + 4 * g;
    float mine[3] = {0.f, 0.f, 0.f};
    hidden_t(w3, p32 + OB3, sA, [&](int nt, const floatx4 (&acc)[4]) {
        float part[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float a3 = gelu(acc[mt][i]);
#pragma unroll
                for (int o = 0; o < 3; ++o) part[o] = fmaf(w4[o * H + mt * 16 + i], a3, part[o]);
            }
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            float v = part[o];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            mine[o] = nt == g ? v : mine[o];
        }
    });
#pragma unroll
    for (int o = 0; o < 3; ++o) y[o] = p32[OB4 + o] + mine[o];
}

// Xhat = base + step_scale MLP(x, t): base is the DoF position x, or (add)
// the predictor's departure point already in X.  One wave of 64 particles
// per block.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void infer_kernel(const MlpArgs A, double t_np1, double step_scale, double* X,
                                                   int add)
{
    __shared__ __align__(16) __bf16 sA[H * LDA];
    const int64_t pid = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool active = pid < A.n;
    double x[3] = {0.0, 0.0, 0.0};
    float in[4] = {0.f, 0.f, 0.f, 0.f};
    if (active) {
        dof_pos(A.geo, A.owned[pid], A.lat_m, x);
        scale_inputs(A, x, t_np1, in);
    }
    float y[3];
    forward_infer(A.p32, A.w2, A.w3, in, sA, y);
    if (active) {
        for (int i = 0; i < 3; ++i) {
            double* xp = X + (int64_t)i * A.n + pid;
            *xp = (add ? *xp : x[i]) + (double)y[i] * step_scale;
        }
    }
}

// raw network on given inputs (test and diagnostics entry): the inference
// forward pass
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void forward_kernel(const MlpArgs A, const float* __restrict__ in4, int64_t n,
                                                     float* __restrict__ out3)
{
    __shared__ __align__(16) __bf16 sA[H * LDA];
    const int64_t s = (int64_t)blockIdx.x * 64 + threadIdx.x;
    float in[4] = {0.f, 0.f, 0.f, 0.f};
    if (s < n)
        for (int i = 0; i < 4; ++i) in[i] = in4[s * 4 + i];
    float y[3];
    forward_infer(A.p32, A.w2, A.w3, in, sA, y);
    if (s < n)
        for (int i = 0; i < 3; ++i) out3[s * 3 + i] = y[i];
}

// -------------------------------------------------------------- training

// One tile of 64 samples: forward, loss, backward; writes this tile's
// gradient (np values) and loss into part[tile].  Sample s of the tile is
// sel[tile * 64 + s] of the recorded pairs (in4 [4], tg3 [3]).
__global__ __launch_bounds__(64) void train_tile_kernel(const MlpArgs A, const float* __restrict__ in4,
                                                        const float* __restrict__ tg3, const int32_t* __restrict__ sel,
                                                        int64_t sel_off, int64_t sel_mod, int64_t sel_stride,
                                                        int64_t batch, float* __restrict__ part,
                                                        float* __restrict__ scratch)
{
    __shared__ __align__(16) __bf16 sA[H * LDA];
    __shared__ __align__(16) __bf16 sA1T[H * LDA];
    __shared__ __align__(16) __bf16 sA2T[H * LDA];
    // dz and dz^T (bf16 operands); before the backward pass the same bytes
    // hold the fp32 last-layer activations
    __shared__ __align__(16) __bf16 sDD[2 * H * LDA];
    __shared__ float sdY[H * 3];
    __shared__ float sX[H * 4];
    __bf16* sD = sDD;
    __bf16* sDT = sDD + H * LDA;
    float* sA3 = reinterpret_cast<float*>(sDD);
    static_assert(2 * H * LDA * 2 >= H * LDF * 4, "fp32 activations must fit the dz buffers");
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    float* gz = scratch + tile * (5 * H * H);  // z1, z2, z3, a3, dz ([s][f] each)
    float* ga3 = gz + 3 * H * H;
    float* gdz = gz + 4 * H * H;
    float* P = part + tile * (NP + 1);
    // the sample: a permutation walk through the selected pairs
    const int64_t pos = (sel_off + (tile * 64 + lane) * sel_stride) % sel_mod;
    const int64_t j = sel ? (int64_t)sel[pos] : pos;
    float xin[4], tg[3];
    for (int i = 0; i < 4; ++i) xin[i] = in4[j * 4 + i];
    for (int i = 0; i < 3; ++i) tg[i] = tg3[j * 3 + i];
    float y[3];
    forward_tile(A.p32, A.w2, A.w3, xin, sA, sA3, y, true, gz, sA1T, sA2T);
    // loss 1/(3B) sum |y - t|^2 and dL/dy
    const float sc = 1.0f / (3.0f * (float)batch);
    float lsum = 0.f;
    for (int o = 0; o < 3; ++o) {
        const float e = y[o] - tg[o];
        lsum += e * e * sc;
        sdY[lane * 3 + o] = 2.0f * e * sc;
    }
    for (int f = 0; f < H; ++f) ga3[lane * H + f] = sA3[lane * LDF + f];
    __syncthreads();
    // layer 4: gW4[o][f] = sum_s dy[s][o] a3[s][f] (lane = f); gb4 (lane < 3)
    for (int o = 0; o < 3; ++o) {
        float acc = 0.f;
        for (int s = 0; s < H; ++s) acc = fmaf(sdY[s * 3 + o], sA3[s * LDF + lane], acc);
        P[OW4 + o * H + lane] = acc;
    }
    if (lane < 3) {
        float acc = 0.f;
        for (int s = 0; s < H; ++s) acc += sdY[s * 3 + lane];
        P[OB4 + lane] = acc;
    }
    // dz3[s][f] = (sum_o dy[s][o] W4[o][f]) gelu'(z3[s][f])   (lane = s)
    for (int f = 0; f < H; ++f) {
        float da = 0.f;
        for (int o = 0; o < 3; ++o) da = fmaf(sdY[lane * 3 + o], A.p32[OW4 + o * H + f], da);
        const float dz = da * gelu_d(gz[2 * H * H + lane * H + f]);
        gdz[lane * H + f] = dz;
        const __bf16 b = (__bf16)dz;
        sD[lane * LDA + f] = b;
        sDT[f * LDA + lane] = b;
    }
    __syncthreads();
    floatx4 acc[4][4];
    for (int layer = 3; layer >= 2; --layer) {
        const int OW = layer == 3 ? OW3 : OW2, OB = layer == 3 ? OB3 : OB2;
        const __bf16* aT = layer == 3 ? sA2T : sA1T;            // [in][s]
        const __bf16* wT = layer == 3 ? A.w3t : A.w2t;          // [in][out]
        // bias gradient: column sums of dz (lane = f)
        {
            float b = 0.f;
            for (int s = 0; s < H; ++s) b += gdz[s * H + lane];
            P[OB + lane] = b;
        }
        // dW[out][in] = dz^T (M = out, K = s) x a (K = s, N = in)
        zero(acc);
        mfma64(sDT, aT, LDA, acc);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) P[OW + acc_row(mt, i) * H + acc_col(nt)] = acc[mt][nt][i];
        // da[s][in] = dz (M = s, K = out) x W (K = out, N = in)
        zero(acc);
        mfma64(sD, wT, H, acc);
        __syncthreads();
        // dz of the layer below: da * gelu'(z)
        const float* zb = gz + (layer == 3 ? 1 : 0) * H * H;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int s = acc_row(mt, i), f = acc_col(nt);
                    const float dz = acc[mt][nt][i] * gelu_d(zb[s * H + f]);
                    gdz[s * H + f] = dz;
                    const __bf16 b = (__bf16)dz;
                    sD[s * LDA + f] = b;
                    sDT[f * LDA + s] = b;
                }
        __syncthreads();
    }
    // layer 1: gW1[f][i] = sum_s dz1[s][f] x[s][i], gb1 (lane = f)
    for (int i = 0; i < 4; ++i) sX[lane * 4 + i] = xin[i];
    __syncthreads();
    {
        float gw[4] = {0.f, 0.f, 0.f, 0.f}, gb = 0.f;
        for (int s = 0; s < H; ++s) {
            const float dz = gdz[s * H + lane];
            gb += dz;
            for (int i = 0; i < 4; ++i) gw[i] = fmaf(dz, sX[s * 4 + i], gw[i]);
        }
        for (int i = 0; i < 4; ++i) P[OW1 + lane * 4 + i] = gw[i];
        P[OB1 + lane] = gb;
    }
    // tile loss
    float l = lsum;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == 0) P[NP] = l;
}

// Sum of the tile gradients in a fixed order, then one Adam step
// (bias-corrected) on the fp32 master parameters and a refresh of the bf16
// copies of the matrix-core weights.  *loss_out (if set) receives the batch loss.
__global__ __launch_bounds__(256) void reduce_adam_kernel(MlpState S, const float* __restrict__ part, int ntiles,
                                                          float lr, float b1, float b2, float eps, int64_t t,
                                                          float* loss_out)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > NP) return;
    float g = 0.f;
    for (int k = 0; k < ntiles; ++k) g += part[(int64_t)k * (NP + 1) + p];
    if (p == NP) {
        if (loss_out) *loss_out = g;
        return;
    }
    if (S.grad) S.grad[p] = g;
    if (lr == 0.f) return;
    const float m = b1 * S.m[p] + (1.f - b1) * g;
    const float v = b2 * S.v[p] + (1.f - b2) * g * g;
    S.m[p] = m;
    S.v[p] = v;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    const float w = S.p32[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    S.p32[p] = w;
    refresh_bf16(S, p, w);
}

__global__ __launch_bounds__(256) void refresh_kernel(MlpState S)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < NP) refresh_bf16(S, p, S.p32[p]);
}

// ---------------------------------------------------------- record / select

// training pairs of one traced step: inputs (x, t) scaled to [-1, 1],
// targets (X - base) / scale with base the DoF position x or, with a
// predictor, its departure point Xp
__global__ __launch_bounds__(256) void record_kernel(const MlpArgs A, double t_np1, double inv_step_scale,
                                                     const double* __restrict__ X, const double* __restrict__ Xp,
                                                     float* __restrict__ in4, float* __restrict__ tg3)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.n) return;
    double x[3];
    dof_pos(A.geo, A.owned[i], A.lat_m, x);
    float in[4];
    scale_inputs(A, x, t_np1, in);
    for (int k = 0; k < 4; ++k) in4[i * 4 + k] = in[k];
    for (int k = 0; k < 3; ++k) {
        const double base = Xp ? Xp[(int64_t)k * A.n + i] : x[k];
        tg3[i * 3 + k] = (float)((X[(int64_t)k * A.n + i] - base) * inv_step_scale);
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    // splitmix64 finaliser (Steele, Lea, Flood 2014)
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// seeded draw (with replacement) of n indices into [0, count)
__global__ __launch_bounds__(256) void draw_kernel(uint64_t seed, int64_t n, int64_t count, int32_t* __restrict__ sel)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    sel[i] = (int32_t)(mix64(seed ^ mix64((uint64_t)i)) % (uint64_t)count);
}

}  // namespace

__device__ void refresh_bf16(const MlpState& S, int p, float w)
{
    if (p >= OW2 && p < OW2 + H * H) {
        const int o = (p - OW2) / H, i = (p - OW2) % H;
        S.w2[o * H + i] = (__bf16)w;
        S.w2t[i * H + o] = (__bf16)w;
    } else if (p >= OW3 && p < OW3 + H * H) {
        const int o = (p - OW3) / H, i = (p - OW3) % H;
        S.w3[o * H + i] = (__bf16)w;
        S.w3t[i * H + o] = (__bf16)w;
    }
}

hipError_t launch_infer(const MlpArgs& a, double t_np1, double step_scale, double* X, int add, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    infer_kernel<<<grid, 64, 0, s>>>(a, t_np1, step_scale, X, add);
    return hipGetLastError();
}

hipError_t launch_forward(const MlpArgs& a, const float* in4, int64_t n, float* out3, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    forward_kernel<<<(unsigned)((n + 63) / 64), 64, 0, s>>>(a, in4, n, out3);
    return hipGetLastError();
}

hipError_t launch_train_step(const MlpArgs& a, const MlpState& st, const float* in4, const float* tg3,
                             const int32_t* sel, int64_t sel_off, int64_t sel_mod, int64_t sel_stride, int64_t batch,
                             float* part, float* scratch, float lr, int64_t t, float* loss_out, hipStream_t s)
{
    const int ntiles = (int)(batch / 64);
    train_tile_kernel<<<ntiles, 64, 0, s>>>(a, in4, tg3, sel, sel_off, sel_mod, sel_stride, batch, part, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_adam_kernel<<<(NP + 1 + 255) / 256, 256, 0, s>>>(st, part, ntiles, lr, 0.9f, 0.999f, 1e-8f, t, loss_out);
    return hipGetLastError();
}

hipError_t launch_refresh(const MlpState& st, hipStream_t s)
{
    refresh_kernel<<<(NP + 255) / 256, 256, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_record(const MlpArgs& a, double t_np1, double inv_step_scale, const double* X, const double* Xp,
                         float* in4, float* tg3, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    record_kernel<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(a, t_np1, inv_step_scale, X, Xp, in4, tg3);
    return hipGetLastError();
}

hipError_t launch_draw(uint64_t seed, int64_t n, int64_t count, int32_t* sel, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    draw_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(seed, n, count, sel);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace mmoc
