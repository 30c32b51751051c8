// mmoc_mlp_internal.h -- layouts shared by the surrogate's host code and
// kernels (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mmoc_internal.h"

namespace mmoc {
namespace mlp {

constexpr int H = 64;
// flat parameter vector: W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
constexpr int OW1 = 0, OB1 = OW1 + 4 * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * H,
              OW4 = OB3 + H, OB4 = OW4 + 3 * H, NP = OB4 + 3;
static_assert(NP == 8835, "parameter count");

// read-only view for inference and the forward/backward pass
struct MlpArgs {
    const MacroGeo* geo;
    const uint64_t* owned;
    int64_t n;            // particles (inference, record)
    int lat_m;  // DoF lattice resolution
    double lo[4], hi[4];  // input box, mapped to [-1, 1]
    const float* p32;     // master parameters
    const __bf16* w2;     // bf16 W2 [out][in]
    const __bf16* w3;
    const __bf16* w2t;    // bf16 W2^T [in][out]
    const __bf16* w3t;
};

// optimizer state (device)
struct MlpState {
    float* p32;
    float* m;
    float* v;
    float* grad;  // optional: last summed gradient
    __bf16* w2;
    __bf16* w3;
    __bf16* w2t;
    __bf16* w3t;
};

__device__ void refresh_bf16(const MlpState& S, int p, float w);

// X = (add ? X : x) + step_scale MLP(x, t_np1) for every particle
hipError_t launch_infer(const MlpArgs& a, double t_np1, double step_scale, double* X, int add, hipStream_t s);
hipError_t launch_forward(const MlpArgs& a, const float* in4, int64_t n, float* out3, hipStream_t s);
// one optimizer step on `batch` samples (multiple of 64); lr == 0: gradient only (into st.grad)
hipError_t launch_train_step(const MlpArgs& a, const MlpState& st, const float* in4, const float* tg3,
                             const int32_t* sel, int64_t sel_off, int64_t sel_mod, int64_t sel_stride, int64_t batch,
                             float* part, float* scratch, float lr, int64_t t, float* loss_out, hipStream_t s);
hipError_t launch_refresh(const MlpState& st, hipStream_t s);
// training pairs: inputs (x, t_np1), targets (X - (Xp ? Xp : x)) * inv_step_scale
hipError_t launch_record(const MlpArgs& a, double t_np1, double inv_step_scale, const double* X, const double* Xp,
                         float* in4, float* tg3, hipStream_t s);
hipError_t launch_draw(uint64_t seed, int64_t n, int64_t count, int32_t* sel, hipStream_t s);

// surrogate step helpers (mmoc_trace.hip)
// particles with hash(seed, i) < fraction, and the smallest hash of every
// tile of `tile` particles, appended to ids (count in *n_ids); flags cleared
hipError_t launch_select_check(int64_t n, int tile, uint64_t seed, float fraction, int32_t* ids,
                               unsigned long long* n_ids, int64_t cap, unsigned char* checked, hipStream_t s);
}  // namespace mlp
}  // namespace mmoc
