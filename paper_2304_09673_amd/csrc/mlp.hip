// Step-predictor MLP kernels: operand-table packing, batched inference on the
// matrix cores (the same device function the tracer calls), forward/backward
// for training, Adam, and a probe of the matrix-instruction lane layout.
#include <cmath>

#include "st_internal.h"
#include "st_mlp.h"

namespace st {

// ---------------------------------------------------------------------------
// operand table from the FP32 master parameters (rounded to binary16) and the
// feature normalisation (mean[8], inverse std[8])
__global__ void mlp_pack_kernel(const float* __restrict__ w, const float* __restrict__ norm, uint32_t* __restrict__ tab) {
    const int l = int(threadIdx.x);
    if (l >= 64) return;
    const int h = l & 31, g = l >> 5;
    tab[0 * 64 + l] = pack_h2(w[kMlpW1 + h * 8 + 4 * g + 0], w[kMlpW1 + h * 8 + 4 * g + 1]);
    tab[1 * 64 + l] = pack_h2(w[kMlpW1 + h * 8 + 4 * g + 2], w[kMlpW1 + h * 8 + 4 * g + 3]);
    for (int c = 0; c < 4; c++) {
        const float* r = w + kMlpW2 + h * 32 + 8 * c + 4 * g;
        tab[(2 + 2 * c) * 64 + l] = pack_h2(r[0], r[1]);
        tab[(3 + 2 * c) * 64 + l] = pack_h2(r[2], r[3]);
    }
    for (int a = 0; a < 16; a++) {
        int row = mlp_row(a, g);
        tab[(10 + a) * 64 + l] = __float_as_uint(round_half(w[kMlpB1 + row]));
        tab[(26 + a) * 64 + l] = __float_as_uint(round_half(w[kMlpB2 + row]));
        tab[(42 + a) * 64 + l] = __float_as_uint(round_half(w[kMlpW3 + row]));
    }
    tab[58 * 64 + l] = __float_as_uint(round_half(w[kMlpB3]));
    if (l < 16) tab[kMlpTabRows * 64 + l] = __float_as_uint(norm[l]);
}

// batched inference: sample i on lane i % 64 of wave i / 64
__global__ void __launch_bounds__(256) mlp_forward_kernel(const uint32_t* __restrict__ tab_g, const float* __restrict__ x,
                                                          int n, float* __restrict__ out) {
    __shared__ uint32_t tab[kMlpTabWords];
    for (int i = threadIdx.x; i < kMlpTabWords; i += blockDim.x) tab[i] = tab_g[i];
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    float f[8];
    for (int k = 0; k < 8; k++) f[k] = i < n ? x[8 * size_t(i) + k] : 0.f;
    float om = mlp_omega(tab, f);   // all lanes active
    if (i < n) out[i] = om;
}

// D = A . B with one v_mfma_f32_32x32x8_f16, A (32x8) and B (8x32) given row-major
// as floats; D written row-major by the accumulator-row formula mlp_row.
__global__ void mfma_probe_kernel(const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ D) {
    const int l = int(threadIdx.x & 63u), g = l >> 5, h = l & 31;
    h4_t a = h4_from(pack_h2(A[h * 8 + 4 * g], A[h * 8 + 4 * g + 1]), pack_h2(A[h * 8 + 4 * g + 2], A[h * 8 + 4 * g + 3]));
    h4_t b = h4_from(pack_h2(B[(4 * g) * 32 + h], B[(4 * g + 1) * 32 + h]),
                     pack_h2(B[(4 * g + 2) * 32 + h], B[(4 * g + 3) * 32 + h]));
    f16_t c;
    for (int k = 0; k < 16; k++) c[k] = 0.f;
    f16_t d = __builtin_amdgcn_mfma_f32_32x32x8f16(a, b, c, 0, 0, 0);
    for (int k = 0; k < 16; k++) D[mlp_row(k, g) * 32 + h] = d[k];
}

// ---------------------------------------------------------------------------
// training: loss mean_i w_i (omega_i - target_i)^2, w_i = over_weight when omega_i > target_i.
// One thread per sample; forward and backward in FP32 with the inference's
// binary16 rounding points (inputs, weights, hidden activations; error signals
// that feed a product); gradients summed per block in LDS, then one global
// atomic per parameter per block.
__global__ void __launch_bounds__(256) mlp_grad_kernel(const float* __restrict__ wm, const float* __restrict__ norm,
                                                       const float* __restrict__ x, const float* __restrict__ tgt, int n,
                                                       float over_weight, float* __restrict__ grad,
                                                       float* __restrict__ loss) {
    __shared__ float W[kMlpParams];
    __shared__ float G[kMlpParams];
    __shared__ float L;
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) {
        W[i] = round_half(wm[i]);
        G[i] = 0.f;
    }
    if (threadIdx.x == 0) L = 0.f;
    __syncthreads();
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        const float inv_n = 1.0f / float(n);
        float xi[8];
        for (int k = 0; k < 8; k++) xi[k] = round_half(mlp_feature(x[8 * size_t(s) + k], norm[k], norm[8 + k]));
        float a1[32], h1[32], a2[32], h2[32];
        for (int j = 0; j < 32; j++) {
            float acc = W[kMlpB1 + j];
            for (int k = 0; k < 8; k++) acc = fmaf(W[kMlpW1 + j * 8 + k], xi[k], acc);
            a1[j] = acc;
            h1[j] = round_half(fmaxf(acc, 0.f));
        }
        for (int j = 0; j < 32; j++) {
            float acc = W[kMlpB2 + j];
            for (int k = 0; k < 32; k++) acc = fmaf(W[kMlpW2 + j * 32 + k], h1[k], acc);
            a2[j] = acc;
            h2[j] = round_half(fmaxf(acc, 0.f));
        }
        float z = W[kMlpB3];
        for (int k = 0; k < 32; k++) z = fmaf(W[kMlpW3 + k], h2[k], z);
        float sg = 1.0f / (1.0f + expf(-z));
        float om = 1.0f + (kOmegaMax - 1.0f) * sg;
        float diff = om - tgt[s];
        float wgt = om > tgt[s] ? over_weight : 1.0f;
        atomicAdd(&L, wgt * diff * diff * inv_n);
        float dz = 2.0f * wgt * diff * inv_n * (kOmegaMax - 1.0f) * sg * (1.0f - sg);
        atomicAdd(&G[kMlpB3], dz);
        float d2[32];
        for (int k = 0; k < 32; k++) {
            atomicAdd(&G[kMlpW3 + k], dz * h2[k]);
            d2[k] = a2[k] > 0.f ? dz * W[kMlpW3 + k] : 0.f;
        }
        for (int j = 0; j < 32; j++) {
            float dh = round_half(d2[j]);
            atomicAdd(&G[kMlpB2 + j], d2[j]);
            if (dh != 0.f)
                for (int k = 0; k < 32; k++) atomicAdd(&G[kMlpW2 + j * 32 + k], dh * h1[k]);
            d2[j] = dh;
        }
        for (int k = 0; k < 32; k++) {
            float acc = 0.f;
            for (int j = 0; j < 32; j++) acc = fmaf(W[kMlpW2 + j * 32 + k], d2[j], acc);
            float d1 = a1[k] > 0.f ? acc : 0.f;
            atomicAdd(&G[kMlpB1 + k], d1);
            float dh = round_half(d1);
            if (dh != 0.f)
                for (int i = 0; i < 8; i++) atomicAdd(&G[kMlpW1 + k * 8 + i], dh * xi[i]);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x)
        if (G[i] != 0.f) atomicAdd(grad + i, G[i]);
    if (threadIdx.x == 0) atomicAdd(loss, L);
}

__global__ void mlp_adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                                float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace st

using namespace st;

extern "C" {

st_status st_mlp_pack(const float* w, const float* norm, uint32_t* tab, void* stream) {
    if (!w || !norm || !tab) { set_error("mlp_pack: NULL argument"); return ST_E_INVALID; }
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, w, norm, tab);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "mlp_pack_kernel");
}

st_status st_mlp_forward(const uint32_t* tab, const float* x, int32_t n, float* omega, void* stream) {
    if (!tab || (n > 0 && (!x || !omega)) || n < 0) { set_error("mlp_forward: bad argument"); return ST_E_INVALID; }
    if (n == 0) return ST_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, tab, x, n, omega);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "mlp_forward_kernel");
}

st_status st_mlp_grad(const float* w, const float* norm, const float* x, const float* target, int32_t n,
                      float over_weight, float* grad, float* loss, void* stream) {
    if (!w || !norm || !grad || !loss || n < 0 || (n > 0 && (!x || !target)) || !(over_weight > 0.f)) {
        set_error("mlp_grad: bad argument");
        return ST_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(grad, 0, kMlpParams * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(loss, 0, 4, st);
    if (e != hipSuccess) return device_error(e, "mlp_grad memset");
    if (n == 0) return ST_OK;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, norm, x, target, n, over_weight,
                       grad, loss);
    e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "mlp_grad_kernel");
}

st_status st_mlp_adam(float* w, float* m, float* v, const float* grad, int32_t n, int32_t step, float lr, float beta1,
                      float beta2, float eps, void* stream) {
    if (!w || !m || !v || !grad || n <= 0 || step < 1) { set_error("mlp_adam: bad argument"); return ST_E_INVALID; }
    float c1 = 1.0f / (1.0f - std::pow(beta1, float(step)));
    float c2 = 1.0f / (1.0f - std::pow(beta2, float(step)));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, w, m, v, grad, n, lr,
                       beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "mlp_adam_kernel");
}

st_status st_debug_mfma_probe(const float* A, const float* B, float* D, void* stream) {
    if (!A || !B || !D) { set_error("mfma_probe: NULL argument"); return ST_E_INVALID; }
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, D);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "mfma_probe_kernel");
}

}  // extern "C"
