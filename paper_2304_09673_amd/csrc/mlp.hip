// Step-predictor MLP kernels: operand-table packing, batched inference on the
// matrix cores (the same device function the tracer calls), forward/backward
// for training, Adam, and a probe of the matrix-instruction lane layout.
#include <algorithm>
#include <cmath>
#include <vector>

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
// training: loss mean_i w_i (omega_i - target_i)^2, w_i = over_weight when
// omega_i > target_i.  One wave per workgroup, 64 samples per pass (lane =
// sample), grid-stride over passes.  Each lane runs its sample's forward and
// backward in FP32 with the inference's binary16 rounding points (inputs,
// weights, hidden activations; error signals that feed a product) and stores
// the per-sample vectors in LDS, row-major [sample][unit]; the weight
// gradients are sums over samples of outer products, i.e. GEMMs with the
// sample index as K, and run on the matrix cores in FP32
// (v_mfma_f32_32x32x2f32: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32], so for samples 2t, 2t + 1 lane l reads the element
// 64t + l of both row-major tables).  Bias gradients and w3 use the same
// instruction with a constant or per-sample B column.  The accumulators stay
// in registers over all passes of the wave; one atomic per parameter per
// wave at the end.  idx (may be NULL) maps sample i to its row in x / tgt.
constexpr int kGradRow = 33;   // padded row: conflict-free LDS stores and loads
typedef float f16v_t __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(64) mlp_grad_kernel(const float* __restrict__ wm, const float* __restrict__ norm,
                                                      const float* __restrict__ x, const float* __restrict__ tgt,
                                                      const uint32_t* __restrict__ idx, int n, float over_weight,
                                                      float loss_scale, float* __restrict__ grad,
                                                      float* __restrict__ loss) {
    __shared__ float W[kMlpParams];
    __shared__ float sH1[64 * kGradRow], sH2[64 * kGradRow], sD2[64 * kGradRow], sDH2[64 * kGradRow];
    __shared__ float sD1[64 * kGradRow], sDH1[64 * kGradRow], sX[64 * 9], sDZ[64];
    const int l = int(threadIdx.x), g = l >> 5, h = l & 31;
    for (int i = l; i < kMlpParams; i += 64) W[i] = round_half(wm[i]);
    __syncthreads();
    f16v_t gW1, gW2, gB1, gB2, gW3;
    for (int r = 0; r < 16; r++) gW1[r] = gW2[r] = gB1[r] = gB2[r] = gW3[r] = 0.f;
    float lsum = 0.f, dzsum = 0.f;
    const float inv_n = 1.0f / float(n);
    for (int base = int(blockIdx.x) * 64; base < n; base += int(gridDim.x) * 64) {
        const int s = base + l;
        const bool valid = s < n;
        const size_t row = valid ? (idx ? size_t(idx[s]) : size_t(s)) : 0u;
        float xi[8];
        for (int k = 0; k < 8; k++) xi[k] = valid ? round_half(mlp_feature(x[8 * row + k], norm[k], norm[8 + k])) : 0.f;
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
        const float sg = 1.0f / (1.0f + expf(-z));
        const float om = 1.0f + (kOmegaMax - 1.0f) * sg;
        const float tv = valid ? tgt[row] : om;
        const float diff = om - tv;
        const float wgt = om > tv ? over_weight : 1.0f;
        lsum += valid ? wgt * diff * diff * inv_n : 0.f;
        const float dz = valid ? 2.0f * wgt * diff * inv_n * (kOmegaMax - 1.0f) * sg * (1.0f - sg) : 0.f;
        dzsum += dz;
        float* rH1 = sH1 + l * kGradRow;
        float* rH2 = sH2 + l * kGradRow;
        float* rD2 = sD2 + l * kGradRow;
        float* rDH2 = sDH2 + l * kGradRow;
        float* rD1 = sD1 + l * kGradRow;
        float* rDH1 = sDH1 + l * kGradRow;
        float dh2[32];
        for (int j = 0; j < 32; j++) {
            const float d2 = a2[j] > 0.f ? dz * W[kMlpW3 + j] : 0.f;
            dh2[j] = round_half(d2);
            rD2[j] = d2;
            rDH2[j] = dh2[j];
            rH1[j] = h1[j];
            rH2[j] = h2[j];
        }
        for (int k = 0; k < 32; k++) {
            float acc = 0.f;
            for (int j = 0; j < 32; j++) acc = fmaf(W[kMlpW2 + j * 32 + k], dh2[j], acc);
            const float d1 = a1[k] > 0.f ? acc : 0.f;
            rD1[k] = d1;
            rDH1[k] = round_half(d1);
        }
        for (int k = 0; k < 8; k++) sX[l * 9 + k] = xi[k];
        sDZ[l] = dz;
        __syncthreads();
        // sums over the 64 samples: 32 matrix instructions of K = 2 each
        for (int t = 0; t < 32; t++) {
            const int r = (2 * t + g) * kGradRow + h;
            const float xb = h < 8 ? sX[(2 * t + g) * 9 + h] : 0.f;
            gW2 = __builtin_amdgcn_mfma_f32_32x32x2f32(sDH2[r], sH1[r], gW2, 0, 0, 0);
            gW1 = __builtin_amdgcn_mfma_f32_32x32x2f32(sDH1[r], xb, gW1, 0, 0, 0);
            gB2 = __builtin_amdgcn_mfma_f32_32x32x2f32(sD2[r], 1.0f, gB2, 0, 0, 0);
            gB1 = __builtin_amdgcn_mfma_f32_32x32x2f32(sD1[r], 1.0f, gB1, 0, 0, 0);
            gW3 = __builtin_amdgcn_mfma_f32_32x32x2f32(sH2[r], sDZ[2 * t + g], gW3, 0, 0, 0);
        }
        __syncthreads();   // the next pass overwrites the tables
    }
    // accumulator element r of lane l: row mlp_row(r, g), column h
    for (int r = 0; r < 16; r++) {
        const int i = mlp_row(r, g);
        atomicAdd(grad + kMlpW2 + i * 32 + h, gW2[r]);
        if (h < 8) atomicAdd(grad + kMlpW1 + i * 8 + h, gW1[r]);
        if (h == 0) {
            atomicAdd(grad + kMlpB2 + i, gB2[r]);
            atomicAdd(grad + kMlpB1 + i, gB1[r]);
            atomicAdd(grad + kMlpW3 + i, gW3[r]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lsum += __shfl_xor(lsum, o);
        dzsum += __shfl_xor(dzsum, o);
    }
    if (l == 0) {
        atomicAdd(grad + kMlpB3, dzsum);
        atomicAdd(loss, lsum * loss_scale);
    }
}

// grid of the gradient kernel: one wave per 64 samples, at most kGradWaves
constexpr int kGradWaves = 2048;
__host__ __forceinline__ unsigned grad_grid(int n) { return unsigned(std::min((n + 63) / 64, kGradWaves)); }

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

// feature standardisation over n samples: norm[f] = mean, norm[8 + f] =
// 1 / max(std, 1e-6) (population std, sums in FP64); one workgroup per feature
__global__ void __launch_bounds__(1024) mlp_norm_kernel(const float* __restrict__ x, int64_t n,
                                                        float* __restrict__ norm) {
    __shared__ double s1[1024], s2[1024];
    const int f = int(blockIdx.x), tid = int(threadIdx.x);
    double a = 0.0, b = 0.0;
    for (int64_t i = tid; i < n; i += 1024) {
        const double v = x[8 * i + f];
        a += v;
        b += v * v;
    }
    s1[tid] = a;
    s2[tid] = b;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o) {
            s1[tid] += s1[tid + o];
            s2[tid] += s2[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double m = s1[0] / double(n);
        const double var = std::max(s2[0] / double(n) - m * m, 0.0);
        norm[f] = float(m);
        norm[8 + f] = float(1.0 / std::max(std::sqrt(var), 1e-6));
    }
}

// host generator of the initial weights and the sample order: splitmix64
// (Steele, Lea and Flood 2014), normals by the Box-Muller transform
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }   // [0, 1)
    double normal() {
        const double u1 = 1.0 - uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

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
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(grad_grid(n)), dim3(64), 0, st, w, norm, x, target,
                       (const uint32_t*)nullptr, n, over_weight, 1.0f, grad, loss);
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

st_status st_train_step_model(const float* x, const float* target, int64_t n, int32_t epochs, int32_t batch,
                              float lr, float over_weight, uint64_t seed, float* weights, float* norm,
                              float* losses, void* stream_v) {
    if (!x || !target || !weights || !norm || n < 1 || n > int64_t(0x7FFFFFFF) || epochs < 1 || batch < 1 ||
        !(lr > 0.f) || !(over_weight > 0.f)) {
        set_error("train_step_model: bad argument");
        return ST_E_INVALID;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    SplitMix64 rng{seed};
    // initial weights: He normal hidden layers, a small output layer, b3 so
    // that omega starts near 1.5; zero biases
    std::vector<float> w0(kMlpParams, 0.f);
    for (int i = 0; i < 256; i++) w0[kMlpW1 + i] = float(rng.normal() * std::sqrt(2.0 / 8.0));
    for (int i = 0; i < 1024; i++) w0[kMlpW2 + i] = float(rng.normal() * std::sqrt(2.0 / 32.0));
    for (int i = 0; i < 32; i++) w0[kMlpW3 + i] = float(rng.normal() * 0.1 / std::sqrt(32.0));
    w0[kMlpB3] = float(std::log(0.5 / (double(kOmegaMax) - 1.0 - 0.5)));
    // one seeded order of the samples for all epochs (Fisher-Yates)
    std::vector<uint32_t> order(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; i++) order[size_t(i)] = uint32_t(i);
    for (int64_t i = n - 1; i > 0; i--) std::swap(order[size_t(i)], order[size_t(rng.next() % uint64_t(i + 1))]);
    uint32_t* d_idx = nullptr;
    float *d_m = nullptr, *d_v = nullptr, *d_g = nullptr, *d_loss = nullptr;
    hipError_t e = hipMalloc(&d_idx, sizeof(uint32_t) * size_t(n));
    if (e == hipSuccess) e = hipMalloc(&d_m, 3 * kMlpParams * sizeof(float) + size_t(epochs) * sizeof(float));
    if (e != hipSuccess) {
        (void)hipFree(d_idx);
        set_error("train_step_model: device allocation failed");
        return ST_E_NOMEM;
    }
    d_v = d_m + kMlpParams;
    d_g = d_v + kMlpParams;
    d_loss = d_g + kMlpParams;
    e = hipMemcpyAsync(d_idx, order.data(), sizeof(uint32_t) * size_t(n), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(weights, w0.data(), kMlpParams * sizeof(float), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_m, 0, 2 * kMlpParams * sizeof(float), stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_loss, 0, size_t(epochs) * sizeof(float), stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(mlp_norm_kernel, dim3(8), dim3(1024), 0, stream, x, n, norm);
        e = hipGetLastError();
    }
    // full batches only (a trailing partial batch is dropped)
    const int64_t nb = std::max<int64_t>(1, n / batch);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int step = 0;
    for (int ep = 0; ep < epochs && e == hipSuccess; ep++) {
        for (int64_t b = 0; b < nb && e == hipSuccess; b++) {
            const int64_t lo = b * batch, cnt = std::min<int64_t>(n, lo + batch) - lo;
            e = hipMemsetAsync(d_g, 0, kMlpParams * sizeof(float), stream);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(mlp_grad_kernel, dim3(grad_grid(int(cnt))), dim3(64), 0, stream, weights, norm, x,
                               target, d_idx + lo, int(cnt), over_weight, 1.0f / float(nb), d_g, d_loss + ep);
            step++;
            const float c1 = 1.0f / (1.0f - std::pow(b1, float(step)));
            const float c2 = 1.0f / (1.0f - std::pow(b2, float(step)));
            hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, weights, d_m,
                               d_v, d_g, kMlpParams, lr, b1, b2, eps, c1, c2);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && losses)
        e = hipMemcpyAsync(losses, d_loss, size_t(epochs) * sizeof(float), hipMemcpyDeviceToHost, stream);
    // the host buffers above and the temporaries live until the work is done
    const hipError_t es = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = es;
    (void)hipFree(d_idx);
    (void)hipFree(d_m);
    return e == hipSuccess ? ST_OK : device_error(e, "train_step_model");
}

st_status st_debug_mfma_probe(const float* A, const float* B, float* D, void* stream) {
    if (!A || !B || !D) { set_error("mfma_probe: NULL argument"); return ST_E_INVALID; }
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, D);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ST_OK : device_error(e, "mfma_probe_kernel");
}

}  // extern "C"
