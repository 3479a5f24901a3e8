// lb_mlp.hip -- kernels of the learned interface closure: FP32 training of
// the 10-64-64-8 network (forward, loss, backward, Adam) and the bf16
// closure evaluation used by the tests.
//
// Training is written as dense layers over a batch, one thread per output
// element; every reduction over the batch runs in a fixed order (per-thread
// strided sums, then a fixed tree in LDS), so gradients are deterministic.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lb.h"
#include "lb_kernels.hpp"
#include "lb_registry.hpp"

using namespace lbk;

namespace {

// out[r][c] = act(sum_k A[r][k] W[c][k] + b[c])
__global__ void k_dense(const float *A, int K, const float *W, const float *b, float *out, int M, int64_t n,
                        int act) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * M) return;
    const int64_t r = idx / M;
    const int c = int(idx % M);
    float s = b ? b[c] : 0.0f;
    for (int k = 0; k < K; ++k) s += A[r * K + k] * W[c * K + k];
    out[idx] = act ? tanhf(s) : s;
}

// out[r][k] = (sum_c D[r][c] W[c][k]) (1 - H[r][k]^2): back through a
// tanh layer
__global__ void k_dense_back(const float *D, int M, const float *W, const float *H, float *out, int K, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * K) return;
    const int64_t r = idx / K;
    const int k = int(idx % K);
    float s = 0.0f;
    for (int c = 0; c < M; ++c) s += D[r * M + c] * W[c * K + k];
    const float h = H[idx];
    out[idx] = s * (1.0f - h * h);
}

// gW[c][k] = sum_r D[r][c] H[r][k], gb[c] = sum_r D[r][c]: one block per
// output element (weights first, then biases); thread t sums the rows
// t, t + 256, ..., and the block adds the 256 partial sums in a fixed
// tree, so the gradient does not depend on scheduling
__global__ __launch_bounds__(256) void k_outer(const float *D, int M, const float *H, int K, int64_t n, float *gW,
                                               float *gb) {
    __shared__ float sh[256];
    const int idx = blockIdx.x;
    const bool bias = idx >= M * K;
    const int c = bias ? idx - M * K : idx / K, k = bias ? 0 : idx % K;
    float s = 0.0f;
    if (bias) {
        for (int64_t r = threadIdx.x; r < n; r += 256) s += D[r * M + c];
    } else {
        for (int64_t r = threadIdx.x; r < n; r += 256) s += D[r * M + c] * H[r * K + k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (bias) gb[c] = sh[0];
        else gW[idx] = sh[0];
    }
}

// per sample: squared error of the 6 regression outputs / 6 + cross-entropy
// of the 2 flag logits; dY = gradient of the batch mean
__global__ void k_loss(const float *Y, const float *T, const int32_t *flag, int64_t n, float *dY, float *lv) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float *y = Y + 8 * r;
    float *d = dY + 8 * r;
    float l = 0.0f;
    for (int c = 0; c < 6; ++c) {
        const float e = y[c] - T[6 * r + c];
        l += e * e / 6.0f;
        d[c] = 2.0f * e / 6.0f / float(n);
    }
    const float z0 = y[6], z1 = y[7], zm = fmaxf(z0, z1);
    const float lse = zm + logf(expf(z0 - zm) + expf(z1 - zm));
    const int f = flag[r];
    l += lse - (f ? z1 : z0);
    d[6] = (expf(z0 - lse) - (f == 0 ? 1.0f : 0.0f)) / float(n);
    d[7] = (expf(z1 - lse) - (f == 1 ? 1.0f : 0.0f)) / float(n);
    lv[r] = l;
}

__global__ void k_mean1(const float *v, int64_t n, float *out) {
    __shared__ float sh[256];
    float s = 0.0f;
    for (int64_t k = threadIdx.x; k < n; k += 256) s += v[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / float(n);
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t np, float lr, float bc1, float bc2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const float gk = g[k];
    const float mk = 0.9f * m[k] + 0.1f * gk;
    const float vk = 0.999f * v[k] + 0.001f * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + 1e-8f);
}

__global__ void k_to_bf16(const float *p, uint16_t *out, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = f_to_bf16(p[k]);
}

// Closure coefficients of n D2Q9 nodes, evaluated as in the lift (the
// matrix-core network of lb_kernels.hpp), from FP32 weights rounded to bf16
__global__ __launch_bounds__(64) void k_closure_eval(const uint16_t *w, ClosureNorm cn, const double *f9, int64_t n,
                                                     double *c36, double rho_ref) {
    __shared__ float xs[16][16];
    __shared__ float hs[16][MLP_NH + 4];
    __shared__ float rs[16];
    __shared__ float c6[16][6];
    const int lane = threadIdx.x;
    const int64_t e0 = int64_t(blockIdx.x) * 16;
    const int nn = int(min(int64_t(16), n - e0));
    if (lane < 16) {
        if (lane < nn) {
            double f[9];
            for (int a = 0; a < 9; ++a) f[a] = f9[9 * (e0 + lane) + a];
            closure_inputs<lbt::VSet<3, 2>>(cn, f, rho_ref, xs[lane], rs[lane]);
        } else {
            for (int k = 0; k < 16; ++k) xs[lane][k] = 0.0f;
            rs[lane] = 0.0f;
        }
    }
    __syncthreads();
    closure_mfma16(w, cn, xs, hs, rs, c6);
    for (int q = lane; q < 36 * nn; q += 64) {
        const int node = q / 36, a = q % 36, k = a / 6, m = a % 6;
        const int mi = missing_index(k, m);
        c36[36 * (e0 + node) + a] = mi >= 0 ? double(c6[node][mi]) : 0.0;
    }
}

int blocks(int64_t n, int t = 256) { return int((n + t - 1) / t); }

// the three dense layers of the forward pass; H1, H2 hold n x 64 floats each
void forward_launch(const float *params, const float *x, float *y, int64_t n, float *H1, float *H2, hipStream_t s) {
    const float *W1 = params, *b1 = params + MLP_OFF_B1, *W2 = params + MLP_OFF_W2, *b2 = params + MLP_OFF_B2;
    const float *W3 = params + MLP_OFF_W3, *b3 = params + MLP_OFF_B3;
    hipLaunchKernelGGL(k_dense, dim3(blocks(n * 64)), dim3(256), 0, s, x, 10, W1, b1, H1, 64, n, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(n * 64)), dim3(256), 0, s, H1, 64, W2, b2, H2, 64, n, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(n * 8)), dim3(256), 0, s, H2, 64, W3, b3, y, 8, n, 0);
}

}  // namespace

// Hidden activations of the allocation-free forward pass: two layers of
// LB_MLP_NOALLOC_MAX_N x 64 floats (8 MiB), one copy per GPU for the life of
// the process.  Host code never uses this name as an address: the device
// address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) float scratch[2 * 64 * LB_MLP_NOALLOC_MAX_N];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up once per
// device with that device current (nullptr on failure, error text set)
float *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        lb_internal_fail(LB_EDEVICE, "no current HIP device for the allocation-free forward pass");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            lb_internal_fail(LB_EDEVICE, "hipGetSymbolAddress of the forward-pass scratch array failed");
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

namespace lbk {
void launch_to_bf16(const float *p, uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(MLP_NPARAM)), dim3(256), 0, s, p, out, MLP_NPARAM);
}
}  // namespace lbk

extern "C" {

int64_t lb_mlp_param_count(void) { return MLP_NPARAM; }

size_t lb_mlp_workspace_bytes(int64_t n) { return size_t(n > 0 ? n : 0) * 273 * 4 + 256; }

lb_status lb_mlp_forward(const float *params, const float *x, float *y, int64_t n, void *ws, void *stream) {
    if (!params || !x || !y || !ws || n < 0) return lb_internal_fail(LB_EINVAL, "bad argument");
    if (n == 0) return LB_OK;
    float *H1 = reinterpret_cast<float *>(ws), *H2 = H1 + n * 64;
    forward_launch(params, x, y, n, H1, H2, reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? LB_OK : lb_internal_fail(LB_EDEVICE, "mlp forward launch failed");
}

lb_status lb_mlp_forward_noalloc(const float *params, const float *x, float *y, int64_t n, void *stream) {
    if (!params || !x || !y || n < 0) return lb_internal_fail(LB_EINVAL, "bad argument");
    if (n > LB_MLP_NOALLOC_MAX_N)
        return lb_internal_fail(LB_EINVAL, "batch above LB_MLP_NOALLOC_MAX_N (16384 rows) for the allocation-free "
                                           "forward pass; use lb_mlp_forward with a workspace");
    if (n == 0) return LB_OK;
    float *base = scratch_on_current_device();
    if (!base) return LB_EDEVICE;
    // every hidden value is written by its layer before the next layer
    // reads it, so nothing in the array has to start at zero
    forward_launch(params, x, y, n, base, base + 64 * LB_MLP_NOALLOC_MAX_N, reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? LB_OK : lb_internal_fail(LB_EDEVICE, "mlp forward launch failed");
}

lb_status lb_mlp_loss_grad(const float *params, const float *x, const float *t, const int32_t *flag, int64_t n,
                           float *grad, float *loss, void *ws, void *stream) {
    if (!params || !x || !t || !flag || !grad || !loss || !ws || n <= 0)
        return lb_internal_fail(LB_EINVAL, "bad argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *H1 = reinterpret_cast<float *>(ws), *H2 = H1 + n * 64, *Y = H2 + n * 64, *dY = Y + n * 8;
    float *dZ2 = dY + n * 8, *dZ1 = dZ2 + n * 64, *lv = dZ1 + n * 64;
    const float *W1 = params, *b1 = params + MLP_OFF_B1, *W2 = params + MLP_OFF_W2, *b2 = params + MLP_OFF_B2;
    const float *W3 = params + MLP_OFF_W3, *b3 = params + MLP_OFF_B3;
    hipLaunchKernelGGL(k_dense, dim3(blocks(n * 64)), dim3(256), 0, s, x, 10, W1, b1, H1, 64, n, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(n * 64)), dim3(256), 0, s, H1, 64, W2, b2, H2, 64, n, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(n * 8)), dim3(256), 0, s, H2, 64, W3, b3, Y, 8, n, 0);
    hipLaunchKernelGGL(k_loss, dim3(blocks(n)), dim3(256), 0, s, Y, t, flag, n, dY, lv);
    hipLaunchKernelGGL(k_outer, dim3(8 * 64 + 8), dim3(256), 0, s, dY, 8, H2, 64, n, grad + MLP_OFF_W3,
                       grad + MLP_OFF_B3);
    hipLaunchKernelGGL(k_dense_back, dim3(blocks(n * 64)), dim3(256), 0, s, dY, 8, W3, H2, dZ2, 64, n);
    hipLaunchKernelGGL(k_outer, dim3(64 * 64 + 64), dim3(256), 0, s, dZ2, 64, H1, 64, n, grad + MLP_OFF_W2,
                       grad + MLP_OFF_B2);
    hipLaunchKernelGGL(k_dense_back, dim3(blocks(n * 64)), dim3(256), 0, s, dZ2, 64, W2, H1, dZ1, 64, n);
    hipLaunchKernelGGL(k_outer, dim3(64 * 10 + 64), dim3(256), 0, s, dZ1, 64, x, 10, n, grad,
                       grad + MLP_OFF_B1);
    hipLaunchKernelGGL(k_mean1, dim3(1), dim3(256), 0, s, lv, n, loss);
    return hipGetLastError() == hipSuccess ? LB_OK : lb_internal_fail(LB_EDEVICE, "mlp gradient launch failed");
}

lb_status lb_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, float lr, void *stream) {
    if (!params || !grad || !m || !v || step < 1) return lb_internal_fail(LB_EINVAL, "bad argument");
    const float bc1 = 1.0f - powf(0.9f, float(step)), bc2 = 1.0f - powf(0.999f, float(step));
    hipLaunchKernelGGL(k_adam, dim3(blocks(MLP_NPARAM)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), params,
                       grad, m, v, int64_t(MLP_NPARAM), lr, bc1, bc2);
    return hipGetLastError() == hipSuccess ? LB_OK : lb_internal_fail(LB_EDEVICE, "adam launch failed");
}

lb_status lb_closure_eval(const float *params, const float *norm, double kn_ref, int32_t tau_rho, double rho_ref,
                          const double *f9, int64_t n, double *c36, void *stream) {
    if (!params || !norm || !f9 || !c36 || n < 0) return lb_internal_fail(LB_EINVAL, "bad argument");
    lbi::ClosureNorm cn{};
    for (int k = 0; k < 10; ++k) {
        cn.xmean[k] = norm[k];
        cn.xstd[k] = norm[10 + k];
    }
    for (int k = 0; k < 6; ++k) {
        cn.tmean[k] = norm[20 + k];
        cn.tstd[k] = norm[26 + k];
    }
    cn.kn_ref = float(kn_ref);
    cn.tau_rho = tau_rho;
    if (n == 0) return LB_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the network's bf16 weights, as lb_set_closure makes them for a lattice
    uint16_t *wb = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&wb), size_t(MLP_NPARAM) * 2, s) != hipSuccess)
        return lb_internal_fail(LB_ENOMEM, "closure weight buffer");
    launch_to_bf16(params, wb, s);
    hipLaunchKernelGGL(k_closure_eval, dim3(unsigned((n + 15) / 16)), dim3(64), 0, s, wb, cn, f9, n, c36, rho_ref);
    const bool ok = hipGetLastError() == hipSuccess;
    (void)hipFreeAsync(wb, s);
    return ok ? LB_OK : lb_internal_fail(LB_EDEVICE, "closure launch failed");
}

}  // extern "C"
