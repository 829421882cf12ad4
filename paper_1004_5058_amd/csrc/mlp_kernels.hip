// HIP kernels and C ABI (include/mlp.h) of the flow-curve surrogate network:
// a 3 -> 64 -> 64 -> 1 tanh multilayer perceptron trained by full-batch Adam.
//
// One wavefront evaluates one training row at a time with lane j owning hidden
// unit j of both layers: the 64-wide layers map one-to-one onto the 64-lane
// wavefront, the weights sit in LDS (W2 in both orientations so that the
// forward and the backward contraction read consecutive addresses), and each
// lane keeps the gradient of its own row of W2 in registers across the rows
// the wave processes.  Per-wave partial gradients go to global memory and a
// second kernel reduces them in a fixed order and applies Adam, so training
// is deterministic.  The network is small (4481 parameters, a few MFLOP per
// epoch): it is latency-bound and uses no matrix cores.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mlp.h"

namespace mlpk {

constexpr int H = 64;
constexpr int NP = MLP_NPARAM;
constexpr int NPL = NP + 1;           // partial row: gradient + loss
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + 3 * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H;
constexpr int WAVES = 4;               // wavefronts per block
constexpr int RPB = 32;                // rows per block

struct Norm {
    float in_mean[3], in_std[3], out_mean, out_std;
};

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct Lds {
    float w1[3 * H], b1[H], w2[H * H], w2t[H * H], b2[H], w3[H], b3;
    float a1[WAVES][H], d2[WAVES][H];
};

__device__ void load_params(Lds& L, const float* __restrict__ th)
{
    for (int i = threadIdx.x; i < 3 * H; i += blockDim.x) L.w1[i] = th[OFF_W1 + i];
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) {
        const float w = th[OFF_W2 + i];
        L.w2[i] = w;
        L.w2t[(i % H) * H + i / H] = w;
    }
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        L.b1[i] = th[OFF_B1 + i];
        L.b2[i] = th[OFF_B2 + i];
        L.w3[i] = th[OFF_W3 + i];
    }
    if (threadIdx.x == 0) L.b3 = th[OFF_B3];
    __syncthreads();
}

// Forward pass of one row by one wave: lane j returns a1_j, a2_j; all lanes
// return the standardised output.
__device__ __forceinline__ float forward_row(Lds& L, int w, int j, const float xs[3], float& a1, float& a2)
{
    const float z1 = L.w1[3 * j] * xs[0] + L.w1[3 * j + 1] * xs[1] + L.w1[3 * j + 2] * xs[2] + L.b1[j];
    a1 = tanhf(z1);
    L.a1[w][j] = a1;
    __builtin_amdgcn_wave_barrier();
    float z2 = L.b2[j];
#pragma unroll 16
    for (int k = 0; k < H; ++k) z2 += L.w2t[k * H + j] * L.a1[w][k];
    a2 = tanhf(z2);
    return wave_sum(L.w3[j] * a2) + L.b3;
}

// Forward + backward over the rows of this block; each wave writes its own
// partial gradient (and loss sum) row.
__global__ void __launch_bounds__(64 * WAVES)
k_fwdbwd(const float* __restrict__ th, Norm nm, const float* __restrict__ X, const float* __restrict__ Y,
         int n, float* __restrict__ part)
{
    __shared__ Lds L;
    load_params(L, th);
    const int w = threadIdx.x / 64, j = threadIdx.x % 64;
    float gw2[H];
#pragma unroll
    for (int k = 0; k < H; ++k) gw2[k] = 0.f;
    float gw1[3] = {0.f, 0.f, 0.f}, gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
    const float inv_n = 1.0f / (float)n;
    const int r0 = blockIdx.x * RPB, r1 = min(r0 + RPB, n);
    for (int r = r0 + w; r < r1; r += WAVES) {
        float xs[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) xs[c] = (X[3 * r + c] - nm.in_mean[c]) / nm.in_std[c];
        const float ys = (Y[r] - nm.out_mean) / nm.out_std;
        float a1, a2;
        const float out = forward_row(L, w, j, xs, a1, a2);
        const float res = out - ys;
        lsum += res * res;
        const float d = 2.0f * res * inv_n;
        gw3 += d * a2;
        gb3 += d;
        const float d2 = d * L.w3[j] * (1.0f - a2 * a2);
        gb2 += d2;
#pragma unroll
        for (int k = 0; k < H; ++k) gw2[k] += d2 * L.a1[w][k];
        L.d2[w][j] = d2;
        __builtin_amdgcn_wave_barrier();
        float s = 0.f;
#pragma unroll 16
        for (int jj = 0; jj < H; ++jj) s += L.w2[jj * H + j] * L.d2[w][jj];
        const float d1 = s * (1.0f - a1 * a1);
        gb1 += d1;
#pragma unroll
        for (int c = 0; c < 3; ++c) gw1[c] += d1 * xs[c];
        __builtin_amdgcn_wave_barrier();
    }
    float* out = part + (size_t)(blockIdx.x * WAVES + w) * NPL;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[OFF_W1 + 3 * j + c] = gw1[c];
    out[OFF_B1 + j] = gb1;
#pragma unroll
    for (int k = 0; k < H; ++k) out[OFF_W2 + j * H + k] = gw2[k];
    out[OFF_B2 + j] = gb2;
    out[OFF_W3 + j] = gw3;
    if (j == 0) {
        out[OFF_B3] = gb3;
        out[NP] = lsum;
    }
}

// Sum of the partial rows in a fixed order; optional Adam update.
__global__ void __launch_bounds__(256)
k_reduce_adam(const float* __restrict__ part, int nparts, float* __restrict__ th, float* __restrict__ m,
              float* __restrict__ v, float* __restrict__ gout, float* __restrict__ loss_out, float inv_n,
              int update, float lr, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NP) return;
    float g = 0.f;
    for (int b = 0; b < nparts; ++b) g += part[(size_t)b * NPL + p];
    if (p == NP) {
        *loss_out = g * inv_n;
        return;
    }
    gout[p] = g;
    if (update) {
        const float mm = 0.9f * m[p] + 0.1f * g;
        const float vv = 0.999f * v[p] + 0.001f * g * g;
        m[p] = mm;
        v[p] = vv;
        th[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
    }
}

__global__ void __launch_bounds__(64 * WAVES)
k_infer(const float* __restrict__ th, Norm nm, const float* __restrict__ X, int n, float* __restrict__ Y)
{
    __shared__ Lds L;
    load_params(L, th);
    const int w = threadIdx.x / 64, j = threadIdx.x % 64;
    const int r0 = blockIdx.x * RPB, r1 = min(r0 + RPB, n);
    for (int r = r0 + w; r < r1; r += WAVES) {
        float xs[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) xs[c] = (X[3 * r + c] - nm.in_mean[c]) / nm.in_std[c];
        float a1, a2;
        const float out = forward_row(L, w, j, xs, a1, a2);
        if (j == 0) Y[r] = out * nm.out_std + nm.out_mean;
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace mlpk

// ---------------------------------------------------------------- runtime --

// The library's thread-local error message (lb_last_error), set in lb_capi.hip.
void lbi_set_error(const char* msg);

namespace {

lb_status mfail(lb_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    lbi_set_error(buf);
    return code;
}

size_t al(size_t v) { return (v + 255) / 256 * 256; }

struct MLayout {
    size_t th, m, v, g, loss, X, Y, Xi, Yi, part, total;
};

MLayout mlayout(int rows)
{
    MLayout L;
    const int nb = (rows + mlpk::RPB - 1) / mlpk::RPB;
    size_t o = 0;
    L.th = o; o += al(sizeof(float) * mlpk::NP);
    L.m = o; o += al(sizeof(float) * mlpk::NP);
    L.v = o; o += al(sizeof(float) * mlpk::NP);
    L.g = o; o += al(sizeof(float) * mlpk::NP);
    L.loss = o; o += al(sizeof(float));
    L.X = o; o += al(sizeof(float) * 3 * rows);
    L.Y = o; o += al(sizeof(float) * rows);
    L.Xi = o; o += al(sizeof(float) * 3 * rows);
    L.Yi = o; o += al(sizeof(float) * rows);
    L.part = o; o += al(sizeof(float) * (size_t)nb * mlpk::WAVES * mlpk::NPL);
    L.total = o;
    return L;
}

}  // namespace


struct mlp_handle {
    char* base = nullptr;
    MLayout lay;
    int max_rows = 0, n = 0;
    long long t = 0;    // Adam step count
    hipStream_t stream = nullptr;
    mlpk::Norm norm;
    float* p(size_t off) { return (float*)(base + off); }
};

#define MHIP(call)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return mfail(LB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace {

lb_status fill_zero(mlp_handle* h, size_t off, size_t count)
{
    std::vector<float> z(count, 0.f);
    MHIP(hipMemcpyAsync(h->p(off), z.data(), count * sizeof(float), hipMemcpyHostToDevice, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

// One forward/backward over the uploaded data; optionally one Adam step.
lb_status fwdbwd(mlp_handle* h, bool update, float lr)
{
    if (h->n < 1) return mfail(LB_ESTATE, "no training data uploaded (mlp_set_data)");
    const int nb = (h->n + mlpk::RPB - 1) / mlpk::RPB;
    hipLaunchKernelGGL(mlpk::k_fwdbwd, dim3(nb), dim3(64 * mlpk::WAVES), 0, h->stream, h->p(h->lay.th), h->norm,
                       h->p(h->lay.X), h->p(h->lay.Y), h->n, h->p(h->lay.part));
    MHIP(hipGetLastError());
    float c1 = 1.f, c2 = 1.f;
    if (update) {
        h->t += 1;
        c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)h->t)));
        c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)h->t)));
    }
    const int threads = 256, blocks = (mlpk::NPL + threads - 1) / threads;
    hipLaunchKernelGGL(mlpk::k_reduce_adam, dim3(blocks), dim3(threads), 0, h->stream, h->p(h->lay.part),
                       nb * mlpk::WAVES, h->p(h->lay.th), h->p(h->lay.m), h->p(h->lay.v), h->p(h->lay.g),
                       h->p(h->lay.loss), 1.0f / (float)h->n, update ? 1 : 0, lr, c1, c2);
    MHIP(hipGetLastError());
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status mlp_state_bytes(int32_t max_rows, size_t* bytes)
{
    if (!bytes || max_rows < 1 || max_rows > (1 << 22)) return mfail(LB_EINVAL, "max_rows must be in [1, 2^22]");
    *bytes = mlayout(max_rows).total;
    return LB_OK;
}

lb_status mlp_init(void* dev_state, size_t bytes, int32_t max_rows, void* stream, mlp_handle** out)
{
    if (!out) return mfail(LB_EINVAL, "null output handle");
    *out = nullptr;
    size_t need = 0;
    lb_status st = mlp_state_bytes(max_rows, &need);
    if (st != LB_OK) return st;
    if (!dev_state || ((uintptr_t)dev_state) % 256) return mfail(LB_EINVAL, "device state must be 256-byte aligned");
    if (bytes < need) return mfail(LB_ENOMEM, "device state of %zu bytes is smaller than the %zu required", bytes, need);
    mlp_handle* h = new (std::nothrow) mlp_handle();
    if (!h) return mfail(LB_ENOMEM, "host allocation failed");
    h->base = (char*)dev_state;
    h->lay = mlayout(max_rows);
    h->max_rows = max_rows;
    h->stream = (hipStream_t)stream;
    for (int c = 0; c < 3; ++c) { h->norm.in_mean[c] = 0.f; h->norm.in_std[c] = 1.f; }
    h->norm.out_mean = 0.f;
    h->norm.out_std = 1.f;
    st = fill_zero(h, 0, h->lay.Y / sizeof(float));
    if (st != LB_OK) { delete h; return st; }
    *out = h;
    return LB_OK;
}

lb_status mlp_set_params(mlp_handle* h, const float* theta)
{
    if (!h || !theta) return mfail(LB_EINVAL, "null argument");
    for (int i = 0; i < mlpk::NP; ++i)
        if (!std::isfinite(theta[i])) return mfail(LB_EINVAL, "non-finite parameter %d", i);
    MHIP(hipMemcpyAsync(h->p(h->lay.th), theta, sizeof(float) * mlpk::NP, hipMemcpyHostToDevice, h->stream));
    h->t = 0;
    lb_status st = fill_zero(h, h->lay.m, mlpk::NP);
    if (st != LB_OK) return st;
    return fill_zero(h, h->lay.v, mlpk::NP);
}

lb_status mlp_get_params(mlp_handle* h, float* theta)
{
    if (!h || !theta) return mfail(LB_EINVAL, "null argument");
    MHIP(hipMemcpyAsync(theta, h->p(h->lay.th), sizeof(float) * mlpk::NP, hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status mlp_set_norm(mlp_handle* h, const float in_mean[3], const float in_std[3], float out_mean, float out_std)
{
    if (!h || !in_mean || !in_std) return mfail(LB_EINVAL, "null argument");
    for (int c = 0; c < 3; ++c)
        if (!(in_std[c] > 0.f) || !std::isfinite(in_mean[c])) return mfail(LB_EINVAL, "bad input standardisation");
    if (!(out_std > 0.f) || !std::isfinite(out_mean)) return mfail(LB_EINVAL, "bad output standardisation");
    for (int c = 0; c < 3; ++c) { h->norm.in_mean[c] = in_mean[c]; h->norm.in_std[c] = in_std[c]; }
    h->norm.out_mean = out_mean;
    h->norm.out_std = out_std;
    return LB_OK;
}

lb_status mlp_set_data(mlp_handle* h, const float* X, const float* y, int32_t n)
{
    if (!h || !X || !y) return mfail(LB_EINVAL, "null argument");
    if (n < 1 || n > h->max_rows) return mfail(LB_EINVAL, "row count %d outside [1, %d]", n, h->max_rows);
    for (int i = 0; i < 3 * n; ++i)
        if (!std::isfinite(X[i])) return mfail(LB_EINVAL, "non-finite input");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(y[i])) return mfail(LB_EINVAL, "non-finite target");
    MHIP(hipMemcpyAsync(h->p(h->lay.X), X, sizeof(float) * 3 * n, hipMemcpyHostToDevice, h->stream));
    MHIP(hipMemcpyAsync(h->p(h->lay.Y), y, sizeof(float) * n, hipMemcpyHostToDevice, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    h->n = n;
    return LB_OK;
}

lb_status mlp_loss_grad(mlp_handle* h, float* loss, float* grad)
{
    if (!h) return mfail(LB_EINVAL, "null handle");
    lb_status st = fwdbwd(h, false, 0.f);
    if (st != LB_OK) return st;
    if (loss) MHIP(hipMemcpyAsync(loss, h->p(h->lay.loss), sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (grad) MHIP(hipMemcpyAsync(grad, h->p(h->lay.g), sizeof(float) * mlpk::NP, hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status mlp_train(mlp_handle* h, int32_t iters, float lr, float* loss)
{
    if (!h) return mfail(LB_EINVAL, "null handle");
    if (iters < 0 || !(lr > 0.f) || !std::isfinite(lr)) return mfail(LB_EINVAL, "need iters >= 0 and lr > 0");
    for (int k = 0; k < iters; ++k) {
        lb_status st = fwdbwd(h, true, lr);
        if (st != LB_OK) return st;
    }
    if (loss) MHIP(hipMemcpyAsync(loss, h->p(h->lay.loss), sizeof(float), hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status mlp_infer(mlp_handle* h, const float* X, int32_t n, float* y)
{
    if (!h || !X || !y) return mfail(LB_EINVAL, "null argument");
    if (n < 1 || n > h->max_rows) return mfail(LB_EINVAL, "row count %d outside [1, %d]", n, h->max_rows);
    MHIP(hipMemcpyAsync(h->p(h->lay.Xi), X, sizeof(float) * 3 * n, hipMemcpyHostToDevice, h->stream));
    const int nb = (n + mlpk::RPB - 1) / mlpk::RPB;
    hipLaunchKernelGGL(mlpk::k_infer, dim3(nb), dim3(64 * mlpk::WAVES), 0, h->stream, h->p(h->lay.th), h->norm,
                       h->p(h->lay.Xi), n, h->p(h->lay.Yi));
    MHIP(hipGetLastError());
    MHIP(hipMemcpyAsync(y, h->p(h->lay.Yi), sizeof(float) * n, hipMemcpyDeviceToHost, h->stream));
    MHIP(hipStreamSynchronize(h->stream));
    return LB_OK;
}

lb_status mlp_destroy(mlp_handle* h)
{
    delete h;
    return LB_OK;
}

}  // extern "C"
