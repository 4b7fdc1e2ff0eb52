// qg_mlp.hip -- the fusion cost model: an MLP with three ReLU hidden layers of
// width H (64), FP32, trained with mean-squared error and Adam, run by these
// kernels.  It predicts the log run time of a candidate pass from its features.
//
// Flat parameter layout: W1[F][H], b1[H], W2[H][H], b2[H], W3[H][H], b3[H],
// W4[H], b4.  Forward: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),
// h3 = relu(h2 W3 + b3), y = h3 . W4 + b4.  All batch reductions run in sample
// order, so results are deterministic.
#include "qg_kernels.h"

namespace qg {
namespace {

constexpr int H = kMlpHidden;

struct Offs {
    int w1, b1, w2, b2, w3, b3, w4, b4, total;
};

__host__ __device__ inline Offs offs(int F) {
    Offs o;
    o.w1 = 0;
    o.b1 = o.w1 + F * H;
    o.w2 = o.b1 + H;
    o.b2 = o.w2 + H * H;
    o.w3 = o.b2 + H;
    o.b3 = o.w3 + H * H;
    o.w4 = o.b3 + H;
    o.b4 = o.w4 + H;
    o.total = o.b4 + 1;
    return o;
}

// zout = relu(zin) W + b for one sample (H x H layer).
__device__ __forceinline__ void layer(const float *__restrict__ W, const float *__restrict__ b,
                                      const float *__restrict__ zin, float *__restrict__ zout) {
    float acc[H];
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = b[j];
    for (int i = 0; i < H; ++i) {
        const float x = fmaxf(zin[i], 0.f);
#pragma unroll
        for (int j = 0; j < H; ++j) acc[j] = fmaf(x, W[i * H + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < H; ++j) zout[j] = acc[j];
}

// One thread per sample; pre-activations z1, z2, z3 [B][H] are stored (the
// next layer reads its input back from them, so only the output row lives in
// registers).
__global__ void __launch_bounds__(256)
k_fwd(const float *__restrict__ th, const float *__restrict__ X, int B, int F, float *__restrict__ z1,
      float *__restrict__ z2, float *__restrict__ z3, float *__restrict__ y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const Offs o = offs(F);
    float acc[H];
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = th[o.b1 + j];
    for (int i = 0; i < F; ++i) {
        const float x = X[(int64_t)s * F + i];
#pragma unroll
        for (int j = 0; j < H; ++j) acc[j] = fmaf(x, th[o.w1 + i * H + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < H; ++j) z1[(int64_t)s * H + j] = acc[j];
    layer(th + o.w2, th + o.b2, z1 + (int64_t)s * H, z2 + (int64_t)s * H);
    layer(th + o.w3, th + o.b3, z2 + (int64_t)s * H, z3 + (int64_t)s * H);
    float out = th[o.b4];
    for (int j = 0; j < H; ++j) out = fmaf(fmaxf(z3[(int64_t)s * H + j], 0.f), th[o.w4 + j], out);
    y[s] = out;
}

// dY = 2 (y - t) / B; loss_acc[slot] += mean (y - t)^2 (single block, fixed order).
__global__ void __launch_bounds__(256)
k_loss(const float *__restrict__ y, const float *__restrict__ t, int B, float *__restrict__ dy,
       double *__restrict__ loss_acc, int slot) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int s = threadIdx.x; s < B; s += blockDim.x) {
        const float d = y[s] - t[s];
        dy[s] = 2.f * d / (float)B;
        acc += (double)d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss_acc) loss_acc[slot] += red[0] / B;
}

// dzin_i = (sum_j dzout_j W[i][j]) if zin_i > 0 else 0, for one sample.
__device__ __forceinline__ void back_layer(const float *__restrict__ W, const float *__restrict__ dzout,
                                           const float *__restrict__ zin, float *__restrict__ dzin) {
    float d[H];
#pragma unroll
    for (int j = 0; j < H; ++j) d[j] = dzout[j];
    for (int i = 0; i < H; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < H; ++j) acc = fmaf(d[j], W[i * H + j], acc);
        dzin[i] = zin[i] > 0.f ? acc : 0.f;
    }
}

// One thread per sample: dz3, dz2, dz1 [B][H].
__global__ void __launch_bounds__(256)
k_bwd_act(const float *__restrict__ th, int B, int F, const float *__restrict__ z1, const float *__restrict__ z2,
          const float *__restrict__ z3, const float *__restrict__ dy, float *__restrict__ dz1,
          float *__restrict__ dz2, float *__restrict__ dz3) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const Offs o = offs(F);
    const float g = dy[s];
    const int64_t r = (int64_t)s * H;
    for (int j = 0; j < H; ++j) dz3[r + j] = z3[r + j] > 0.f ? g * th[o.w4 + j] : 0.f;
    back_layer(th + o.w3, dz3 + r, z2 + r, dz2 + r);
    back_layer(th + o.w2, dz2 + r, z1 + r, dz1 + r);
}

// One thread per parameter: sum over samples in order.
__global__ void __launch_bounds__(256)
k_bwd_w(const float *__restrict__ X, int B, int F, const float *__restrict__ z1, const float *__restrict__ z2,
        const float *__restrict__ z3, const float *__restrict__ dz1, const float *__restrict__ dz2,
        const float *__restrict__ dz3, const float *__restrict__ dy, float *__restrict__ grad) {
    const Offs o = offs(F);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= o.total) return;
    float acc = 0.f;
    if (p < o.b1) {  // W1[i][j] = sum_s x[s][i] dz1[s][j]
        const int i = p / H, j = p % H;
        for (int s = 0; s < B; ++s) acc = fmaf(X[(int64_t)s * F + i], dz1[(int64_t)s * H + j], acc);
    } else if (p < o.w2) {
        const int j = p - o.b1;
        for (int s = 0; s < B; ++s) acc += dz1[(int64_t)s * H + j];
    } else if (p < o.b2) {  // W2[i][j] = sum_s relu(z1[s][i]) dz2[s][j]
        const int i = (p - o.w2) / H, j = (p - o.w2) % H;
        for (int s = 0; s < B; ++s) acc = fmaf(fmaxf(z1[(int64_t)s * H + i], 0.f), dz2[(int64_t)s * H + j], acc);
    } else if (p < o.w3) {
        const int j = p - o.b2;
        for (int s = 0; s < B; ++s) acc += dz2[(int64_t)s * H + j];
    } else if (p < o.b3) {
        const int i = (p - o.w3) / H, j = (p - o.w3) % H;
        for (int s = 0; s < B; ++s) acc = fmaf(fmaxf(z2[(int64_t)s * H + i], 0.f), dz3[(int64_t)s * H + j], acc);
    } else if (p < o.w4) {
        const int j = p - o.b3;
        for (int s = 0; s < B; ++s) acc += dz3[(int64_t)s * H + j];
    } else if (p < o.b4) {
        const int j = p - o.w4;
        for (int s = 0; s < B; ++s) acc = fmaf(fmaxf(z3[(int64_t)s * H + j], 0.f), dy[s], acc);
    } else {
        for (int s = 0; s < B; ++s) acc += dy[s];
    }
    grad[p] = acc;
}

__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    th[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather(const float *__restrict__ X, const float *__restrict__ T, const int32_t *__restrict__ idx,
                         int B, int F, float *__restrict__ Xb, float *__restrict__ Tb) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const int r = idx[s];
    for (int i = 0; i < F; ++i) Xb[(int64_t)s * F + i] = X[(int64_t)r * F + i];
    Tb[s] = T[r];
}

inline dim3 blocks(int n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

int mlp_param_count(int n_in) { return offs(n_in).total; }

hipError_t launch_mlp_forward(const float *th, const float *X, int B, int F, float *z1, float *z2, float *z3, float *y,
                              hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd, blocks(B), dim3(256), 0, st, th, X, B, F, z1, z2, z3, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *th, const float *X, const float *T, int B, int F, float *z1, float *z2,
                           float *z3, float *y, float *dy, float *dz1, float *dz2, float *dz3, float *grad,
                           double *loss_acc, int loss_slot, hipStream_t st) {
    if (B <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fwd, blocks(B), dim3(256), 0, st, th, X, B, F, z1, z2, z3, y);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, y, T, B, dy, loss_acc, loss_slot);
    hipLaunchKernelGGL(k_bwd_act, blocks(B), dim3(256), 0, st, th, B, F, z1, z2, z3, dy, dz1, dz2, dz3);
    hipLaunchKernelGGL(k_bwd_w, blocks(offs(F).total), dim3(256), 0, st, X, B, F, z1, z2, z3, dz1, dz2, dz3, dy, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *th, const float *g, float *m, float *v, int n, float lr, int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, blocks(n), dim3(256), 0, st, th, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_gather(const float *X, const float *T, const int32_t *idx, int B, int F, float *Xb, float *Tb,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_gather, blocks(B), dim3(256), 0, st, X, T, idx, B, F, Xb, Tb);
    return hipGetLastError();
}

}  // namespace qg
