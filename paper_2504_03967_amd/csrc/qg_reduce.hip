// qg_reduce.hip -- reductions of the state: probabilities, Z-string
// expectations, shot sampling, and the adjoint helpers.
//
// All sums are FP64 (for both amplitude precisions) and use a fixed
// association order (per-block partials in index order, butterfly wave sums,
// then a sequential sum over blocks), so repeated calls are bitwise identical.
#include <mutex>

#include "qg_kernels.h"

namespace qg {
namespace {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename C>
__device__ __forceinline__ double prob(C v) {
    const double x = v.x, y = v.y;
    return x * x + y * y;
}

__device__ __forceinline__ int popc(uint32_t x) { return __popc(x); }
__device__ __forceinline__ int popc(uint64_t x) { return __popcll(x); }

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int kThreads = 256;

inline uint32_t grid_for(uint64_t work, uint64_t per_block, uint32_t cap = 65536) {
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

// ------------------------------------------------------------- state init

template <typename R>
__global__ void k_zero_state(typename V2<R>::T *psi, uint64_t dim) {
    using C = typename V2<R>::T;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        C v;
        v.x = i == 0 ? (R)1 : (R)0;
        v.y = (R)0;
        psi[i] = v;
    }
}

// ----------------------------------------------------------------- probs

template <typename R>
__global__ void k_probs(const typename V2<R>::T *__restrict__ psi, uint64_t dim,
                        const uint64_t *__restrict__ idx, int64_t n, double *__restrict__ out) {
    const uint64_t cnt = idx ? (uint64_t)n : dim;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < cnt;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = idx ? idx[k] : k;
        out[k] = prob(psi[i]);
    }
}

// ---------------------------------------------------------------- expval

// Masks evaluated per read of the state (1, 4, 16 or 64 at a time).
constexpr int kTermsPerPass = 64;
// A group is 16 x kThreads consecutive amplitudes: thread t holds index bits
// 0..7 = t and 16 rows j (index bits 8..11); the bits above are uniform over
// the block.
constexpr int kGroupRows = 16;
constexpr uint64_t kGroup = (uint64_t)kGroupRows * kThreads;

inline int expval_blocks(uint64_t dim) {
    uint64_t b = dim / kGroup;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

// <Z_m> restricted to a block's chunk, for TM masks per read.  With i = g | j << 8 | t
// (g the group's high bits), (-1)^{popcount(i & m)} factors into a thread sign
// (bits 0..7), a row sign (bits 8..11) and a group sign.  Per group each thread
// takes the Walsh-Hadamard transform W_k = sum_j (-1)^{popcount(j & k)} p_j of
// its 16 probabilities; mask m then adds (group sign) * W_{(m >> 8) & 15}, with
// a uniform index into the thread's registers.  The thread sign is applied once
// at the end.  So the work per amplitude no longer grows with the mask count.
template <typename R, int TM>
__global__ void __launch_bounds__(kThreads)
k_expval_part(const typename V2<R>::T *__restrict__ psi, uint64_t dim, const uint64_t *__restrict__ masks,
              int n_terms, int term0, double *__restrict__ part, int nblocks) {
    __shared__ double red[TM][kThreads / 64];
    const uint32_t tid = threadIdx.x;
    double acc[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) acc[t] = 0.0;
    const uint64_t chunk = (dim + nblocks - 1) / nblocks;
    const uint64_t lo = blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < dim ? lo + chunk : dim;
    for (uint64_t g = lo; g < hi; g += kGroup) {
        double w[kGroupRows];
        if (g + kGroup <= hi) {
#pragma unroll
            for (int j = 0; j < kGroupRows; ++j) w[j] = prob(psi[g + j * kThreads + tid]);
        } else {
#pragma unroll
            for (int j = 0; j < kGroupRows; ++j) {
                const uint64_t i = g + j * kThreads + tid;
                w[j] = i < hi ? prob(psi[i]) : 0.0;
            }
        }
#pragma unroll
        for (int s = 1; s < kGroupRows; s <<= 1)
#pragma unroll
            for (int j = 0; j < kGroupRows; ++j)
                if (!(j & s)) {
                    const double a = w[j], b = w[j | s];
                    w[j] = a + b;
                    w[j | s] = a - b;
                }
        const uint64_t gh = g >> 12;
#pragma unroll
        for (int t = 0; t < TM; ++t) {
            const uint64_t m = term0 + t < n_terms ? masks[term0 + t] : 0ull;
            const double v = w[(m >> 8) & (kGroupRows - 1)];
            acc[t] += (__popcll(gh & (m >> 12)) & 1) ? -v : v;
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const uint64_t m = term0 + t < n_terms ? masks[term0 + t] : 0ull;
        const double v = wave_sum((__popc(tid & (uint32_t)m & 0xffu) & 1) ? -acc[t] : acc[t]);
        if (lane == 0) red[t][wave] = v;
    }
    __syncthreads();
    if (tid < TM && term0 + (int)tid < n_terms) {
        double so = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) so += red[tid][w];
        part[(int64_t)(term0 + tid) * nblocks + blockIdx.x] = so;
    }
}

__global__ void k_expval_final(const double *__restrict__ part, int nblocks, int n_terms,
                               const double *__restrict__ coeff, double *__restrict__ terms,
                               double *__restrict__ out_terms, double *__restrict__ out_sum) {
    for (int t = threadIdx.x; t < n_terms; t += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += part[(int64_t)t * nblocks + b];
        terms[t] = s;
        if (out_terms) out_terms[t] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0 && out_sum) {
        double s = 0.0;
        for (int t = 0; t < n_terms; ++t) s += coeff[t] * terms[t];
        *out_sum = s;
    }
}

// ---------------------------------------------------------------- sampling

constexpr int kFan = 64;
constexpr int kMaxLevels = 8;

struct Levels {
    int n;                       // stored levels (level 1..n); level 0 = amplitudes
    uint64_t size[kMaxLevels + 1];
    int64_t off[kMaxLevels + 1];  // offset of level l (l >= 1) in the tree buffer
};

Levels make_levels(uint64_t dim) {
    Levels L{};
    L.size[0] = dim;
    int64_t off = 0;
    uint64_t s = dim;
    while (s > (uint64_t)kFan) {
        s = (s + kFan - 1) / kFan;
        ++L.n;
        L.size[L.n] = s;
        L.off[L.n] = off;
        off += (int64_t)s;
    }
    return L;
}

// One wave per kLeafNodes consecutive nodes: node j of the output = sum of
// probabilities [64 j, 64 j + 64); all loads of a lane are issued together.
constexpr int kLeafNodes = 8;

template <typename R>
__global__ void k_tree_leaf(const typename V2<R>::T *__restrict__ psi, uint64_t dim, double *__restrict__ out,
                            uint64_t nout) {
    using C = typename V2<R>::T;
    const uint64_t wave_id = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const uint64_t node0 = wave_id * kLeafNodes;
    if (node0 >= nout) return;  // whole waves exit together (blockDim is a multiple of 64)
    C v[kLeafNodes];
#pragma unroll
    for (int k = 0; k < kLeafNodes; ++k) {
        const uint64_t i = (node0 + k) * kFan + lane;
        if (i < dim) v[k] = psi[i];
        else {
            v[k].x = (R)0;
            v[k].y = (R)0;
        }
    }
#pragma unroll
    for (int k = 0; k < kLeafNodes; ++k) {
        const double s = wave_sum(prob(v[k]));
        if (lane == 0 && node0 + k < nout) out[node0 + k] = s;
    }
}

__global__ void k_tree_up(const double *__restrict__ in, uint64_t nin, double *__restrict__ out, uint64_t nout) {
    const uint64_t node = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (node >= nout) return;
    const uint64_t i = node * kFan + lane;
    double v = i < nin ? in[i] : 0.0;
    v = wave_sum(v);
    if (lane == 0) out[node] = v;
}

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint64_t philox_word(uint64_t seed, uint64_t ctr) {
    uint32_t c0 = (uint32_t)ctr, c1 = (uint32_t)(ctr >> 32), c2 = 0, c3 = 0;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return ((uint64_t)c1 << 32) | c0;
}

template <typename R>
__global__ void k_sample(const typename V2<R>::T *__restrict__ psi, const double *__restrict__ tree, Levels L,
                         uint64_t seed, int64_t shots, uint64_t *__restrict__ out) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= shots) return;
    auto val = [&](int lev, uint64_t k) -> double {
        return lev == 0 ? prob(psi[k]) : tree[L.off[lev] + k];
    };
    const int top = L.n;
    double total = 0.0;
    for (uint64_t k = 0; k < L.size[top]; ++k) total += val(top, k);
    const double u = (double)(philox_word(seed, (uint64_t)s) >> 11) * (1.0 / 9007199254740992.0);
    double r = u * total;
    uint64_t base = 0;
    uint64_t cnt = L.size[top];
    uint64_t pick = 0;
    for (int lev = top; lev >= 0; --lev) {
        double acc = 0.0;
        int64_t found = -1, last_nz = -1;
        for (uint64_t k = 0; k < cnt; ++k) {
            const double x = val(lev, base + k);
            if (x > 0.0) last_nz = (int64_t)k;
            if (acc + x > r) {
                found = (int64_t)k;
                r -= acc;
                break;
            }
            acc += x;
        }
        if (found < 0) {
            // r lies past the rounded sum of these children: take the last non-zero one.
            found = last_nz < 0 ? 0 : last_nz;
            r = val(lev, base + (uint64_t)found);
        }
        pick = base + (uint64_t)found;
        if (lev > 0) {
            base = pick * kFan;
            const uint64_t below = L.size[lev - 1];
            cnt = base + kFan <= below ? kFan : below - base;
        }
    }
    out[s] = pick;
}

// ----------------------------------------------------------------- adjoint

template <typename R>
__global__ void k_apply_observable(const typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam,
                                   uint64_t dim, const uint64_t *__restrict__ masks,
                                   const double *__restrict__ coeff, int n_terms) {
    using C = typename V2<R>::T;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double o = 0.0;
        for (int t = 0; t < n_terms; ++t) o += (__popcll(i & masks[t]) & 1) ? -coeff[t] : coeff[t];
        C v = psi[i], w;
        w.x = (R)(o * v.x);
        w.y = (R)(o * v.y);
        lam[i] = w;
    }
}

// One block of kGradThreads per row: each thread sums a strided quarter of the
// row into four accumulators (independent loads in flight), then waves and the
// block combine in a fixed order, so a row's sum does not depend on timing.
constexpr int kGradThreads = 1024;
__global__ void __launch_bounds__(kGradThreads) k_grad_rows(const double *__restrict__ gpart, int64_t gstride,
                                                            int64_t count, int n_rows, double *__restrict__ rows) {
    __shared__ double wsum[kGradThreads / 64];
    const int r = blockIdx.x;
    const int tid = threadIdx.x;
    if (r >= n_rows) return;
    const double *p = gpart + (int64_t)r * gstride;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t k = tid;
    for (; k + 3 * kGradThreads < count; k += 4 * kGradThreads) {
        s0 += p[k];
        s1 += p[k + kGradThreads];
        s2 += p[k + 2 * kGradThreads];
        s3 += p[k + 3 * kGradThreads];
    }
    for (; k < count; k += kGradThreads) s0 += p[k];
    double s = wave_sum((s0 + s1) + (s2 + s3));
    if ((tid & 63) == 0) wsum[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kGradThreads / 64; ++w) t += wsum[w];
        rows[r] = t;
    }
}

__global__ void k_grad_slots(const double *__restrict__ rows, const int32_t *__restrict__ slot, int n_rows,
                             double *__restrict__ grad, int n_params) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_params) return;
    double g = 0.0;
    for (int r = 0; r < n_rows; ++r)
        if (slot[r] == s) g += rows[r];
    grad[s] = g;
}

}  // namespace

hipError_t launch_zero_state(bool c64, void *psi, uint64_t dim, hipStream_t st) {
    const uint32_t g = grid_for(dim, kThreads * 8, 1 << 20);
    if (c64) hipLaunchKernelGGL(k_zero_state<float>, dim3(g), dim3(kThreads), 0, st, (float2 *)psi, dim);
    else hipLaunchKernelGGL(k_zero_state<double>, dim3(g), dim3(kThreads), 0, st, (double2 *)psi, dim);
    return hipGetLastError();
}

hipError_t launch_probs(bool c64, const void *psi, uint64_t dim, const uint64_t *idx, int64_t n, double *out,
                        hipStream_t st) {
    const uint64_t cnt = idx ? (uint64_t)n : dim;
    if (cnt == 0) return hipSuccess;
    const uint32_t g = grid_for(cnt, kThreads * 4, 1 << 20);
    if (c64) hipLaunchKernelGGL(k_probs<float>, dim3(g), dim3(kThreads), 0, st, (const float2 *)psi, dim, idx, n, out);
    else hipLaunchKernelGGL(k_probs<double>, dim3(g), dim3(kThreads), 0, st, (const double2 *)psi, dim, idx, n, out);
    return hipGetLastError();
}

int64_t expval_partials(uint64_t dim, int n_terms) {
    return (int64_t)n_terms * expval_blocks(dim) + n_terms;
}

hipError_t launch_expval(bool c64, const void *psi, uint64_t dim, const uint64_t *masks, const double *coeff,
                         int n_terms, double *part, double *out_terms, double *out_sum, hipStream_t st) {
    if (n_terms <= 0) return hipSuccess;
    const int nb = expval_blocks(dim);
#define QG_EXPVAL_LAUNCH(TM)                                                                                      \
    do {                                                                                                          \
        if (c64)                                                                                                  \
            hipLaunchKernelGGL((k_expval_part<float, TM>), dim3(nb), dim3(kThreads), 0, st, (const float2 *)psi,   \
                               dim, masks, n_terms, t0, part, nb);                                                \
        else                                                                                                      \
            hipLaunchKernelGGL((k_expval_part<double, TM>), dim3(nb), dim3(kThreads), 0, st, (const double2 *)psi, \
                               dim, masks, n_terms, t0, part, nb);                                                \
    } while (0)
    for (int t0 = 0; t0 < n_terms; t0 += kTermsPerPass) {
        const int left = n_terms - t0;
        if (left <= 1) QG_EXPVAL_LAUNCH(1);
        else if (left <= 4) QG_EXPVAL_LAUNCH(4);
        else if (left <= 16) QG_EXPVAL_LAUNCH(16);
        else QG_EXPVAL_LAUNCH(kTermsPerPass);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
#undef QG_EXPVAL_LAUNCH
    double *terms = part + (int64_t)n_terms * nb;
    hipLaunchKernelGGL(k_expval_final, dim3(1), dim3(kThreads), 0, st, part, nb, n_terms, coeff, terms, out_terms,
                       out_sum);
    return hipGetLastError();
}

// ------------------------------------------------ expval without allocation

namespace {

// Scratch of the allocation-free expectation call, one copy per device for the
// life of the process: masks, coefficients, per-block partials, term sums.
constexpr int kNoAllocMasksOff = 0;
constexpr int kNoAllocCoeffOff = kNoAllocMaxTerms;
constexpr int kNoAllocPartOff = 2 * kNoAllocMaxTerms;
constexpr int64_t kNoAllocDoubles = 2 * kNoAllocMaxTerms + (int64_t)kNoAllocMaxTerms * 1024 + kNoAllocMaxTerms;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

// Masks and coefficients of up to 64 terms travel by value (no host staging).
struct TermChunk {
    uint64_t mask[kTermsPerPass];
    double coeff[kTermsPerPass];
};

__global__ void k_stage_terms(const TermChunk c, int count, uint64_t *__restrict__ masks, double *__restrict__ coeff) {
    const int t = threadIdx.x;
    if (t < count) {
        masks[t] = c.mask[t];
        coeff[t] = c.coeff[t];
    }
}

__global__ void k_zero_scalar(double *p) { *p = 0.0; }

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(double **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t noalloc_scratch_init() {
    double *p = nullptr;
    return scratch_address(&p);
}

hipError_t launch_expval_noalloc(bool c64, const void *psi, uint64_t dim, const uint64_t *masks,
                                 const double *coeff, int n_terms, double *out_terms, double *out_sum,
                                 hipStream_t st) {
    if (n_terms < 0 || n_terms > kNoAllocMaxTerms) return hipErrorInvalidValue;
    if (expval_partials(dim, n_terms) > (int64_t)kNoAllocMaxTerms * 1024 + kNoAllocMaxTerms)
        return hipErrorInvalidValue;
    if (n_terms == 0) {
        if (out_sum) hipLaunchKernelGGL(k_zero_scalar, dim3(1), dim3(1), 0, st, out_sum);
        return hipGetLastError();
    }
    double *sc = nullptr;
    hipError_t e = scratch_address(&sc);
    if (e != hipSuccess) return e;
    uint64_t *dm = reinterpret_cast<uint64_t *>(sc + kNoAllocMasksOff);
    double *dc = sc + kNoAllocCoeffOff;
    for (int t0 = 0; t0 < n_terms; t0 += kTermsPerPass) {
        TermChunk c{};
        const int cnt = n_terms - t0 < kTermsPerPass ? n_terms - t0 : kTermsPerPass;
        for (int t = 0; t < cnt; ++t) {
            c.mask[t] = masks[t0 + t];
            c.coeff[t] = coeff ? coeff[t0 + t] : 0.0;
        }
        hipLaunchKernelGGL(k_stage_terms, dim3(1), dim3(kTermsPerPass), 0, st, c, cnt, dm + t0, dc + t0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_expval(c64, psi, dim, dm, dc, n_terms, sc + kNoAllocPartOff, out_terms, out_sum, st);
}

int64_t sample_tree_doubles(uint64_t dim) {
    Levels L = make_levels(dim);
    int64_t t = 0;
    for (int l = 1; l <= L.n; ++l) t += (int64_t)L.size[l];
    return t < 1 ? 1 : t;
}

hipError_t launch_sample(bool c64, const void *psi, uint64_t dim, int64_t shots, uint64_t seed, double *tree,
                         uint64_t *out, hipStream_t st) {
    if (shots <= 0) return hipSuccess;
    Levels L = make_levels(dim);
    if (L.n > kMaxLevels) return hipErrorInvalidValue;
    for (int l = 1; l <= L.n; ++l) {
        const uint64_t nout = L.size[l];
        const uint32_t g = (uint32_t)((nout * 64 + kThreads - 1) / kThreads);
        if (l == 1) {
            const uint32_t gl = (uint32_t)(((nout + kLeafNodes - 1) / kLeafNodes * 64 + kThreads - 1) / kThreads);
            if (c64) hipLaunchKernelGGL(k_tree_leaf<float>, dim3(gl), dim3(kThreads), 0, st, (const float2 *)psi, dim, tree + L.off[1], nout);
            else hipLaunchKernelGGL(k_tree_leaf<double>, dim3(gl), dim3(kThreads), 0, st, (const double2 *)psi, dim, tree + L.off[1], nout);
        } else {
            hipLaunchKernelGGL(k_tree_up, dim3(g), dim3(kThreads), 0, st, tree + L.off[l - 1], L.size[l - 1],
                               tree + L.off[l], nout);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint32_t g = (uint32_t)((shots + kThreads - 1) / kThreads);
    if (c64) hipLaunchKernelGGL(k_sample<float>, dim3(g), dim3(kThreads), 0, st, (const float2 *)psi, tree, L, seed, shots, out);
    else hipLaunchKernelGGL(k_sample<double>, dim3(g), dim3(kThreads), 0, st, (const double2 *)psi, tree, L, seed, shots, out);
    return hipGetLastError();
}

hipError_t launch_apply_observable(bool c64, const void *psi, void *lam, uint64_t dim, const uint64_t *masks,
                                   const double *coeff, int n_terms, hipStream_t st) {
    const uint32_t g = grid_for(dim, kThreads * 8, 1 << 20);
    if (c64) hipLaunchKernelGGL(k_apply_observable<float>, dim3(g), dim3(kThreads), 0, st, (const float2 *)psi, (float2 *)lam, dim, masks, coeff, n_terms);
    else hipLaunchKernelGGL(k_apply_observable<double>, dim3(g), dim3(kThreads), 0, st, (const double2 *)psi, (double2 *)lam, dim, masks, coeff, n_terms);
    return hipGetLastError();
}

hipError_t launch_grad_rows(const double *gpart, int64_t gstride, int64_t count, int n_rows, double *rows,
                            hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_rows, dim3(n_rows), dim3(kGradThreads), 0, st, gpart, gstride, count, n_rows, rows);
    return hipGetLastError();
}

hipError_t launch_grad_slots(const double *rows, const int32_t *row_slot, int n_rows, double *grad, int n_params,
                             hipStream_t st) {
    if (n_params <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_slots, dim3((n_params + 255) / 256), dim3(256), 0, st, rows, row_slot, n_rows, grad,
                       n_params);
    return hipGetLastError();
}

}  // namespace qg
