// qg_dense.hip -- a fused k-qubit block applied as one dense 2^k x 2^k complex
// matrix on the matrix cores (App. D.2's fused gates, taken as a dense
// contraction).
//
// A tile is the 2^(k+L) amplitudes that agree on all qubits outside the block
// qubits Q (k of them) and the L lowest other qubits.  In LDS the tile is the
// matrix X[r][c]: row r = the Q bits, column c = the low bits, so that every
// wavefront load or store of a row is a contiguous run.  Y = U X is computed in
// 16x16 output blocks with v_mfma_{f64,f32}_16x16x4: for complex numbers,
// Yr = Ur Xr + (-Ui) Xi and Yi = Ur Xi + Ui Xr, four real products per k-step.
// U is read transposed from device memory (UT[c][r] = U[r][c]) so that the 16
// lanes of an A fragment read consecutive addresses.
#include "qg_kernels.h"

namespace qg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
// Operand layout of both 16x16x4 forms: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Output: lane l, register r holds D[row(l / 16, r)][l % 16]
// (measured on gfx950: rows l/16 + 4 r for f64, 4 (l/16) + r for f32).
template <> struct Mfma<double> {
    using C = double2;
    using Acc = d4;
    static __device__ __forceinline__ Acc mac(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
    using C = float2;
    using Acc = f4;
    static __device__ __forceinline__ Acc mac(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// Global index offset of the low-bit pattern `v` over the qubit list q[0..cnt).
__device__ __forceinline__ uint64_t deposit(uint32_t v, const int8_t *q, int cnt) {
    uint64_t o = 0;
    for (int j = 0; j < cnt; ++j)
        if ((v >> j) & 1u) o |= 1ull << q[j];
    return o;
}

template <typename R, int KB>
__global__ void __launch_bounds__(256)
k_dense(const DenseDesc D, const R *__restrict__ ut_re, const R *__restrict__ ut_im,
        typename Mfma<R>::C *__restrict__ psi) {
    using C = typename Mfma<R>::C;
    using Acc = typename Mfma<R>::Acc;
    constexpr int ROWS = 1 << KB;
    const int L = D.l;
    const int COLS = 1 << L;
    extern __shared__ __align__(16) unsigned char smem[];
    C *X = reinterpret_cast<C *>(smem);  // [ROWS][COLS]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    // Tile base: deposit the block index into the free runs.
    uint64_t gbase = 0;
    {
        uint64_t w = blockIdx.x;
        for (int r = 0; r < D.n_runs; ++r) {
            const int len = D.run_len[r];
            gbase |= (w & ((1ull << len) - 1)) << D.run_start[r];
            w >>= len;
        }
    }
    // Load: thread covers column c = tid % COLS of rows tid / COLS, + 256 / COLS, ...
    const int cstep = 256 < COLS ? 256 : COLS;
    const int rstep = 256 / cstep;
    const int c0 = tid % cstep;
    const int r0 = tid / cstep;
    for (int c = c0; c < COLS; c += cstep) {
        const uint64_t cg = deposit(c, D.low_q, L);
        for (int r = r0; r < ROWS; r += rstep)
            X[r * COLS + c] = psi[gbase | cg | deposit(r, D.blk_q, KB)];
    }
    __syncthreads();

    // Output blocks (I, J) of 16 x 16, dealt to the 4 waves.
    const int nbi = ROWS / 16, nbj = COLS / 16;
    const int nblk = nbi * nbj;
    const int li = lane & 15, lk = lane >> 4;
    // Each wave accumulates up to kMaxBlk output blocks before anyone overwrites X.
    constexpr int kMaxBlk = 8;
    Acc accr[kMaxBlk], acci[kMaxBlk];
#pragma unroll
    for (int q = 0; q < kMaxBlk; ++q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            accr[q][r] = (R)0;
            acci[q][r] = (R)0;
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxBlk; ++q) {
        const int blk = wave + 4 * q;
        if (blk < nblk) {
            const int I = blk / nbj, J = blk % nbj;
            for (int s = 0; s < ROWS; s += 4) {
                // A[i][k] = U[16 I + i][s + k] = UT[s + k][16 I + i]; B[k][j] = X[s + k][16 J + j]
                const int ka = s + lk;
                const R ar = ut_re[ka * ROWS + 16 * I + li];
                const R ai = ut_im[ka * ROWS + 16 * I + li];
                const C b = X[ka * COLS + 16 * J + li];
                accr[q] = Mfma<R>::mac(ar, b.x, accr[q]);
                accr[q] = Mfma<R>::mac(-ai, b.y, accr[q]);
                acci[q] = Mfma<R>::mac(ar, b.y, acci[q]);
                acci[q] = Mfma<R>::mac(ai, b.x, acci[q]);
            }
        }
    }
    __syncthreads();
    // D fragment: lane holds rows 16 I + row(lane / 16, r), column 16 J + lane % 16.
#pragma unroll
    for (int q = 0; q < kMaxBlk; ++q) {
        const int blk = wave + 4 * q;
        if (blk < nblk) {
            const int I = blk / nbj, J = blk % nbj;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                C y;
                y.x = accr[q][r];
                y.y = acci[q][r];
                X[(16 * I + Mfma<R>::row(lk, r)) * COLS + 16 * J + li] = y;
            }
        }
    }
    __syncthreads();
    for (int c = c0; c < COLS; c += cstep) {
        const uint64_t cg = deposit(c, D.low_q, L);
        for (int r = r0; r < ROWS; r += rstep)
            psi[gbase | cg | deposit(r, D.blk_q, KB)] = X[r * COLS + c];
    }
}

template <typename R, int KB>
hipError_t launch_k(const DenseDesc &D, const void *ut_re, const void *ut_im, void *psi, hipStream_t st) {
    using C = typename Mfma<R>::C;
    const size_t lds = (size_t(1) << (KB + D.l)) * sizeof(C);
    if (lds > 65536) {
        static bool done = false;
        if (!done) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dense<R, KB>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    hipLaunchKernelGGL((k_dense<R, KB>), dim3((uint32_t)D.n_tiles), dim3(256), lds, st, D,
                       static_cast<const R *>(ut_re), static_cast<const R *>(ut_im), static_cast<C *>(psi));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense(bool c64, const DenseDesc &D, const void *ut_re, const void *ut_im, void *psi,
                        hipStream_t st) {
    // 16 x 16 output blocks: 2^k >= 16 rows, 2^L >= 16 columns, at most 8 blocks per wave.
    if (D.k < 4 || D.k > 6 || D.l < 4 || D.k + D.l > 13 || (1 << (D.k - 4)) * (1 << (D.l - 4)) > 32 ||
        D.n_tiles == 0 || D.n_tiles > 0x7fffffffull)
        return hipErrorInvalidValue;
    switch (D.k) {
    case 4: return c64 ? launch_k<float, 4>(D, ut_re, ut_im, psi, st) : launch_k<double, 4>(D, ut_re, ut_im, psi, st);
    case 5: return c64 ? launch_k<float, 5>(D, ut_re, ut_im, psi, st) : launch_k<double, 5>(D, ut_re, ut_im, psi, st);
    case 6: return c64 ? launch_k<float, 6>(D, ut_re, ut_im, psi, st) : launch_k<double, 6>(D, ut_re, ut_im, psi, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace qg
