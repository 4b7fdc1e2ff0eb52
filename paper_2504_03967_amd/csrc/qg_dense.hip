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
// Each wave owns a 16-row stripe of U (4 waves: 4 stripes at k = 6; at k = 5
// and 4 the waves of a stripe split its column blocks) and keeps that stripe's
// A fragments in registers for the whole tile; U is read transposed
// (UT[c][r] = U[r][c]) so that the 16 lanes of a fragment read consecutive
// addresses.
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

template <typename R, int KB, int LB>
__global__ void __launch_bounds__(256)
k_dense(const DenseDesc D, const R *__restrict__ ut_re, const R *__restrict__ ut_im,
        typename Mfma<R>::C *__restrict__ psi) {
    using C = typename Mfma<R>::C;
    using Acc = typename Mfma<R>::Acc;
    constexpr int ROWS = 1 << KB;
    constexpr int COLS = 1 << LB;
    constexpr int NBI = ROWS / 16;                // 16-row stripes of U (and of Y)
    constexpr int WPI = 4 / NBI;                  // waves per stripe
    constexpr int KS = ROWS / 4;                  // k-steps of 4
    constexpr int NBJ = COLS / 16;                // 16-column blocks of X (and of Y)
    constexpr int JPW = (NBJ + WPI - 1) / WPI;    // column blocks per wave
    constexpr int CSTEP = COLS < 256 ? COLS : 256;
    constexpr int RSTEP = 256 / CSTEP;            // <= 16 <= ROWS
    constexpr int NCOL = COLS / CSTEP;            // columns per thread
    constexpr int NROW = ROWS / RSTEP;            // rows per thread and column
    extern __shared__ __align__(16) unsigned char smem[];
    C *X = reinterpret_cast<C *>(smem);           // [ROWS][COLS]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int I = wave % NBI;                     // this wave's stripe
    const int j0 = wave / NBI;                    // its column blocks: j0, j0 + WPI, ...

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
    // Global offsets of the block-qubit patterns (rows), once per tile, in LDS
    // after the tile.  A thread covers columns c0 + m CSTEP and in each the rows
    // r0 + q RSTEP; all of its loads are issued before the first store to LDS.
    uint64_t *rowoff = reinterpret_cast<uint64_t *>(X + ROWS * COLS);
    if (tid < ROWS) rowoff[tid] = deposit(tid, D.blk_q, KB);
    const int c0 = tid % CSTEP;
    const int r0 = tid / CSTEP;
    uint64_t cg[NCOL];
#pragma unroll
    for (int m = 0; m < NCOL; ++m) cg[m] = gbase | deposit(c0 + m * CSTEP, D.low_q, LB);
    __syncthreads();
    {
        C v[NCOL][NROW];
#pragma unroll
        for (int m = 0; m < NCOL; ++m)
#pragma unroll
            for (int q = 0; q < NROW; ++q) v[m][q] = psi[cg[m] | rowoff[r0 + q * RSTEP]];
#pragma unroll
        for (int m = 0; m < NCOL; ++m)
#pragma unroll
            for (int q = 0; q < NROW; ++q) X[(r0 + q * RSTEP) * COLS + c0 + m * CSTEP] = v[m][q];
    }

    // The stripe's A fragments for every k-step (U is shared by all tiles and
    // stays in the caches): A[i][k] = U[16 I + i][s + k] = UT[s + k][16 I + i],
    // lane (li, lk) holding i = li, k = lk.
    R ar[KS], ai[KS];
#pragma unroll
    for (int q = 0; q < KS; ++q) {
        const int ka = 4 * q + lk;
        ar[q] = ut_re[ka * ROWS + 16 * I + li];
        ai[q] = ut_im[ka * ROWS + 16 * I + li];
    }
    __syncthreads();

    // Y[16 I .. 16 I + 15][16 J ..] for this wave's column blocks J; for complex
    // numbers Yr = Ur Xr + (-Ui) Xi and Yi = Ur Xi + Ui Xr.
    Acc accr[JPW], acci[JPW];
#pragma unroll
    for (int q = 0; q < JPW; ++q) {
        const int J = j0 + WPI * q;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            accr[q][r] = (R)0;
            acci[q][r] = (R)0;
        }
        if (J < NBJ) {
#pragma unroll
            for (int t = 0; t < KS; ++t) {
                const C b = X[(4 * t + lk) * COLS + 16 * J + li];
                accr[q] = Mfma<R>::mac(ar[t], b.x, accr[q]);
                accr[q] = Mfma<R>::mac(-ai[t], b.y, accr[q]);
                acci[q] = Mfma<R>::mac(ar[t], b.y, acci[q]);
                acci[q] = Mfma<R>::mac(ai[t], b.x, acci[q]);
            }
        }
    }
    __syncthreads();
    // D fragment: lane holds rows 16 I + row(lane / 16, r), column 16 J + lane % 16.
#pragma unroll
    for (int q = 0; q < JPW; ++q) {
        const int J = j0 + WPI * q;
        if (J < NBJ) {
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
    {
        C v[NCOL][NROW];
#pragma unroll
        for (int m = 0; m < NCOL; ++m)
#pragma unroll
            for (int q = 0; q < NROW; ++q) v[m][q] = X[(r0 + q * RSTEP) * COLS + c0 + m * CSTEP];
#pragma unroll
        for (int m = 0; m < NCOL; ++m)
#pragma unroll
            for (int q = 0; q < NROW; ++q) psi[cg[m] | rowoff[r0 + q * RSTEP]] = v[m][q];
    }
}

template <typename R, int KB, int LB>
hipError_t launch_kl(const DenseDesc &D, const void *ut_re, const void *ut_im, void *psi, hipStream_t st) {
    using C = typename Mfma<R>::C;
    // the tile, then the 2^k row offsets (uint64)
    const size_t lds = (size_t(1) << (KB + LB)) * sizeof(C) + (size_t(8) << KB);
    if (lds > 65536) {
        static bool done = false;
        if (!done) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dense<R, KB, LB>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    hipLaunchKernelGGL((k_dense<R, KB, LB>), dim3((uint32_t)D.n_tiles), dim3(256), lds, st, D,
                       static_cast<const R *>(ut_re), static_cast<const R *>(ut_im), static_cast<C *>(psi));
    return hipGetLastError();
}

// Tile widths: 2^L columns for L in 4 .. 13 - k.
template <typename R, int KB>
hipError_t launch_k(const DenseDesc &D, const void *ut_re, const void *ut_im, void *psi, hipStream_t st) {
    switch (D.l) {
    case 4: return launch_kl<R, KB, 4>(D, ut_re, ut_im, psi, st);
    case 5: return launch_kl<R, KB, 5>(D, ut_re, ut_im, psi, st);
    case 6: return launch_kl<R, KB, 6>(D, ut_re, ut_im, psi, st);
    case 7: return launch_kl<R, KB, 7>(D, ut_re, ut_im, psi, st);
    case 8:
        if constexpr (KB + 8 <= 13) return launch_kl<R, KB, 8>(D, ut_re, ut_im, psi, st);
        break;
    case 9:
        if constexpr (KB + 9 <= 13) return launch_kl<R, KB, 9>(D, ut_re, ut_im, psi, st);
        break;
    }
    return hipErrorInvalidValue;
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
