// qg_batch.hip -- batched form: many independent circuits (the paper's parallel
// mode, Sec. 2.4) in one persistent launch.
//
// Workgroups take circuits from a device work counter in the host's
// longest-first order.  A circuit whose state fits one tile (2^tile_bits
// amplitudes) runs entirely in registers and LDS: it starts from |0...0> in
// registers, runs its single pass and reduces its observable without touching
// HBM.  A larger circuit runs its passes over a state in the workgroup's own
// HBM scratch slot, tile after tile, with a fence and barrier between passes.
#include "qg_kernels.h"
#include "qg_tile_dev.h"

namespace qg {
namespace {

using namespace dev;

__device__ __forceinline__ double zz_chain(uint64_t i, int n) {
    const uint64_t mask = n >= 2 ? ((1ull << (n - 1)) - 1) : 0;
    // __popcll is unsigned: convert before subtracting
    return (double)(n - 1) - 2.0 * (double)__popcll((i ^ (i >> 1)) & mask);
}

__global__ void k_batch_reset(int *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

template <typename R, int RB>
__global__ void __launch_bounds__(256)
k_batch(const BatchCirc *__restrict__ circs, const int32_t *__restrict__ order, int n_circ,
        const PassDesc *__restrict__ passes, const PhaseDesc *__restrict__ phases, const DevOp *__restrict__ ops,
        const uint64_t *__restrict__ masks, const double *__restrict__ coeff, int obs_kind, int *counter,
        typename V2<R>::T *__restrict__ scratch, uint64_t scratch_stride, double *__restrict__ out) {
    using C = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    __shared__ int s_item;
    __shared__ double s_red[4];
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= n_circ) break;
        const int ci = order[item];
        const BatchCirc &bc = circs[ci];
        const int n = bc.n;
        double acc = 0.0;
        // A circuit whose state is one tile lives in registers and LDS only.
        const bool one_tile = bc.n_pass == 1 && passes[bc.pass_begin].n_tiles == 1;
        C *psi = scratch + (uint64_t)blockIdx.x * scratch_stride;
        C *const st[2] = {psi, nullptr};
        const uint64_t dim = 1ull << n;
        if (!one_tile) {
            for (uint64_t i = tid; i < dim; i += blockDim.x) {
                C v;
                v.x = i == 0 ? (R)1 : (R)0;
                v.y = (R)0;
                psi[i] = v;
            }
            __threadfence();
            __syncthreads();
        }
        for (int p = 0; p < bc.n_pass; ++p) {
            const PassDesc &P = passes[bc.pass_begin + p];
            const PhaseDesc *ph = phases + P.phase_begin;
            const bool active = tid < (1 << P.tb);
            for (uint64_t t = 0; t < P.n_tiles; ++t) {
                const uint64_t gbase = tile_gbase(P, t);
                C a[1][1 << RB];
                if (one_tile) tile_zero<R, RB>(P, ph[0], gbase, a, tid);
                else if (active) tile_load<R, RB, 1>(P, ph[0], gbase, st, a, tid);
                tile_phases<R, RB, 1>(P, ph, ops, DiagTables{nullptr, nullptr}, gbase, a, lds, nullptr, 0, t, tid, active);
                const PhaseDesc &last = ph[P.n_phase - 1];
                if (one_tile) {
                    if (active)
                        acc = obs_kind == QG_OBS_ZZ_CHAIN
                                  ? tile_obs_zz_chain<R, RB>(P, last, gbase, a, tid, n)
                                  : tile_obs_terms<R, RB>(P, last, gbase, a, tid, masks + bc.obs_begin,
                                                          coeff + bc.obs_begin, bc.obs_count);
                } else if (active) {
                    tile_store<R, RB, 1>(P, last, gbase, st, a, tid);
                }
            }
            if (!one_tile) {
                __threadfence();
                __syncthreads();
            }
        }
        if (!one_tile) {
            for (uint64_t i = tid; i < dim; i += blockDim.x) {
                const C v = psi[i];
                const double pr = (double)v.x * v.x + (double)v.y * v.y;
                double o;
                if (obs_kind == QG_OBS_ZZ_CHAIN) {
                    o = zz_chain(i, n);
                } else {
                    o = 0.0;
                    for (int k = 0; k < bc.obs_count; ++k)
                        o += (__popcll(i & masks[bc.obs_begin + k]) & 1) ? -coeff[bc.obs_begin + k]
                                                                         : coeff[bc.obs_begin + k];
                }
                acc += pr * o;
            }
        }
        acc = wave_sum(acc, 64);
        if ((tid & 63) == 0) s_red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += s_red[w];
            out[ci] = s;
        }
        __syncthreads();
    }
}

template <typename R, int RB>
hipError_t launch_batch_t(const BatchLaunch &L, hipStream_t st) {
    using C = typename V2<R>::T;
    const size_t lds = (size_t(1) << L.tile_bits) * sizeof(C);
    if (lds > 65536) {
        static bool done = false;
        if (!done) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<R, RB>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, L.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_batch<R, RB>), dim3(L.grid), dim3(256), lds, st, L.circs, L.order, L.n_circ, L.passes,
                       L.phases, L.ops, L.masks, L.coeff, L.obs_kind, L.counter, static_cast<C *>(L.scratch),
                       L.scratch_stride, L.out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch(bool c64, int rb, const BatchLaunch &L, hipStream_t st) {
    if (L.grid < 1 || L.n_circ < 0) return hipErrorInvalidValue;
    if (c64) {
        if (rb == 5) return launch_batch_t<float, 5>(L, st);
        if (rb == 4) return launch_batch_t<float, 4>(L, st);
    } else {
        if (rb == 4) return launch_batch_t<double, 4>(L, st);
        if (rb == 3) return launch_batch_t<double, 3>(L, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace qg
