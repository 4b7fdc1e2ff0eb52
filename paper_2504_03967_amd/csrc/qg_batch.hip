// qg_batch.hip -- batched form: many independent circuits (the paper's parallel
// mode, Sec. 2.4).
//
// Circuits whose state fits one tile (2^tile_bits amplitudes) run in one
// persistent launch: workgroups take them from a device work counter in the
// host's longest-first order, start from |0...0> in registers, run the single
// pass and reduce the observable without touching device memory.
//
// Larger circuits keep their states in device memory and run pass by pass:
// each launch applies the next pass of every circuit of a group that has one
// left, one workgroup per (circuit, tile), so a launch has as many workgroups
// as the group's states have tiles and streams like a pass over one large
// state.  Each state is filled with |0...0> first; from there a first pass
// that visits every tile changes only the tile holding index 0 (its ops mix
// amplitudes within tiles, and a zero tile stays zero), so it runs on that one
// tile, starting from |0...0> in registers.  The observable is reduced per chunk of
// kBatchChunk amplitudes, then per circuit in a fixed order.
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
        double *__restrict__ out) {
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
        const PassDesc &P = passes[bc.pass_begin];
        const PhaseDesc *ph = phases + P.phase_begin;
        const bool active = tid < (1 << P.tb);
        const uint64_t gbase = tile_gbase(P, 0);
        C a[1][1 << RB];
        tile_zero<R, RB>(P, ph[0], gbase, a, tid);
        tile_phases<R, RB, 1>(P, ph, ops, DiagTables{nullptr, nullptr}, gbase, a, lds, nullptr, 0, 0, tid, active);
        const PhaseDesc &last = ph[P.n_phase - 1];
        double acc = 0.0;
        if (active)
            acc = obs_kind == QG_OBS_ZZ_CHAIN ? tile_obs_zz_chain<R, RB>(P, last, gbase, a, tid, bc.n)
                                              : tile_obs_terms<R, RB>(P, last, gbase, a, tid, masks + bc.obs_begin,
                                                                      coeff + bc.obs_begin, bc.obs_count);
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

// Register budget of the pass kernel: the complex128 form with 16 amplitudes
// per thread and the complex64 form with 32 fit three workgroups per CU, as the
// single-state tile pass does.
template <typename R, int RB>
struct BatchWaves {
    static constexpr int value = ((sizeof(R) == 8 && RB == 4) || (sizeof(R) == 4 && RB == 5)) ? 3 : 1;
};

// One pass of one circuit on one tile of its state.
template <typename R, int RB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BatchWaves<R, RB>::value)))
k_batch_pass(const BatchItem *__restrict__ items, const int32_t *__restrict__ map,
             const PassDesc *__restrict__ passes, const PhaseDesc *__restrict__ phases,
             const DevOp *__restrict__ ops, typename V2<R>::T *__restrict__ states) {
    using C = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int tid = threadIdx.x;
    const BatchItem it = items[map[blockIdx.x]];
    const PassDesc &P = passes[it.pass];
    const PhaseDesc *ph = phases + P.phase_begin;
    const uint64_t t = blockIdx.x - it.begin;
    const uint64_t gbase = tile_gbase(P, t);
    C *const st[2] = {states + it.state_off, nullptr};
    const bool active = tid < (1 << P.tb);
    C a[1][1 << RB];
    if (it.zero_init) tile_zero<R, RB>(P, ph[0], gbase, a, tid);
    else if (active) tile_load<R, RB, 1>(P, ph[0], gbase, st, a, tid);
    tile_phases<R, RB, 1>(P, ph, ops, DiagTables{nullptr, nullptr}, gbase, a, lds, nullptr, 0, t, tid, active);
    if (active) tile_store<R, RB, 1>(P, ph[P.n_phase - 1], gbase, st, a, tid);
}

// |0...0> over one chunk of a state.
template <typename R>
__global__ void __launch_bounds__(256)
k_batch_fill(const BatchChunkItem *__restrict__ items, const int32_t *__restrict__ map,
             typename V2<R>::T *__restrict__ states) {
    using C = typename V2<R>::T;
    const BatchChunkItem it = items[map[blockIdx.x]];
    const uint64_t c0 = (uint64_t)(blockIdx.x - it.begin) * kBatchChunk;
    C *psi = states + it.state_off;
    for (int k = threadIdx.x; k < kBatchChunk; k += blockDim.x) {
        C v;
        v.x = c0 + k == 0 ? (R)1 : (R)0;
        v.y = (R)0;
        psi[c0 + k] = v;
    }
}

// sum_i |psi_i|^2 O(i) over one chunk of a state.
template <typename R>
__global__ void __launch_bounds__(256)
k_batch_obs_part(const BatchChunkItem *__restrict__ items, const int32_t *__restrict__ map,
                 const typename V2<R>::T *__restrict__ states, const BatchCirc *__restrict__ circs,
                 const uint64_t *__restrict__ masks, const double *__restrict__ coeff, int obs_kind,
                 double *__restrict__ partial) {
    using C = typename V2<R>::T;
    __shared__ double s_red[4];
    const int tid = threadIdx.x;
    const BatchChunkItem it = items[map[blockIdx.x]];
    const uint64_t c0 = (uint64_t)(blockIdx.x - it.begin) * kBatchChunk;
    const C *psi = states + it.state_off;
    const BatchCirc &bc = circs[it.circ];
    double acc = 0.0;
    for (int k = tid; k < kBatchChunk; k += blockDim.x) {
        const uint64_t i = c0 + k;
        const C v = psi[i];
        const double pr = (double)v.x * v.x + (double)v.y * v.y;
        double o;
        if (obs_kind == QG_OBS_ZZ_CHAIN) {
            o = zz_chain(i, it.n);
        } else {
            o = 0.0;
            for (int m = 0; m < bc.obs_count; ++m)
                o += (__popcll(i & masks[bc.obs_begin + m]) & 1) ? -coeff[bc.obs_begin + m] : coeff[bc.obs_begin + m];
        }
        acc += pr * o;
    }
    acc = wave_sum(acc, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += s_red[w];
        partial[blockIdx.x] = s;
    }
}

// Each multi-tile circuit's partials in chunk order.
__global__ void k_batch_obs_final(const BatchObsSum *__restrict__ sums, int n, const double *__restrict__ partial,
                                  double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const BatchObsSum s = sums[i];
    double acc = 0.0;
    for (int k = 0; k < s.count; ++k) acc += partial[s.partial_begin + k];
    out[s.circ] = acc;
}

template <typename R, int RB>
hipError_t launch_batch_t(const BatchLaunch &L, hipStream_t st) {
    using C = typename V2<R>::T;
    const size_t lds = (size_t(1) << L.tile_bits) * sizeof(C);
    if (lds > 65536) return hipErrorInvalidValue;  // tile_bits is 12 (complex128) or 13 (complex64)
    if (L.n_circ > 0) {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, L.counter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_batch<R, RB>), dim3(L.grid), dim3(256), lds, st, L.circs, L.order, L.n_circ, L.passes,
                           L.phases, L.ops, L.masks, L.coeff, L.obs_kind, L.counter, L.out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    C *states = static_cast<C *>(L.states);
    for (const BatchStep &s : L.steps) {
        if (s.blocks == 0) continue;
        if (s.blocks > 0x7fffffffull || s.lds > 65536) return hipErrorInvalidValue;
        const dim3 grid((uint32_t)s.blocks), block(256);
        const int32_t *map = L.map + s.map_off;
        if (s.kind == BATCH_PASS) {
            hipLaunchKernelGGL((k_batch_pass<R, RB>), grid, block, s.lds, st, L.items, map, L.passes, L.phases,
                               L.ops, states);
        } else if (s.kind == BATCH_FILL) {
            hipLaunchKernelGGL(k_batch_fill<R>, grid, block, 0, st, L.chunks, map, states);
        } else {
            hipLaunchKernelGGL(k_batch_obs_part<R>, grid, block, 0, st, L.chunks, map, states, L.circs, L.masks,
                               L.coeff, L.obs_kind, L.partial + s.partial_off);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (L.n_sums > 0) {
        hipLaunchKernelGGL(k_batch_obs_final, dim3((L.n_sums + 255) / 256), dim3(256), 0, st, L.sums, L.n_sums,
                           L.partial, L.out);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_batch(bool c64, int rb, const BatchLaunch &L, hipStream_t st) {
    if ((L.n_circ > 0 && L.grid < 1) || L.n_circ < 0) return hipErrorInvalidValue;
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
