// qg_tile.hip -- the pass kernel: one workgroup streams one active tile of the
// state through registers and applies the pass's ops (App. A: single-qubit
// operators of eq. (tp), controlled operators of eq. (cx), the diagonal CR1 of
// eq. (cr1)).  Every pass reads and writes each active amplitude once.
#include <mutex>
#include <vector>

#include "qg_kernels.h"
#include "qg_tile_dev.h"

namespace qg {
namespace {

using namespace dev;

// Occupancy floor for the compiler's register budget: the complex128 kernel
// with 16 amplitudes per thread runs multi-phase passes with half-LDS
// exchanges at three workgroups per CU when it fits 168 registers, and so does
// the adjoint's two-state kernel with 8 amplitudes of each state per thread
// (a few registers spill there; it is still faster than at two workgroups).
// The complex64 kernel with 16 amplitudes per thread runs four workgroups per
// CU in 128 registers (also with a small spill, and faster than three).
template <typename R, int RB, int NS>
struct TileWaves {
    static constexpr int value = (sizeof(R) == 8 && ((RB == 4 && NS == 1) || (RB == 3 && NS == 2))) ? 3
                                 : (sizeof(R) == 4 && RB == 4 && NS == 1)                            ? 4
                                                                                                     : 1;
};

template <typename R, int RB, int NS>
__device__ __forceinline__ void tile_pass(const PassDesc &P, const PhaseDesc *__restrict__ phases,
                                          const DevOp *__restrict__ ops, const DiagTables &dt,
                                          typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam,
                                          double *__restrict__ gpart, int64_t gstride) {
    using C = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int tid = threadIdx.x;
    const uint64_t gbase = tile_gbase(P, blockIdx.x);
    C *const st[2] = {psi, lam};
    C a[NS][1 << RB];
    tile_load<R, RB, NS>(P, phases[0], gbase, st, a, tid);
    tile_phases<R, RB, NS>(P, phases, ops, dt, gbase, a, lds, gpart, gstride, blockIdx.x, tid, true);
    tile_store<R, RB, NS>(P, phases[P.n_phase - 1], gbase, st, a, tid);
}

// Persistent form (forward passes): each block walks a strided sequence of
// tiles and issues the loads of its next tile before computing the current
// one, so that memory traffic overlaps the arithmetic and the LDS exchanges.
// With PASS_XCD the blocks of XCD x (x = block mod 8) cover the x-th eighth
// of the tiles; the host launches a multiple of 8 blocks, at most n_tiles.
template <typename R, int RB>
__device__ __forceinline__ void tile_pass_pipe(const PassDesc &P, const PhaseDesc *__restrict__ phases,
                                               const DevOp *__restrict__ ops, const DiagTables &dt,
                                               typename V2<R>::T *__restrict__ psi) {
    using C = typename V2<R>::T;
    constexpr int NR = 1 << RB;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int tid = threadIdx.x;
    const uint64_t T = P.n_tiles, G = gridDim.x;
    uint64_t w, step, end;
    if (P.flags & PASS_XCD) {
        const uint64_t span = T >> 3;
        w = (blockIdx.x & 7) * span + (blockIdx.x >> 3);
        step = G >> 3;
        end = ((blockIdx.x & 7) + 1) * span;
    } else {
        w = blockIdx.x;
        step = G;
        end = T;
    }
    C *const st[2] = {psi, nullptr};
    C a[1][NR], nx[1][NR];
    const PhaseDesc &first = phases[0];
    const PhaseDesc &last = phases[P.n_phase - 1];
    tile_load<R, RB, 1>(P, first, tile_deposit(P, w), st, a, tid);
    for (;;) {
        const uint64_t wn = w + step;
        const bool more = wn < end;
        if (more) tile_load<R, RB, 1>(P, first, tile_deposit(P, wn), st, nx, tid);
        const uint64_t gbase = tile_deposit(P, w);
        tile_phases<R, RB, 1>(P, phases, ops, dt, gbase, a, lds, nullptr, 0, w, tid, true);
        tile_store<R, RB, 1>(P, last, gbase, st, a, tid);
        if (!more) break;
#pragma unroll
        for (int e = 0; e < NR; ++e) a[0][e] = nx[0][e];
        w = wn;
    }
}

template <typename R, int RB>
__global__ void __launch_bounds__(256)
k_tile_pipe(const unsigned char *__restrict__ dev, const ProgOffsets offs, int pass_idx,
            typename V2<R>::T *__restrict__ psi) {
    const PassDesc &P = reinterpret_cast<const PassDesc *>(dev + offs.pass)[pass_idx];
    const DiagTables dt{reinterpret_cast<const DiagRun *>(dev + offs.run),
                        reinterpret_cast<const DiagEntry *>(dev + offs.entry)};
    tile_pass_pipe<R, RB>(P, reinterpret_cast<const PhaseDesc *>(dev + offs.phase) + P.phase_begin,
                          reinterpret_cast<const DevOp *>(dev + offs.op), dt, psi);
}

template <typename R, int RB>
__global__ void __launch_bounds__(256) k_tile_inl_pipe(const InlineProg prog, typename V2<R>::T *__restrict__ psi) {
    tile_pass_pipe<R, RB>(prog.pass, prog.phases, prog.ops, DiagTables{nullptr, nullptr}, psi);
}

template <typename R, int RB, int NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TileWaves<R, RB, NS>::value)))
k_tile(const unsigned char *__restrict__ dev, const ProgOffsets offs, int pass_idx,
       typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam, double *__restrict__ gpart,
       int64_t gstride) {
    const PassDesc &P = reinterpret_cast<const PassDesc *>(dev + offs.pass)[pass_idx];
    const DiagTables dt{reinterpret_cast<const DiagRun *>(dev + offs.run),
                        reinterpret_cast<const DiagEntry *>(dev + offs.entry)};
    tile_pass<R, RB, NS>(P, reinterpret_cast<const PhaseDesc *>(dev + offs.phase) + P.phase_begin,
                         reinterpret_cast<const DevOp *>(dev + offs.op), dt, psi, lam, gpart, gstride);
}

template <typename R, int RB, int NS>
__global__ void __launch_bounds__(256)
k_tile_inl(const InlineProg prog, typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam,
           double *__restrict__ gpart, int64_t gstride) {
    tile_pass<R, RB, NS>(prog.pass, prog.phases, prog.ops, DiagTables{nullptr, nullptr}, psi, lam, gpart, gstride);
}

// Resident blocks per CU of a kernel at a block size and dynamic LDS size,
// times the CU count (cached per kernel, configuration and device).
int resident_blocks(const void *fn, int threads, size_t lds) {
    struct Key {
        const void *fn;
        int threads;
        size_t lds;
        int dev;
        int blocks;
    };
    static std::mutex mu;
    static std::vector<Key> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    for (const Key &k : cache)
        if (k.fn == fn && k.threads == threads && k.lds == lds && k.dev == dev) return k.blocks;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cache.push_back({fn, threads, lds, dev, per_cu * cus});
    return per_cu * cus;
}

template <typename R, int RB, int NS>
hipError_t launch_one(const PassDesc &hp, const InlineProg *inl, const void *dev, const ProgOffsets &offs,
                      int pass_idx, void *psi, void *lam, double *gpart, int64_t gstride, hipStream_t st) {
    using C = typename V2<R>::T;
    const size_t lds = hp.n_phase > 1 ? (size_t(1) << hp.b) * ((hp.flags & PASS_HALFX) ? sizeof(R) : sizeof(C)) : 0;
    const bool pipe = NS == 1 && (hp.flags & PASS_PIPE);
    if (lds > 65536) {
        static bool done = false;
        if (!done) {
            hipError_t e = hipSuccess;
            for (const void *fn : {reinterpret_cast<const void *>(&k_tile<R, RB, NS>),
                                   reinterpret_cast<const void *>(&k_tile_inl<R, RB, NS>),
                                   reinterpret_cast<const void *>(&k_tile_pipe<R, RB>),
                                   reinterpret_cast<const void *>(&k_tile_inl_pipe<R, RB>)})
                if (e == hipSuccess) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    dim3 block(1u << hp.tb);
    if (pipe) {
        const void *fn = inl ? reinterpret_cast<const void *>(&k_tile_inl_pipe<R, RB>)
                             : reinterpret_cast<const void *>(&k_tile_pipe<R, RB>);
        uint64_t g = (uint64_t)resident_blocks(fn, (int)block.x, lds);
        if (g == 0) return hipErrorInvalidValue;
        if (g > hp.n_tiles) g = hp.n_tiles;
        // The XCD schedule needs a multiple of 8 blocks (n_tiles >= 8 under PASS_XCD).
        if (hp.flags & PASS_XCD) g &= ~7ull;
        if (g == 0) return hipErrorInvalidValue;
        if (inl) {
            hipLaunchKernelGGL((k_tile_inl_pipe<R, RB>), dim3((uint32_t)g), block, lds, st, *inl,
                               static_cast<C *>(psi));
        } else {
            hipLaunchKernelGGL((k_tile_pipe<R, RB>), dim3((uint32_t)g), block, lds, st,
                               static_cast<const unsigned char *>(dev), offs, pass_idx, static_cast<C *>(psi));
        }
        return hipGetLastError();
    }
    dim3 grid((uint32_t)hp.n_tiles);
    if (inl) {
        hipLaunchKernelGGL((k_tile_inl<R, RB, NS>), grid, block, lds, st, *inl, static_cast<C *>(psi),
                           static_cast<C *>(lam), gpart, gstride);
    } else {
        hipLaunchKernelGGL((k_tile<R, RB, NS>), grid, block, lds, st, static_cast<const unsigned char *>(dev), offs,
                           pass_idx, static_cast<C *>(psi), static_cast<C *>(lam), gpart, gstride);
    }
    return hipGetLastError();
}

template <typename R, int NS>
hipError_t launch_rb(const PassDesc &hp, const InlineProg *inl, const void *dev, const ProgOffsets &o, int pi,
                     void *psi, void *lam, double *gp, int64_t gs, hipStream_t st) {
    switch (hp.rb) {
    case 1: return launch_one<R, 1, NS>(hp, inl, dev, o, pi, psi, lam, gp, gs, st);
    case 2: return launch_one<R, 2, NS>(hp, inl, dev, o, pi, psi, lam, gp, gs, st);
    case 3: return launch_one<R, 3, NS>(hp, inl, dev, o, pi, psi, lam, gp, gs, st);
    case 4: return launch_one<R, 4, NS>(hp, inl, dev, o, pi, psi, lam, gp, gs, st);
    case 5: return launch_one<R, 5, NS>(hp, inl, dev, o, pi, psi, lam, gp, gs, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_tile(bool c64, const PassDesc &hp, const InlineProg *inl, const void *dev, const ProgOffsets &offs,
                       int pass_idx, int ns, void *psi, void *lam, double *gpart, int64_t gstride, hipStream_t st) {
    if (hp.n_tiles == 0 || hp.n_tiles > 0x7fffffffull || hp.tb > kMaxThreadBits || hp.n_phase < 1)
        return hipErrorInvalidValue;
    if (ns == 2) {
        return c64 ? launch_rb<float, 2>(hp, inl, dev, offs, pass_idx, psi, lam, gpart, gstride, st)
                   : launch_rb<double, 2>(hp, inl, dev, offs, pass_idx, psi, lam, gpart, gstride, st);
    }
    return c64 ? launch_rb<float, 1>(hp, inl, dev, offs, pass_idx, psi, nullptr, nullptr, 0, st)
               : launch_rb<double, 1>(hp, inl, dev, offs, pass_idx, psi, nullptr, nullptr, 0, st);
}

}  // namespace qg
