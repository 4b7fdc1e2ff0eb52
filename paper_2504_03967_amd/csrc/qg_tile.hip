// qg_tile.hip -- the pass kernel: one workgroup streams one active tile of the
// state through registers and applies the pass's ops (App. A: single-qubit
// operators of eq. (tp), controlled operators of eq. (cx), the diagonal CR1 of
// eq. (cr1)).  Every pass reads and writes each active amplitude once.
#include "qg_kernels.h"
#include "qg_tile_dev.h"

namespace qg {
namespace {

using namespace dev;

template <typename R, int RB, int NS>
__device__ __forceinline__ void tile_pass(const PassDesc &P, const PhaseDesc *__restrict__ phases,
                                          const DevOp *__restrict__ ops, typename V2<R>::T *__restrict__ psi,
                                          typename V2<R>::T *__restrict__ lam, double *__restrict__ gpart,
                                          int64_t gstride) {
    using C = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int tid = threadIdx.x;
    const uint64_t gbase = tile_gbase(P, blockIdx.x);
    C *const st[2] = {psi, lam};
    C a[NS][1 << RB];
    tile_load<R, RB, NS>(P, phases[0], gbase, st, a, tid);
    tile_phases<R, RB, NS>(P, phases, ops, gbase, a, lds, gpart, gstride, blockIdx.x, tid, true);
    tile_store<R, RB, NS>(P, phases[P.n_phase - 1], gbase, st, a, tid);
}

template <typename R, int RB, int NS>
__global__ void __launch_bounds__(256)
k_tile(const unsigned char *__restrict__ dev, uint32_t pass_off, uint32_t phase_off, uint32_t op_off,
       int pass_idx, typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam,
       double *__restrict__ gpart, int64_t gstride) {
    const PassDesc &P = reinterpret_cast<const PassDesc *>(dev + pass_off)[pass_idx];
    tile_pass<R, RB, NS>(P, reinterpret_cast<const PhaseDesc *>(dev + phase_off) + P.phase_begin,
                         reinterpret_cast<const DevOp *>(dev + op_off), psi, lam, gpart, gstride);
}

template <typename R, int RB, int NS>
__global__ void __launch_bounds__(256)
k_tile_inl(const InlineProg prog, typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam,
           double *__restrict__ gpart, int64_t gstride) {
    tile_pass<R, RB, NS>(prog.pass, prog.phases, prog.ops, psi, lam, gpart, gstride);
}

template <typename R, int RB, int NS>
hipError_t launch_one(const PassDesc &hp, const InlineProg *inl, const void *dev, size_t pass_off,
                      size_t phase_off, size_t op_off, int pass_idx, void *psi, void *lam, double *gpart,
                      int64_t gstride, hipStream_t st) {
    using C = typename V2<R>::T;
    const size_t lds = hp.n_phase > 1 ? (size_t(1) << hp.b) * sizeof(C) : 0;
    if (lds > 65536) {
        static bool done = false;
        if (!done) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile<R, RB, NS>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile_inl<R, RB, NS>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    dim3 grid((uint32_t)hp.n_tiles), block(1u << hp.tb);
    if (inl) {
        hipLaunchKernelGGL((k_tile_inl<R, RB, NS>), grid, block, lds, st, *inl, static_cast<C *>(psi),
                           static_cast<C *>(lam), gpart, gstride);
    } else {
        hipLaunchKernelGGL((k_tile<R, RB, NS>), grid, block, lds, st, static_cast<const unsigned char *>(dev),
                           (uint32_t)pass_off, (uint32_t)phase_off, (uint32_t)op_off, pass_idx,
                           static_cast<C *>(psi), static_cast<C *>(lam), gpart, gstride);
    }
    return hipGetLastError();
}

template <typename R, int NS>
hipError_t launch_rb(const PassDesc &hp, const InlineProg *inl, const void *dev, size_t a, size_t b, size_t c,
                     int pi, void *psi, void *lam, double *gp, int64_t gs, hipStream_t st) {
    switch (hp.rb) {
    case 1: return launch_one<R, 1, NS>(hp, inl, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 2: return launch_one<R, 2, NS>(hp, inl, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 3: return launch_one<R, 3, NS>(hp, inl, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 4: return launch_one<R, 4, NS>(hp, inl, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 5: return launch_one<R, 5, NS>(hp, inl, dev, a, b, c, pi, psi, lam, gp, gs, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_tile(bool c64, const PassDesc &hp, const InlineProg *inl, const void *dev, size_t pass_off,
                       size_t phase_off, size_t op_off, int pass_idx, int ns, void *psi, void *lam, double *gpart,
                       int64_t gstride, hipStream_t st) {
    if (hp.n_tiles == 0 || hp.n_tiles > 0x7fffffffull || hp.tb > kMaxThreadBits || hp.n_phase < 1)
        return hipErrorInvalidValue;
    if (ns == 2) {
        return c64 ? launch_rb<float, 2>(hp, inl, dev, pass_off, phase_off, op_off, pass_idx, psi, lam, gpart, gstride, st)
                   : launch_rb<double, 2>(hp, inl, dev, pass_off, phase_off, op_off, pass_idx, psi, lam, gpart, gstride, st);
    }
    return c64 ? launch_rb<float, 1>(hp, inl, dev, pass_off, phase_off, op_off, pass_idx, psi, nullptr, nullptr, 0, st)
               : launch_rb<double, 1>(hp, inl, dev, pass_off, phase_off, op_off, pass_idx, psi, nullptr, nullptr, 0, st);
}

}  // namespace qg
