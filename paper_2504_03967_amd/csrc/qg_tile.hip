// qg_tile.hip -- the pass kernel: streams every active tile of the state through
// registers once and applies a pass's ops (App. A: single-qubit operators of
// eq. (tp), controlled operators of eq. (cx), the diagonal CR1 of eq. (cr1)).
//
// Layout of one workgroup's tile (b tile qubits = tb thread bits + rb register
// bits): thread `tid` holds amplitudes a[e], e in [0, 2^rb), at tile position
// tp(tid) | ep(e), where the current phase decides which tile positions are
// register bits.  A phase change moves the tile through LDS.  The global
// index of (tid, e) is gbase(tile) | tg(tid) | eg(e); with the lowest tile
// positions on consecutive lanes, every wavefront load/store of fixed e is a
// run of contiguous amplitudes (one HBM read and write per pass).
#include <type_traits>

#include "qg_kernels.h"

namespace qg {
namespace {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

// LDS slot of tile position p: XOR-swizzle the low bits of a 256-byte bank row
// with the next bits so that strided register layouts spread over the banks.
template <typename R>
__device__ __forceinline__ uint32_t swz(uint32_t p) {
    constexpr uint32_t S = sizeof(R) == 8 ? 4 : 5;
    return p ^ ((p >> S) & ((1u << S) - 1));
}

template <typename C, typename R>
__device__ __forceinline__ void mat2(const R (&m)[8], C v0, C v1, C &o0, C &o1) {
    o0.x = m[0] * v0.x - m[1] * v0.y + m[2] * v1.x - m[3] * v1.y;
    o0.y = m[0] * v0.y + m[1] * v0.x + m[2] * v1.y + m[3] * v1.x;
    o1.x = m[4] * v0.x - m[5] * v0.y + m[6] * v1.x - m[7] * v1.y;
    o1.y = m[4] * v0.y + m[5] * v0.x + m[6] * v1.y + m[7] * v1.x;
}

template <typename C, typename R>
__device__ __forceinline__ C cmul(C v, R re, R im) {
    C o;
    o.x = v.x * re - v.y * im;
    o.y = v.x * im + v.y * re;
    return o;
}

__device__ __forceinline__ double wave_sum(double v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
    return v;
}

// Index bit of a qubit reference: a tile position (bit of the amplitude's
// tile position) or a qubit outside the tile (constant over the tile).
struct Bit {
    uint32_t mask;
    bool fixed_one;
    __device__ __forceinline__ bool of(uint32_t pos) const { return mask ? (pos & mask) != 0 : fixed_one; }
};

__device__ __forceinline__ Bit make_bit(int ref, uint64_t gbase) {
    Bit b;
    b.mask = ref >= 0 ? (1u << ref) : 0u;
    b.fixed_one = ref < 0 && ((gbase >> (-1 - ref)) & 1ull);
    return b;
}

// Component-wise select (a select of whole 16-byte vectors can become a select
// of their addresses, which forces the register arrays into scratch memory).
template <typename C>
__device__ __forceinline__ C sel(bool c, C x, C y) {
    C o;
    o.x = c ? x.x : y.x;
    o.y = c ? x.y : y.y;
    return o;
}

// Im(conj(l) * p)
template <typename C>
__device__ __forceinline__ double im_conj_mul(C l, C p) {
    return (double)l.x * p.y - (double)l.y * p.x;
}

template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_mat(C (&a)[NS][NR], const R (&m)[8]) {
    constexpr int jb = 1 << J;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            if (e & jb) continue;
            const C v0 = a[s][e], v1 = a[s][e | jb];
            mat2(m, v0, v1, a[s][e], a[s][e | jb]);
        }
}

template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_cmat(C (&a)[NS][NR], const R (&m)[8], uint32_t tp, const uint32_t (&ep)[NR],
                                           int cref) {
    constexpr int jb = 1 << J;
    const uint32_t cm = cref >= 0 ? (1u << cref) : 0u;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        if (e & jb) continue;
        const bool on = cm == 0u || ((tp | ep[e]) & cm) != 0u;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            C o0, o1;
            mat2(m, a[s][e], a[s][e | jb], o0, o1);
            a[s][e] = sel(on, o0, a[s][e]);
            a[s][e | jb] = sel(on, o1, a[s][e | jb]);
        }
    }
}

// sum_e Im(conj(lam_e) (P psi)_e) for P = X or Y on register slot J.
template <int J, int NS, int NR, typename C>
__device__ __forceinline__ double grad_xy(const C (&a)[NS][NR], bool isy) {
    constexpr int jb = 1 << J;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        const C l = a[NS - 1][e], q = a[0][e ^ jb];
        if (isy) {
            const double v = (double)l.x * q.x + (double)l.y * q.y;
            acc += (e & jb) ? v : -v;
        } else {
            acc += im_conj_mul(l, q);
        }
    }
    return acc;
}

template <typename R, int RB, int NS>
__global__ void __launch_bounds__(256)
k_tile(const unsigned char *__restrict__ dev, uint32_t pass_off, uint32_t phase_off, uint32_t op_off,
       int pass_idx, typename V2<R>::T *__restrict__ psi, typename V2<R>::T *__restrict__ lam,
       double *__restrict__ gpart, int64_t gstride) {
    using C = typename V2<R>::T;
    constexpr int NR = 1 << RB;
    const PassDesc &P = reinterpret_cast<const PassDesc *>(dev + pass_off)[pass_idx];
    const PhaseDesc *phases = reinterpret_cast<const PhaseDesc *>(dev + phase_off) + P.phase_begin;
    const DevOp *ops = reinterpret_cast<const DevOp *>(dev + op_off);
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);

    const int tid = threadIdx.x;
    const int tb = P.tb;

    // Global index bits of this tile: deposit the block index into the free runs.
    uint64_t gbase = P.fixed_val;
    {
        uint64_t w = blockIdx.x;
        for (int r = 0; r < P.n_runs; ++r) {
            const int len = P.run_len[r];
            gbase |= (w & ((1ull << len) - 1)) << P.run_start[r];
            w >>= len;
        }
    }

    C a[NS][NR];
    C *const st[2] = {psi, lam};

    // Load in the first phase's layout.
    {
        const PhaseDesc &ph = phases[0];
        uint64_t tg = 0;
        for (int k = 0; k < tb; ++k)
            if ((tid >> k) & 1) tg |= ph.thr_goff[k];
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            uint64_t eg = 0;
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if ((e >> j) & 1) eg |= ph.reg_goff[j];
            const uint64_t off = gbase | tg | eg;
#pragma unroll
            for (int s = 0; s < NS; ++s) a[s][e] = st[s][off];
        }
    }

    const int n_phase = P.n_phase;
    for (int p = 0; p < n_phase; ++p) {
        const PhaseDesc &ph = phases[p];
        uint32_t tp = 0;
        for (int k = 0; k < tb; ++k)
            if ((tid >> k) & 1) tp |= ph.thr_poff[k];
        uint32_t ep[NR];
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if ((e >> j) & 1) v |= ph.reg_poff[j];
            ep[e] = v;
        }
        if (p > 0) {
            // Move the tile into the new register layout through LDS.
            const PhaseDesc &prev = phases[p - 1];
            uint32_t tq = 0;
            for (int k = 0; k < tb; ++k)
                if ((tid >> k) & 1) tq |= prev.thr_poff[k];
            uint32_t eq[NR];
#pragma unroll
            for (int e = 0; e < NR; ++e) {
                uint32_t v = 0;
#pragma unroll
                for (int j = 0; j < RB; ++j)
                    if ((e >> j) & 1) v |= prev.reg_poff[j];
                eq[e] = v;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                __syncthreads();
#pragma unroll
                for (int e = 0; e < NR; ++e) lds[swz<R>(tq | eq[e])] = a[s][e];
                __syncthreads();
#pragma unroll
                for (int e = 0; e < NR; ++e) a[s][e] = lds[swz<R>(tp | ep[e])];
            }
        }

        for (int i = ph.op_begin; i < ph.op_end; ++i) {
            const DevOp &op = ops[i];
            R m[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) m[k] = (R)op.m[k];
            const int kind = op.kind;
            if (kind == OP_MAT) {
                switch (op.a) {
                case 0: apply_mat<0>(a, m); break;
                case 1: if constexpr (RB > 1) apply_mat<1>(a, m); break;
                case 2: if constexpr (RB > 2) apply_mat<2>(a, m); break;
                case 3: if constexpr (RB > 3) apply_mat<3>(a, m); break;
                case 4: if constexpr (RB > 4) apply_mat<4>(a, m); break;
                }
            } else if (kind == OP_CMAT) {
                if (op.c < 0 && !((gbase >> (-1 - op.c)) & 1ull)) continue;
                switch (op.a) {
                case 0: apply_cmat<0>(a, m, tp, ep, op.c); break;
                case 1: if constexpr (RB > 1) apply_cmat<1>(a, m, tp, ep, op.c); break;
                case 2: if constexpr (RB > 2) apply_cmat<2>(a, m, tp, ep, op.c); break;
                case 3: if constexpr (RB > 3) apply_cmat<3>(a, m, tp, ep, op.c); break;
                case 4: if constexpr (RB > 4) apply_cmat<4>(a, m, tp, ep, op.c); break;
                }
            } else if (kind == OP_DIAG1) {
                const Bit ba = make_bit(op.a, gbase);
#pragma unroll
                for (int e = 0; e < NR; ++e) {
                    const bool one = ba.of(tp | ep[e]);
                    const R re = one ? m[2] : m[0], im = one ? m[3] : m[1];
#pragma unroll
                    for (int s = 0; s < NS; ++s) a[s][e] = cmul(a[s][e], re, im);
                }
            } else if (kind == OP_DIAG2) {
                const Bit ba = make_bit(op.a, gbase), bc = make_bit(op.c, gbase);
#pragma unroll
                for (int e = 0; e < NR; ++e) {
                    const bool both = ba.of(tp | ep[e]) && bc.of(tp | ep[e]);
#pragma unroll
                    for (int s = 0; s < NS; ++s) a[s][e] = sel(both, cmul(a[s][e], m[0], m[1]), a[s][e]);
                }
            } else {
                if constexpr (NS == 2) {
                    double acc = 0.0;
                    if (kind == OP_GRADZ) {
                        const Bit ba = make_bit(op.a, gbase);
#pragma unroll
                        for (int e = 0; e < NR; ++e) {
                            const double v = im_conj_mul(a[1][e], a[0][e]);
                            acc += ba.of(tp | ep[e]) ? -v : v;
                        }
                    } else if (kind == OP_GRADP11) {
                        const Bit ba = make_bit(op.a, gbase), bc = make_bit(op.c, gbase);
#pragma unroll
                        for (int e = 0; e < NR; ++e) {
                            const double v = im_conj_mul(a[1][e], a[0][e]);
                            acc += (ba.of(tp | ep[e]) && bc.of(tp | ep[e])) ? -2.0 * v : 0.0;
                        }
                    } else {
                        const bool isy = kind == OP_GRADY;
                        switch (op.a) {
                        case 0: acc = grad_xy<0>(a, isy); break;
                        case 1: if constexpr (RB > 1) acc = grad_xy<1>(a, isy); break;
                        case 2: if constexpr (RB > 2) acc = grad_xy<2>(a, isy); break;
                        case 3: if constexpr (RB > 3) acc = grad_xy<3>(a, isy); break;
                        case 4: if constexpr (RB > 4) acc = grad_xy<4>(a, isy); break;
                        }
                    }
                    const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
                    acc = wave_sum(acc, width);
                    if ((tid & (width - 1)) == 0) {
                        const int waves = (blockDim.x + 63) / 64;
                        gpart[(int64_t)op.g * gstride + (int64_t)blockIdx.x * waves + tid / 64] = acc;
                    }
                }
            }
        }
    }

    // Store in the last phase's layout.
    {
        const PhaseDesc &ph = phases[n_phase - 1];
        uint64_t tg = 0;
        for (int k = 0; k < tb; ++k)
            if ((tid >> k) & 1) tg |= ph.thr_goff[k];
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            uint64_t eg = 0;
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if ((e >> j) & 1) eg |= ph.reg_goff[j];
            const uint64_t off = gbase | tg | eg;
#pragma unroll
            for (int s = 0; s < NS; ++s) st[s][off] = a[s][e];
        }
    }
}

template <typename R, int RB, int NS>
hipError_t launch_one(const PassDesc &hp, const void *dev, size_t pass_off, size_t phase_off,
                      size_t op_off, int pass_idx, void *psi, void *lam, double *gpart,
                      int64_t gstride, hipStream_t st) {
    using C = typename V2<R>::T;
    const size_t lds = hp.n_phase > 1 ? (size_t(1) << hp.b) * sizeof(C) : 0;
    if (lds > 65536) {
        static bool done = false;
        if (!done) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile<R, RB, NS>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            done = true;
        }
    }
    dim3 grid((uint32_t)hp.n_tiles), block(1u << hp.tb);
    hipLaunchKernelGGL((k_tile<R, RB, NS>), grid, block, lds, st,
                       static_cast<const unsigned char *>(dev), (uint32_t)pass_off, (uint32_t)phase_off,
                       (uint32_t)op_off, pass_idx, static_cast<C *>(psi), static_cast<C *>(lam), gpart,
                       gstride);
    return hipGetLastError();
}

template <typename R, int NS>
hipError_t launch_rb(const PassDesc &hp, const void *dev, size_t a, size_t b, size_t c, int pi,
                     void *psi, void *lam, double *gp, int64_t gs, hipStream_t st) {
    switch (hp.rb) {
    case 1: return launch_one<R, 1, NS>(hp, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 2: return launch_one<R, 2, NS>(hp, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 3: return launch_one<R, 3, NS>(hp, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 4: return launch_one<R, 4, NS>(hp, dev, a, b, c, pi, psi, lam, gp, gs, st);
    case 5: return launch_one<R, 5, NS>(hp, dev, a, b, c, pi, psi, lam, gp, gs, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_tile(bool c64, const PassDesc &hp, const void *dev, size_t pass_off, size_t phase_off,
                       size_t op_off, int pass_idx, int ns, void *psi, void *lam, double *gpart,
                       int64_t gstride, hipStream_t st) {
    if (hp.n_tiles == 0 || hp.n_tiles > 0x7fffffffull || hp.tb > kMaxThreadBits || hp.n_phase < 1)
        return hipErrorInvalidValue;
    if (ns == 2) {
        return c64 ? launch_rb<float, 2>(hp, dev, pass_off, phase_off, op_off, pass_idx, psi, lam, gpart, gstride, st)
                   : launch_rb<double, 2>(hp, dev, pass_off, phase_off, op_off, pass_idx, psi, lam, gpart, gstride, st);
    }
    return c64 ? launch_rb<float, 1>(hp, dev, pass_off, phase_off, op_off, pass_idx, psi, nullptr, nullptr, 0, st)
               : launch_rb<double, 1>(hp, dev, pass_off, phase_off, op_off, pass_idx, psi, nullptr, nullptr, 0, st);
}

}  // namespace qg
