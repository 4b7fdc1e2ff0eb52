// qg_tile_dev.h -- device-side pieces of a tile pass, shared by the pass kernel
// (one tile per workgroup) and the batched persistent kernel (whole circuits per
// workgroup).  See qg_internal.h for the program format.
//
// Thread `tid` holds amplitudes a[s][e], e in [0, 2^RB), of state s (psi, and
// lambda in adjoint sweeps) at tile position tp(tid) | ep(e); global index
// gbase(tile) | tg(tid) | eg(e).  In a batched launch a workgroup may have more
// threads than the tile needs; threads with tid >= 2^tb are inactive: they
// take part in barriers only.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "qg_internal.h"

namespace qg {
namespace dev {

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

// The same XOR map for a tile held as separate real or imaginary parts (slots
// of sizeof(R) bytes: 2^S of them span the 256 bytes of all LDS banks).
template <typename R>
__device__ __forceinline__ uint32_t swz_half(uint32_t p) {
    constexpr uint32_t S = sizeof(R) == 8 ? 5 : 6;
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

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_nt(const double2 *p) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    double2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
__device__ __forceinline__ float2 ld_nt(const float2 *p) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    float2 r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
__device__ __forceinline__ void st_nt(double2 *p, double2 a) {
    d2v v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, reinterpret_cast<d2v *>(p));
}
__device__ __forceinline__ void st_nt(float2 *p, float2 a) {
    f2v v;
    v.x = a.x;
    v.y = a.y;
    __builtin_nontemporal_store(v, reinterpret_cast<f2v *>(p));
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

// The fused diagonal runs of the running program (null where a program has none).
struct DiagTables {
    const DiagRun *runs;
    const DiagEntry *entries;
};

// (r, i) *= the product of entries [begin, end) for this thread: f1 where the
// entry's qubits are all 1, else f0.  The part of the condition on qubits
// outside the tile is the same for the whole tile, and where it fails an entry
// with f0 = 1 is skipped.
__device__ __forceinline__ void entries_mul(const DiagEntry *__restrict__ es, int begin, int end, uint64_t gbase,
                                            uint32_t tp, double &r, double &i) {
    for (int k = begin; k < end; ++k) {
        const DiagEntry &x = es[k];
        const bool tile_on = (gbase & x.gmask) == x.gmask;
        if (!tile_on && x.f0_one) continue;
        const bool on = tile_on && (tp & x.tmask) == x.tmask;
        const double fr = on ? x.f1[0] : x.f0[0], fi = on ? x.f1[1] : x.f0[1];
        const double nr = r * fr - i * fi;
        i = r * fi + i * fr;
        r = nr;
    }
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

// The register ops read `a` and write every element of `o` (o may be a).
template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_mat(const C (&a)[NS][NR], C (&o)[NS][NR], const R (&m)[8]) {
    constexpr int jb = 1 << J;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            if (e & jb) continue;
            const C v0 = a[s][e], v1 = a[s][e | jb];
            mat2(m, v0, v1, o[s][e], o[s][e | jb]);
        }
}

// Real matrix m = {m00, -, m01, -, m10, -, m11, -} on register slot J.
template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_matr(const C (&a)[NS][NR], C (&o)[NS][NR], const R (&m)[8]) {
    constexpr int jb = 1 << J;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            if (e & jb) continue;
            const C v0 = a[s][e], v1 = a[s][e | jb];
            o[s][e].x = m[0] * v0.x + m[2] * v1.x;
            o[s][e].y = m[0] * v0.y + m[2] * v1.y;
            o[s][e | jb].x = m[4] * v0.x + m[6] * v1.x;
            o[s][e | jb].y = m[4] * v0.y + m[6] * v1.y;
        }
}

// Real diagonal, imaginary off-diagonal: m = {m00, -, -, Im m01, -, Im m10, m11, -}.
template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_matrx(const C (&a)[NS][NR], C (&o)[NS][NR], const R (&m)[8]) {
    constexpr int jb = 1 << J;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int e = 0; e < NR; ++e) {
            if (e & jb) continue;
            const C v0 = a[s][e], v1 = a[s][e | jb];
            o[s][e].x = m[0] * v0.x - m[3] * v1.y;
            o[s][e].y = m[0] * v0.y + m[3] * v1.x;
            o[s][e | jb].x = m[6] * v1.x - m[5] * v0.y;
            o[s][e | jb].y = m[6] * v1.y + m[5] * v0.x;
        }
}

// Diagonal 1-qubit op on register slot J: factor {m0, m1} where the bit is 0,
// {m2, m3} where it is 1.
template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_diag1r(const C (&a)[NS][NR], C (&o)[NS][NR], const R (&m)[8]) {
    constexpr int jb = 1 << J;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int e = 0; e < NR; ++e) o[s][e] = (e & jb) ? cmul(a[s][e], m[2], m[3]) : cmul(a[s][e], m[0], m[1]);
}

// Phase {m0, m1} on the amplitudes whose register slots J and k are both 1
// (k is uniform, so the factor of each amplitude is a scalar choice).
template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_diag2rk(const C (&a)[NS][NR], C (&o)[NS][NR], const R (&m)[8], int k) {
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        if (!((e >> J) & 1)) {
#pragma unroll
            for (int s = 0; s < NS; ++s) o[s][e] = a[s][e];
            continue;
        }
        const bool on = (e >> k) & 1;
        const R re = on ? m[0] : (R)1, im = on ? m[1] : (R)0;
#pragma unroll
        for (int s = 0; s < NS; ++s) o[s][e] = cmul(a[s][e], re, im);
    }
}

// Multiplies the amplitudes whose register slot J is 1 by {re, im}.
template <int J, int NS, int NR, typename C, typename R>
__device__ __forceinline__ void apply_slot_factor(const C (&a)[NS][NR], C (&o)[NS][NR], R re, R im) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int e = 0; e < NR; ++e) o[s][e] = ((e >> J) & 1) ? cmul(a[s][e], re, im) : a[s][e];
}

// Slot dispatch: slots are < RB (the planner guarantees it).  A path that
// leaves the registers untouched would make the compiler copy all of them
// around every op, so impossible cases are marked unreachable.
#define QG_SLOT_SWITCH(slot, CALL)                                                         \
    switch (slot) {                                                                        \
    case 0: { constexpr int J_ = 0; CALL; } break;                                         \
    case 1: if constexpr (RB > 1) { constexpr int J_ = 1; CALL; } else __builtin_unreachable(); break; \
    case 2: if constexpr (RB > 2) { constexpr int J_ = 2; CALL; } else __builtin_unreachable(); break; \
    case 3: if constexpr (RB > 3) { constexpr int J_ = 3; CALL; } else __builtin_unreachable(); break; \
    case 4: if constexpr (RB > 4) { constexpr int J_ = 4; CALL; } else __builtin_unreachable(); break; \
    default: __builtin_unreachable();                                                      \
    }

// Controlled X whose control is not a register slot (a thread bit, or a qubit
// outside the tile): one condition per thread, the same for every pair on
// register slot J.
template <int J, int NS, int NR, typename C>
__device__ __forceinline__ void apply_cx(const C (&a)[NS][NR], C (&o)[NS][NR], bool on) {
    constexpr int jb = 1 << J;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        if (e & jb) continue;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C x = a[s][e], y = a[s][e | jb];
            o[s][e] = sel(on, y, x);
            o[s][e | jb] = sel(on, x, y);
        }
    }
}

// Controlled X with target slot J and control register slot k (uniform): the
// condition of each pair is a scalar (the element index is a constant after
// unrolling), so the exchange costs the selects alone.
template <int J, int NS, int NR, typename C>
__device__ __forceinline__ void apply_cx_slot(const C (&a)[NS][NR], C (&o)[NS][NR], int k) {
    constexpr int jb = 1 << J;
    const uint32_t km = 1u << k;
#pragma unroll
    for (int e = 0; e < NR; ++e) {
        if (e & jb) continue;
        const bool on = ((uint32_t)e & km) != 0u;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const C x = a[s][e], y = a[s][e | jb];
            o[s][e] = sel(on, y, x);
            o[s][e | jb] = sel(on, x, y);
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


// Adjoint partial of the X or Y generator on the runtime register slot
// `slot` (< RB); the last slot is the fall-through.
template <int J, int RB, int NS, typename C>
__device__ __forceinline__ double dispatch_grad_xy(int slot, const C (&a)[NS][1 << RB], bool isy) {
    if constexpr (J == RB - 1) {
        return grad_xy<J>(a, isy);
    } else {
        return slot == J ? grad_xy<J>(a, isy) : dispatch_grad_xy<J + 1, RB>(slot, a, isy);
    }
}

// Global index bits of logical tile w: deposit w into the free runs (after
// the optional swizzle).
__device__ __forceinline__ uint64_t tile_deposit(const PassDesc &P, uint64_t w) {
    uint64_t gbase = P.fixed_val;
    if (P.swz_bits > 0) {
        // Neighbouring blocks take tiles whose addresses differ in higher bits.
        const uint64_t m = (1ull << P.swz_bits) - 1;
        w ^= (w >> P.swz_bits) & m;
    }
    for (int r = 0; r < P.n_runs; ++r) {
        const int len = P.run_len[r];
        gbase |= (w & ((1ull << len) - 1)) << P.run_start[r];
        w >>= len;
    }
    return gbase;
}

// Global index bits of the tile of block w (one tile per block).
__device__ __forceinline__ uint64_t tile_gbase(const PassDesc &P, uint64_t w) {
    if (P.flags & PASS_XCD) {
        // Blocks are dealt to the 8 XCDs in turn: give each XCD a contiguous
        // eighth of the tiles.
        const int lt = 63 - __builtin_clzll(P.n_tiles);
        w = ((w & 7) << (lt - 3)) | (w >> 3);
    }
    return tile_deposit(P, w);
}

__device__ __forceinline__ uint64_t thread_goff(const PhaseDesc &ph, int tb, int tid) {
    uint64_t tg = 0;
    for (int k = 0; k < tb; ++k)
        if ((tid >> k) & 1) tg |= ph.thr_goff[k];
    return tg;
}

__device__ __forceinline__ uint32_t thread_poff(const PhaseDesc &ph, int tb, int tid) {
    uint32_t tp = 0;
    for (int k = 0; k < tb; ++k)
        if ((tid >> k) & 1) tp |= ph.thr_poff[k];
    return tp;
}

template <int RB>
__device__ __forceinline__ uint64_t elem_goff(const PhaseDesc &ph, int e) {
    uint64_t eg = 0;
#pragma unroll
    for (int j = 0; j < RB; ++j)
        if ((e >> j) & 1) eg |= ph.reg_goff[j];
    return eg;
}

template <int RB>
__device__ __forceinline__ uint32_t elem_poff(const PhaseDesc &ph, int e) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < RB; ++j)
        if ((e >> j) & 1) v |= ph.reg_poff[j];
    return v;
}

template <typename R, int RB, int NS>
__device__ __forceinline__ void tile_load(const PassDesc &P, const PhaseDesc &ph, uint64_t gbase,
                                          typename V2<R>::T *const (&st)[2],
                                          typename V2<R>::T (&a)[NS][1 << RB], int tid) {
    const bool nt = (P.flags & PASS_NT) != 0;
    const uint64_t tg = thread_goff(ph, P.tb, tid);
#pragma unroll
    for (int e = 0; e < (1 << RB); ++e) {
        const uint64_t off = gbase | tg | elem_goff<RB>(ph, e);
#pragma unroll
        for (int s = 0; s < NS; ++s) a[s][e] = nt ? ld_nt(st[s] + off) : st[s][off];
    }
}

template <typename R, int RB, int NS>
__device__ __forceinline__ void tile_store(const PassDesc &P, const PhaseDesc &ph, uint64_t gbase,
                                           typename V2<R>::T *const (&st)[2],
                                           const typename V2<R>::T (&a)[NS][1 << RB], int tid) {
    const bool nt = (P.flags & PASS_NT) != 0;
    const uint64_t tg = thread_goff(ph, P.tb, tid);
#pragma unroll
    for (int e = 0; e < (1 << RB); ++e) {
        const uint64_t off = gbase | tg | elem_goff<RB>(ph, e);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (nt) st_nt(st[s] + off, a[s][e]);
            else st[s][off] = a[s][e];
        }
    }
}

// |0...0> restricted to this tile.
template <typename R, int RB>
__device__ __forceinline__ void tile_zero(const PassDesc &P, const PhaseDesc &ph, uint64_t gbase,
                                          typename V2<R>::T (&a)[1][1 << RB], int tid) {
    const uint64_t tg = thread_goff(ph, P.tb, tid);
#pragma unroll
    for (int e = 0; e < (1 << RB); ++e) {
        a[0][e].x = (gbase | tg | elem_goff<RB>(ph, e)) == 0 ? (R)1 : (R)0;
        a[0][e].y = (R)0;
    }
}

// sum_e |a_e|^2 (sum_{q < n-1} Z_q Z_{q+1})(index of a_e): the open-chain ZZ
// observable, (n-1) - 2 popcount((i ^ (i >> 1)) & (2^(n-1) - 1)).
template <typename R, int RB>
__device__ __forceinline__ double tile_obs_zz_chain(const PassDesc &P, const PhaseDesc &ph, uint64_t gbase,
                                                    const typename V2<R>::T (&a)[1][1 << RB], int tid, int n) {
    const uint64_t tg = thread_goff(ph, P.tb, tid);
    const uint64_t mask = n >= 2 ? ((1ull << (n - 1)) - 1) : 0;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < (1 << RB); ++e) {
        const uint64_t i = gbase | tg | elem_goff<RB>(ph, e);
        const double p = (double)a[0][e].x * a[0][e].x + (double)a[0][e].y * a[0][e].y;
        acc += p * ((double)(n - 1) - 2.0 * (double)__popcll((i ^ (i >> 1)) & mask));
    }
    return acc;
}

// sum_e |a_e|^2 sum_t coeff_t (-1)^{popcount(i & mask_t)}
template <typename R, int RB>
__device__ __forceinline__ double tile_obs_terms(const PassDesc &P, const PhaseDesc &ph, uint64_t gbase,
                                                 const typename V2<R>::T (&a)[1][1 << RB], int tid,
                                                 const uint64_t *__restrict__ masks, const double *__restrict__ coeff,
                                                 int n_terms) {
    const uint64_t tg = thread_goff(ph, P.tb, tid);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < (1 << RB); ++e) {
        const uint64_t i = gbase | tg | elem_goff<RB>(ph, e);
        const double p = (double)a[0][e].x * a[0][e].x + (double)a[0][e].y * a[0][e].y;
        double o = 0.0;
        for (int t = 0; t < n_terms; ++t) o += (__popcll(i & masks[t]) & 1) ? -coeff[t] : coeff[t];
        acc += p * o;
    }
    return acc;
}

// One op of a phase: reads the registers `a`, writes every element of `o`
// (o may be a); gradient ops (adjoint sweeps) also write their per-wave
// partial sum and copy a to o.
template <typename R, int RB, int NS>
__device__ __forceinline__ void apply_op(const DevOp &op, const DiagTables &dt, const typename V2<R>::T (&a)[NS][1 << RB],
                                         typename V2<R>::T (&o)[NS][1 << RB], uint64_t gbase, uint32_t tp,
                                         const uint32_t (&ep)[1 << RB], double *__restrict__ gpart,
                                         int64_t gstride, uint64_t tile_idx, int tid) {
    constexpr int NR = 1 << RB;
    R m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = (R)op.m[k];
    const int kind = op.kind;
    if (kind == OP_MAT) {
        QG_SLOT_SWITCH(op.a, (apply_mat<J_>(a, o, m)));
    } else if (kind == OP_MATR) {
        QG_SLOT_SWITCH(op.a, (apply_matr<J_>(a, o, m)));
    } else if (kind == OP_MATRX) {
        QG_SLOT_SWITCH(op.a, (apply_matrx<J_>(a, o, m)));
    } else if (kind == OP_CX) {
        // The control is a thread bit or lies outside the tile (constant over
        // it); when it is 0 every select keeps the input (no branch: a path
        // that leaves the registers untouched makes the compiler copy all of
        // them).
        const bool on = make_bit(op.c, gbase).of(tp);
        QG_SLOT_SWITCH(op.a, (apply_cx<J_>(a, o, on)));
    } else if (kind == OP_CXRR) {
        QG_SLOT_SWITCH(op.a, (apply_cx_slot<J_>(a, o, op.c)));
    } else if (kind == OP_DIAG1R) {
        QG_SLOT_SWITCH(op.a, (apply_diag1r<J_>(a, o, m)));
    } else if (kind == OP_DIAG2RR) {
        QG_SLOT_SWITCH(op.a, (apply_diag2rk<J_>(a, o, m, op.c)));
    } else if (kind == OP_DIAG2R) {
        // the other qubit is a thread bit or outside the tile: one
        // factor per thread
        const bool on = make_bit(op.c, gbase).of(tp);
        const R re = on ? m[0] : (R)1, im = on ? m[1] : (R)0;
        QG_SLOT_SWITCH(op.a, (apply_slot_factor<J_>(a, o, re, im)));
    } else if (kind == OP_DIAGRUN) {
        // Factor of element e: tf * prod_{slot j of e} r_j * prod_{slots j<k of e} q_jk,
        // built in FP64 from the element without its top slot bit.
        const DiagRun &d = dt.runs[op.a];
        double tr = d.c0[0], ti = d.c0[1];
        entries_mul(dt.entries, d.e_begin, d.s_begin[0], gbase, tp, tr, ti);
        double rr[RB], ri[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            rr[j] = d.r[j][0];
            ri[j] = d.r[j][1];
            entries_mul(dt.entries, d.s_begin[j], d.s_begin[j + 1], gbase, tp, rr[j], ri[j]);
        }
        double fr[NR], fi[NR];
        fr[0] = tr;
        fi[0] = ti;
#pragma unroll
        for (int s = 0; s < NS; ++s) o[s][0] = cmul(a[s][0], (R)tr, (R)ti);
#pragma unroll
        for (int e = 1; e < NR; ++e) {
            const int j = 31 - __builtin_clz((unsigned)e);
            const int e0 = e ^ (1 << j);
            double xr = fr[e0] * rr[j] - fi[e0] * ri[j], xi = fr[e0] * ri[j] + fi[e0] * rr[j];
#pragma unroll
            for (int k = 0; k < j; ++k) {
                if (!((e0 >> k) & 1)) continue;
                const double qr = d.q[j * (j - 1) / 2 + k][0], qi = d.q[j * (j - 1) / 2 + k][1];
                const double nr = xr * qr - xi * qi;
                xi = xr * qi + xi * qr;
                xr = nr;
            }
            fr[e] = xr;
            fi[e] = xi;
            // applied at once, so that only the factors still needed as parents stay live
#pragma unroll
            for (int s = 0; s < NS; ++s) o[s][e] = cmul(a[s][e], (R)xr, (R)xi);
        }
    } else if (kind == OP_DIAG1) {
        // thread bit or outside the tile: one factor per thread
        const bool one = make_bit(op.a, gbase).of(tp);
        const R re = one ? m[2] : m[0], im = one ? m[3] : m[1];
#pragma unroll
        for (int e = 0; e < NR; ++e)
#pragma unroll
            for (int s = 0; s < NS; ++s) o[s][e] = cmul(a[s][e], re, im);
    } else if (kind == OP_DIAG2) {
        const bool on = make_bit(op.a, gbase).of(tp) && make_bit(op.c, gbase).of(tp);
        const R re = on ? m[0] : (R)1, im = on ? m[1] : (R)0;
#pragma unroll
        for (int e = 0; e < NR; ++e)
#pragma unroll
            for (int s = 0; s < NS; ++s) o[s][e] = cmul(a[s][e], re, im);
    } else if constexpr (NS == 1) {
        __builtin_unreachable();  // gradient ops only occur in adjoint programs
    } else {
        {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < NR; ++e) o[s][e] = a[s][e];
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
                acc = dispatch_grad_xy<0, RB>(op.a, a, isy);
            }
            const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
            acc = wave_sum(acc, width);
            if ((tid & (width - 1)) == 0) {
                const int waves = (blockDim.x + 63) / 64;
                gpart[(int64_t)op.g * gstride + (int64_t)tile_idx * waves + tid / 64] = acc;
            }
        }
    }
}

// Runs every phase of a pass on the registers: LDS exchanges between layouts,
// then the phase's ops.  `active` is false for threads beyond the tile's 2^tb.
template <typename R, int RB, int NS>
__device__ __forceinline__ void tile_phases(const PassDesc &P, const PhaseDesc *__restrict__ phases,
                                            const DevOp *__restrict__ ops, const DiagTables &dt, uint64_t gbase,
                                            typename V2<R>::T (&a)[NS][1 << RB], typename V2<R>::T *lds,
                                            double *__restrict__ gpart, int64_t gstride, uint64_t tile_idx,
                                            int tid, bool active) {
    using C = typename V2<R>::T;
    constexpr int NR = 1 << RB;
    const int tb = P.tb;
    const int n_phase = P.n_phase;
    for (int p = 0; p < n_phase; ++p) {
        const PhaseDesc &ph = phases[p];
        const uint32_t tp = thread_poff(ph, tb, tid);
        uint32_t ep[NR];
#pragma unroll
        for (int e = 0; e < NR; ++e) ep[e] = elem_poff<RB>(ph, e);
        if (p > 0) {
            // Move the tile into the new register layout through LDS.
            // The slot map is XOR-linear and thread and register offsets have
            // disjoint bits, so swz(t | r) = swz(t) ^ swz(r): one per-thread
            // term and one uniform (scalar) term per element.
            // (readfirstlane keeps the uniform term from being folded back into
            // the per-thread expression.)  Offsets are in bytes.
            const PhaseDesc &prev = phases[p - 1];
            unsigned char *lb = reinterpret_cast<unsigned char *>(lds);
            if (P.flags & PASS_HALFX) {
                // Half the LDS: the real parts go through first, then the
                // imaginary parts (twice the barriers, half the bytes per
                // workgroup, so more workgroups fit on a CU).
                constexpr uint32_t SZ = sizeof(R);
                const uint32_t sq = swz_half<R>(thread_poff(prev, tb, tid)) * SZ, sp = swz_half<R>(tp) * SZ;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    R t[NR];
                    __syncthreads();
                    if (active) {
#pragma unroll
                        for (int e = 0; e < NR; ++e) {
                            const uint32_t u = __builtin_amdgcn_readfirstlane(swz_half<R>(elem_poff<RB>(prev, e)) * SZ);
                            *reinterpret_cast<R *>(lb + (sq ^ u)) = a[s][e].x;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int e = 0; e < NR; ++e) {
                        const uint32_t u = __builtin_amdgcn_readfirstlane(swz_half<R>(ep[e]) * SZ);
                        t[e] = *reinterpret_cast<const R *>(lb + (sp ^ u));
                    }
                    __syncthreads();
                    if (active) {
#pragma unroll
                        for (int e = 0; e < NR; ++e) {
                            const uint32_t u = __builtin_amdgcn_readfirstlane(swz_half<R>(elem_poff<RB>(prev, e)) * SZ);
                            *reinterpret_cast<R *>(lb + (sq ^ u)) = a[s][e].y;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int e = 0; e < NR; ++e) {
                        const uint32_t u = __builtin_amdgcn_readfirstlane(swz_half<R>(ep[e]) * SZ);
                        a[s][e].x = t[e];
                        a[s][e].y = *reinterpret_cast<const R *>(lb + (sp ^ u));
                    }
                }
            } else {
            constexpr uint32_t SZ = sizeof(C);
            const uint32_t sq = swz<R>(thread_poff(prev, tb, tid)) * SZ, sp = swz<R>(tp) * SZ;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                __syncthreads();
                if (active) {
#pragma unroll
                    for (int e = 0; e < NR; ++e) {
                        const uint32_t u = __builtin_amdgcn_readfirstlane(swz<R>(elem_poff<RB>(prev, e)) * SZ);
                        *reinterpret_cast<C *>(lb + (sq ^ u)) = a[s][e];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < NR; ++e) {
                    const uint32_t u = __builtin_amdgcn_readfirstlane(swz<R>(ep[e]) * SZ);
                    a[s][e] = *reinterpret_cast<const C *>(lb + (sp ^ u));
                }
            }
            }
        }
        // Each op reads one register set and writes the other, so that no op
        // has to update its inputs in place (which costs a copy of every
        // register per op at the loop's back edge).
        // The descriptor of the op after next is loaded while the current pair
        // runs: a long program does not fit the scalar cache, and a descriptor
        // fetched only when its op starts would expose the memory latency once
        // per op.  (The look-ahead index stays inside the phase.)
        C b[NS][NR];
        const int end = ph.op_end;
        int i = ph.op_begin;
        if (i < end) {
            DevOp c0 = ops[i];
            for (; i + 1 < end; i += 2) {
                const DevOp c1 = ops[i + 1];
                apply_op<R, RB, NS>(c0, dt, a, b, gbase, tp, ep, gpart, gstride, tile_idx, tid);
                const DevOp c2 = ops[i + 2 < end ? i + 2 : end - 1];
                apply_op<R, RB, NS>(c1, dt, b, a, gbase, tp, ep, gpart, gstride, tile_idx, tid);
                c0 = c2;
            }
            if (i < end) apply_op<R, RB, NS>(c0, dt, a, a, gbase, tp, ep, gpart, gstride, tile_idx, tid);
        }
    }
}

}  // namespace dev
}  // namespace qg
