// qg_perm.hip -- standalone single-gate kernels outside the tile pass: SWAP of
// two qubits as a pure permutation, and one-qubit gates or CX whose target lies
// inside a cache line as a cross-lane exchange.
//
// k_swap2: only the amplitudes whose two bits differ move (half the state),
// each exchanged with its partner.  Used for a standalone SWAP whose lower
// qubit is at or above the cache-line offset bits, so every wavefront access
// covers whole 128-byte lines.
//
// k_swap_lane: the lower qubit lies inside a cache line, so every line holds
// moving amplitudes and the whole state is streamed.  Each wavefront loads 64
// consecutive amplitudes (coalesced) and exchanges partners across lanes.
//
// k_lane_gate: a single one-qubit gate (or CX) whose target lies inside a
// cache line, with the same coalesced loads and cross-lane exchange.
//
// Every wavefront access covers whole lines, so all use non-temporal loads
// and stores (measured: 4.8 -> 5.8 TB/s for SWAP(15, 16) on 30 qubits).
#include "qg_kernels.h"
#include "qg_tile_dev.h"

namespace qg {
namespace {

template <typename C, int U>
__global__ void __launch_bounds__(256) k_swap2(C *__restrict__ psi, int lo, int hi, uint64_t bit_a, uint64_t bit_b,
                                               uint64_t n_pairs, int xcd_shift) {
    // pair p: insert zeros at lo then hi; the two members carry bit_a or bit_b.
    uint64_t blk = blockIdx.x;
    if (xcd_shift > 0) blk = ((blk & 7) << xcd_shift) | (blk >> 3);  // gridDim.x = 8 << xcd_shift
    const uint64_t base_p = (blk * blockDim.x * U) + threadIdx.x;
    C va[U], vb[U];
    uint64_t ia[U], ib[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t p = base_p + (uint64_t)u * blockDim.x;
        uint64_t x = ((p >> lo) << (lo + 1)) | (p & ((1ull << lo) - 1));
        x = ((x >> hi) << (hi + 1)) | (x & ((1ull << hi) - 1));
        ia[u] = x | bit_a;
        ib[u] = x | bit_b;
        if (p < n_pairs) {
            va[u] = dev::ld_nt(psi + ia[u]);
            vb[u] = dev::ld_nt(psi + ib[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t p = base_p + (uint64_t)u * blockDim.x;
        if (p < n_pairs) {
            dev::st_nt(psi + ia[u], vb[u]);
            dev::st_nt(psi + ib[u], va[u]);
        }
    }
}

// Lane bits: the lower SWAP qubit lo < 6 is a lane bit of every wavefront access.
// hi < 6 too: one load per element, partner = lane with bits lo and hi exchanged.
// hi >= 6: pair p holds amplitude i0 (bit hi = 0) and i1 = i0 | 2^hi, both on the
// same lane; an i0 with bit lo set swaps with the i1 of the lane across bit lo.
template <typename C, int U>
__global__ void __launch_bounds__(256) k_swap_lane(C *__restrict__ psi, int lo, int hi, uint64_t n_items,
                                                   int xcd_shift) {
    uint64_t blk = blockIdx.x;
    if (xcd_shift > 0) blk = ((blk & 7) << xcd_shift) | (blk >> 3);  // gridDim.x = 8 << xcd_shift
    const uint64_t base = blk * blockDim.x * U + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int mlo = 1 << lo;
    const bool blo = (lane >> lo) & 1;
    if (hi < 6) {
        const bool moves = blo != (((lane >> hi) & 1) != 0);
        const int mask = mlo | (1 << hi);
        C v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = dev::ld_nt(psi + base + (uint64_t)u * blockDim.x);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            C w;
            w.x = __shfl_xor(v[u].x, mask, 64);
            w.y = __shfl_xor(v[u].y, mask, 64);
            if (moves) v[u] = w;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) dev::st_nt(psi + base + (uint64_t)u * blockDim.x, v[u]);
    } else {
        const uint64_t bh = 1ull << hi;
        C v0[U], v1[U];
        uint64_t i0[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t p = base + (uint64_t)u * blockDim.x;
            i0[u] = ((p >> hi) << (hi + 1)) | (p & (bh - 1));
            v0[u] = dev::ld_nt(psi + i0[u]);
            v1[u] = dev::ld_nt(psi + (i0[u] | bh));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            C a, b;
            a.x = __shfl_xor(v1[u].x, mlo, 64);
            a.y = __shfl_xor(v1[u].y, mlo, 64);
            b.x = __shfl_xor(v0[u].x, mlo, 64);
            b.y = __shfl_xor(v0[u].y, mlo, 64);
            if (blo) v0[u] = a;
            else v1[u] = b;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dev::st_nt(psi + i0[u], v0[u]);
            dev::st_nt(psi + (i0[u] | bh), v1[u]);
        }
    }
    (void)n_items;
}

// One-qubit gate (or CX) on a target t < 6, a lane bit: lane l holds amplitude
// i (64 consecutive per wavefront, whole lines) and its partner i ^ 2^t sits on
// lane l ^ 2^t.  Output = m_self i + m_other partner with the row of the matrix
// chosen by bit t; a CX takes the partner where its control bit is 1.  A CX
// whose control c >= 6 visits only the half of the state with bit c set (item
// p -> index with a 1 inserted at bit c; lanes stay consecutive).
template <typename C, typename R, int U>
__global__ void __launch_bounds__(256) k_lane_gate(C *__restrict__ psi, const LaneGateArgs g, int xcd_shift) {
    uint64_t blk = blockIdx.x;
    if (xcd_shift > 0) blk = ((blk & 7) << xcd_shift) | (blk >> 3);  // gridDim.x = 8 << xcd_shift
    const uint64_t base = blk * blockDim.x * U + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int mt = 1 << g.t;
    const bool bit = (lane >> g.t) & 1;
    const R sr = (R)(bit ? g.m[6] : g.m[0]), si = (R)(bit ? g.m[7] : g.m[1]);
    const R pr = (R)(bit ? g.m[4] : g.m[2]), pi = (R)(bit ? g.m[5] : g.m[3]);
    const bool half = g.c >= 6;
    uint64_t idx[U];
    C v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t q = base + (uint64_t)u * blockDim.x;
        idx[u] = half ? (((q >> g.c) << (g.c + 1)) | (1ull << g.c) | (q & ((1ull << g.c) - 1))) : q;
        v[u] = dev::ld_nt(psi + idx[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        C p;
        p.x = __shfl_xor(v[u].x, mt, 64);
        p.y = __shfl_xor(v[u].y, mt, 64);
        if (g.c >= 0) {
            if (half || ((idx[u] >> g.c) & 1)) v[u] = p;
        } else {
            C o;
            o.x = sr * v[u].x - si * v[u].y + pr * p.x - pi * p.y;
            o.y = sr * v[u].y + si * v[u].x + pr * p.y + pi * p.x;
            v[u] = o;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) dev::st_nt(psi + idx[u], v[u]);
}

}  // namespace

hipError_t launch_lane_gate(bool c64, void *psi, int n, const LaneGateArgs &g, bool xcd, hipStream_t st) {
    if (g.t < 0 || g.t >= 6 || g.t >= n || g.c >= n || g.c == g.t || n < 12) return hipErrorInvalidValue;
    constexpr int U = 4;
    const uint64_t items = g.c >= 6 ? (1ull << (n - 1)) : (1ull << n);  // a high control halves the work
    const uint64_t grid = items / (256ull * U);
    if (grid == 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
    int xcd_shift = 0;
    if (xcd && grid >= 16) xcd_shift = 63 - __builtin_clzll(grid) - 3;
    if (c64)
        hipLaunchKernelGGL((k_lane_gate<float2, float, U>), dim3((uint32_t)grid), dim3(256), 0, st,
                           static_cast<float2 *>(psi), g, xcd_shift);
    else
        hipLaunchKernelGGL((k_lane_gate<double2, double, U>), dim3((uint32_t)grid), dim3(256), 0, st,
                           static_cast<double2 *>(psi), g, xcd_shift);
    return hipGetLastError();
}

hipError_t launch_swap_lane(bool c64, void *psi, int n, int a, int b, bool xcd, hipStream_t st) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    if (a == b || lo < 0 || hi >= n || lo >= 6 || n < 12) return hipErrorInvalidValue;
    constexpr int U = 4;
    // items: amplitudes (hi < 6) or pairs (hi >= 6); 256 * U per block, a power of two
    const uint64_t items = hi < 6 ? (1ull << n) : (1ull << (n - 1));
    const uint64_t grid = items / (256ull * U);
    if (grid == 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
    int xcd_shift = 0;
    if (xcd && grid >= 16) xcd_shift = 63 - __builtin_clzll(grid) - 3;
    if (c64)
        hipLaunchKernelGGL((k_swap_lane<float2, U>), dim3((uint32_t)grid), dim3(256), 0, st,
                           static_cast<float2 *>(psi), lo, hi, items, xcd_shift);
    else
        hipLaunchKernelGGL((k_swap_lane<double2, U>), dim3((uint32_t)grid), dim3(256), 0, st,
                           static_cast<double2 *>(psi), lo, hi, items, xcd_shift);
    return hipGetLastError();
}

hipError_t launch_swap2(bool c64, void *psi, int n, int a, int b, bool xcd, hipStream_t st) {
    if (a == b || a < 0 || b < 0 || a >= n || b >= n || n < 2) return hipErrorInvalidValue;
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const uint64_t n_pairs = 1ull << (n - 2);
    constexpr int U = 4;
    const uint64_t per_block = 256ull * U;
    const uint64_t grid = (n_pairs + per_block - 1) / per_block;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    // XCD order needs a power-of-two grid of at least 16 blocks
    int xcd_shift = 0;
    if (xcd && grid >= 16 && (grid & (grid - 1)) == 0) xcd_shift = 63 - __builtin_clzll(grid) - 3;
    if (c64)
        hipLaunchKernelGGL((k_swap2<float2, U>), dim3((uint32_t)grid), dim3(256), 0, st, static_cast<float2 *>(psi), lo,
                           hi, 1ull << a, 1ull << b, n_pairs, xcd_shift);
    else
        hipLaunchKernelGGL((k_swap2<double2, U>), dim3((uint32_t)grid), dim3(256), 0, st, static_cast<double2 *>(psi),
                           lo, hi, 1ull << a, 1ull << b, n_pairs, xcd_shift);
    return hipGetLastError();
}

}  // namespace qg
