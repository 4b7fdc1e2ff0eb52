// qg_perm.hip -- SWAP of two qubits as a pure permutation: only the amplitudes
// whose two bits differ move (half the state), each exchanged with its partner.
// Used for a standalone SWAP whose lower qubit is at or above the cache-line
// offset bits, so every wavefront access covers whole 128-byte lines.
#include "qg_kernels.h"

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
            va[u] = psi[ia[u]];
            vb[u] = psi[ib[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t p = base_p + (uint64_t)u * blockDim.x;
        if (p < n_pairs) {
            psi[ia[u]] = vb[u];
            psi[ib[u]] = va[u];
        }
    }
}

}  // namespace

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
