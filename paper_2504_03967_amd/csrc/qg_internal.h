// qg_internal.h -- device program format shared by the host planner and the kernels.
//
// A circuit is executed as a sequence of passes.  A pass streams every "tile"
// of the state through registers once: a tile is the set of 2^b amplitudes
// whose indices agree on all qubits outside the pass's b tile qubits.  Inside
// a tile each thread holds 2^rb amplitudes (rb "register" tile positions) and
// the 2^tb threads of the workgroup cover the other tile positions.  Ops that
// mix amplitudes (dense 2x2, controlled 2x2) need their target as a register
// position; phases re-map which tile positions are register positions by an
// exchange through LDS.  Diagonal ops and controls read index bits directly,
// so they need no particular position and may even act on qubits outside the
// tile (whose bits are constant over a tile).
#pragma once
#include <stdint.h>

namespace qg {

constexpr int kMaxTileBits = 14;
constexpr int kMaxRegBits = 5;
constexpr int kMaxThreadBits = 8;
constexpr int kMaxRuns = 20;

enum OpKind : int32_t {
    OP_MAT = 0,    // dense 2x2 on register slot a: m = {m00, m01, m10, m11} (re, im)
    OP_CX = 1,     // exchange the pair on register slot a where the bit of qubit-ref c is 1
    OP_DIAG1 = 2,  // amplitude *= (bit of ref a ? {m[2],m[3]} : {m[0],m[1]})
    OP_DIAG2 = 3,  // amplitude *= {m[0], m[1]} where bits of refs a and c are both 1
    OP_GRADX = 4,  // adjoint partial: Im<lam|X_a|psi>, a = register slot, into grad row g
    OP_GRADY = 5,  // adjoint partial: Im<lam|Y_a|psi>
    OP_GRADZ = 6,  // adjoint partial: Im<lam|Z_a|psi>, a = qubit-ref
    OP_GRADP11 = 7, // adjoint partial: -2 Im<lam|P11(a,c)|psi>, a, c = qubit-refs
    // Cheaper forms chosen by the planner (same semantics as the general kind):
    OP_MATR = 8,    // OP_MAT with a real matrix (H, RY, X)
    OP_MATRX = 9,   // OP_MAT with real diagonal and imaginary off-diagonal entries (RX)
    OP_DIAG1R = 10, // OP_DIAG1 whose qubit is register slot a
    OP_DIAG2R = 11, // OP_DIAG2 with one qubit on register slot a, the other qubit-ref c
    OP_DIAG2RR = 12,// OP_DIAG2 with both qubits on register slots a and c
    OP_DIAGRUN = 13,// a run of diagonal ops fused into one factor per amplitude: DiagRun a
    OP_CXRR = 14    // OP_CX whose control is register slot c: a fixed permutation of the registers
};

// Qubit reference: r >= 0 is a tile position; r < 0 is global qubit (-1 - r), outside the tile.
constexpr int qref_global(int q) { return -1 - q; }

// A run of consecutive diagonal ops of one phase (OP_DIAGRUN), as one factor
// per amplitude:  F = tf * prod_{register slot j set} r_j * prod_{slots j<k set} q_jk
// where tf starts at c0 and r_j at r[j] (the uniform parts, computed on the
// host), and each entry multiplies tf (entries [e_begin, s_begin[0])) or r_j
// (entries [s_begin[j], s_begin[j+1])) by f1 where its condition holds, else
// by f0.  The condition reads thread bits or qubits outside the tile only:
// every tile position in tmask (thread bits) and every qubit in gmask (outside
// the tile, the same for the whole tile) is 1.
constexpr int32_t kNoRef = 1 << 30;
struct DiagEntry {
    uint32_t tmask;   // tile positions held by thread bits
    uint32_t f0_one;  // 1: f0 is exactly 1, so a tile where gmask fails skips the entry
    uint64_t gmask;   // qubits outside the tile
    double f0[2], f1[2];
};
struct DiagRun {
    double c0[2];
    double r[kMaxRegBits][2];
    double q[kMaxRegBits * (kMaxRegBits - 1) / 2][2];  // pair (j, k), j < k: index k (k - 1) / 2 + j
    int32_t e_begin;
    int32_t s_begin[kMaxRegBits + 1];
};

// Byte offsets of a program's arrays in its device copy.
struct ProgOffsets {
    uint32_t pass, phase, op, run, entry;
};

struct DevOp {
    int32_t kind;
    int32_t a;
    int32_t c;
    int32_t g;      // gradient row for OP_GRAD*
    double m[8];
};

struct PhaseDesc {
    uint64_t thr_goff[kMaxThreadBits];  // global index offset of thread bit k
    uint64_t reg_goff[kMaxRegBits];     // global index offset of register bit j
    uint32_t thr_poff[kMaxThreadBits];  // tile position offset of thread bit k
    uint32_t reg_poff[kMaxRegBits];     // tile position offset of register bit j
    int32_t op_begin, op_end;
    int32_t pad;
};

struct PassDesc {
    int32_t b, rb, tb, n_runs;
    int32_t run_start[kMaxRuns];   // runs of consecutive free (non-tile, non-fixed) qubits
    int32_t run_len[kMaxRuns];
    uint64_t fixed_mask, fixed_val;  // only tiles with (index & fixed_mask) == fixed_val are active
    int32_t phase_begin, n_phase;
    int32_t grad_base;   // first gradient row written by this pass (adjoint sweeps)
    int32_t n_grad;      // gradient rows written by this pass
    uint64_t n_tiles;    // active tiles = launch size
    int32_t flags;       // PASS_* bits
    int32_t swz_bits;    // block index: XOR the low swz_bits bits with the next ones
};

enum PassFlags : int32_t {
    PASS_NT = 1,     // non-temporal loads and stores of the state (streaming, no reuse)
    PASS_DENSE = 2,  // the pass is a dense block: phase_begin indexes the program's DenseDesc list
    PASS_SWAP2 = 4,  // the pass is a standalone SWAP of qubits run_start[0] and run_start[1]
    PASS_XCD = 8,    // tile order: block b takes tile (b mod 8) * n_tiles / 8 + b / 8
    PASS_PIPE = 16,  // persistent blocks that load their next tile while computing the current one
    PASS_SWAPL = 64, // standalone SWAP of qubits run_start[0], run_start[1] with the lower one
                     // inside a cache line: coalesced loads and a cross-lane exchange
    PASS_LANE1 = 128,// single one-qubit gate (or CX) whose target run_start[0] lies inside a
                     // cache line: cross-lane exchange; run_start[1] = CX control or -1;
                     // phase_begin indexes the program's op holding the 2x2 matrix
    PASS_HALFX = 256,// layout exchanges move real and imaginary parts in turn through
                     // half the LDS (2^b scalars instead of 2^b complex values)
};

// A dense k-qubit block (k in 4..6): tiles are the block qubits blk_q plus the l
// lowest other qubits low_q; the rest are free runs enumerated by the block index.
struct DenseDesc {
    int32_t k, l, n_runs, pad;
    int8_t blk_q[8];
    int8_t low_q[16];
    int32_t run_start[kMaxRuns];
    int32_t run_len[kMaxRuns];
    uint64_t n_tiles;
    int64_t u_index;  // first element of this block's transposed matrix in the program's matrix list
};

// One circuit of a batched launch: its passes are passes[pass_begin, +n_pass);
// its observable terms (QG_OBS_CSR) are masks/coeff[obs_begin, +obs_count).
struct BatchCirc {
    int32_t n;
    int32_t pass_begin;
    int32_t n_pass;
    int32_t obs_begin;
    int32_t obs_count;
    int32_t pad;
};

// A small pass passed by value as the kernel argument (no upload on the stream).
constexpr int kInlinePhases = 2;
constexpr int kInlineOps = 12;
struct InlineProg {
    PassDesc pass;   // phase_begin = 0
    PhaseDesc phases[kInlinePhases];
    DevOp ops[kInlineOps];
};

}  // namespace qg
