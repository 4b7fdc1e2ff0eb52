// qg_plan.h -- host-side circuit validation, fusion planning and device-program building.
#pragma once
#include <complex>
#include <string>
#include <vector>

#include "../../include/qg.h"
#include "qg_internal.h"

namespace qg {

using cd = std::complex<double>;

struct Gate {
    int op, q0, q1;
    double p[3];
    int pidx;
};

// Tiling and fusion knobs of one plan.
struct PlanConfig {
    int n = 0;
    bool c64 = false;
    int tile_bits = 12;   // qubits per tile (capped at n)
    int reg_bits = 4;     // tile positions held in registers (amplitudes per thread = 2^reg_bits)
    int low_bits = 7;     // lowest qubits always in a fused tile (coalesced runs)
    int max_high = 5;     // fused pass: distinct required qubits >= low_bits
    int fusion = QG_FUSE_GREEDY;
    bool reverse = false; // adjoint sweep: reversed gates, daggered, with gradient ops
    int flags = 0;        // PASS_* bits for every pass
    int nt_mode = 1;      // 0 off, 1 only for line-aligned layouts, 2 always
    int swz_bits = 0;     // tile-order swizzle of the block index
    int max_gates_per_pass = 4096;
    int dense_min_gates = 0;  // a run on <= 6 qubits with this many gates runs as a dense block;
                              // 0: the measured break-even of Tuning::dense_auto; 1 << 30: never
    bool use_classes = true;        // single-gate passes take their tile shape from the class table
    int diag_run_min = 3;           // consecutive diagonal ops fused into one (0: never)
    bool half_lds = false;          // multi-phase passes exchange real and imaginary parts in turn
};

// Pass classes for tuning: by the highest qubit a pass needs in registers.
// 0: below the cache-line bits, 1: below 12, 2: below 20, 3: 20 and above,
// 4: no such qubit (diagonal-only pass).
constexpr int kPassClasses = 5;
int pass_class(uint64_t required, bool c64);

// Process-wide tuning of the planner (defaults measured on MI355X; set by
// qg_set_tuning or the autotuner).
struct Tuning {
    // Fused passes: [c128, c64].  Measured on config-3, QFT and ansatz circuits:
    // complex64 runs faster with 2^12-amplitude tiles and 16 registers per
    // thread than with 2^13 and 32 (two workgroups per CU either way, shorter
    // exchanges, lower register pressure).
    int tile_bits[2] = {12, 12};
    int reg_bits[2] = {4, 4};
    int low_bits[2] = {7, 7};
    int max_high[2] = {5, 5};
    int nt = 1;
    int swz_bits = 4;
    int xcd = 1;
    int diag_run_min = 3;  // fuse runs of at least this many diagonal ops (0: never)
    int lane_swap = 1;     // standalone SWAP with a qubit inside a cache line: cross-lane kernel
    int lane_gate = 1;     // single gate with its target inside a cache line: cross-lane kernel
    // Multi-phase passes exchange real and imaginary parts in turn through half
    // the LDS: [c128, c64].
    int half_lds[2] = {1, 0};
    int pipe = 0;          // persistent prefetching blocks: 0 never, 1 heavy passes, 2 always
    int pipe_min_ops = 4;  // a pass is heavy with several phases or at least this many ops
    int dense_min_gates = 0;
    // Gates from which a run on k = 4, 5, 6 qubits runs faster as one dense block
    // than as a tile pass, [c128, c64][k - 4] (measured on MI355X at 30 qubits
    // complex128 and 31 complex64, random gates of all ten kinds).
    int dense_auto[2][3] = {{24, 20, 28}, {16, 16, 24}};
    int batch_group_mib = 32768;  // batched form: device states of multi-tile circuits per group (MiB)
    int adjoint_tile_bits = 10;  // reverse sweeps in complex128: tile qubits (two states in registers)
    int adjoint_low_bits = 5;    // and the low block of their passes
    int dense_tile_bits = 11;  // a dense block's tile: its k qubits and the (this - k) lowest other qubits
    // Per pass class (see pass_class): tile bits, register bits and swizzle of
    // single-gate passes, and the swizzle of fused passes.  [dtype][class]
    int cls_tile[2][kPassClasses] = {{12, 12, 12, 10, 12}, {13, 13, 13, 11, 13}};
    int cls_reg[2][kPassClasses] = {{4, 4, 4, 2, 4}, {5, 5, 5, 3, 5}};
    int cls_swz[2][kPassClasses] = {{4, 4, 4, 0, 4}, {4, 4, 4, 0, 4}};
    // Per target qubit, for single-gate passes of a one-qubit mixing gate:
    // {tile bits, register bits, swizzle, xcd order}; tile 0 = use the class.
    int tgt[2][64][4] = {};
};
Tuning &tuning();
// Returns 0 on success, -1 for an unknown key or out-of-range value.
int set_tuning(const char *key, int64_t value);
int get_tuning(const char *key, int64_t *value);

PlanConfig default_config(int n, bool c64, int fusion);
// Re-establishes the invariants between knobs after a field was changed.
void clamp_config(PlanConfig *c);

// One fused pass as a gate range [g_begin, g_end) in execution order.
struct PassRange {
    int g_begin, g_end;
};

struct Program {
    std::vector<PassDesc> passes;
    std::vector<PhaseDesc> phases;
    std::vector<DevOp> ops;
    std::vector<int> pass_of_gate;   // index into execution order
    std::vector<int> grad_row_slot;  // adjoint: parameter slot of each gradient row
    int64_t max_grad_part = 0;       // adjoint: largest per-pass partial-sum block (doubles)
    std::vector<DenseDesc> dense;    // dense steps (passes flagged PASS_DENSE)
    std::vector<double> dense_ut;    // their transposed matrices: re block then im block, 4^k each
    std::vector<DiagRun> runs;       // fused diagonal runs (OP_DIAGRUN ops)
    std::vector<DiagEntry> entries;  // their per-thread factors
};

// Validates a circuit (qubits in range, q0 != q1, known code, finite params,
// trainable slots only on RX/RY/RZ/CP and below n_params when n_params >= 0).
// Returns QG_OK or QG_EINVAL with *err set.
qg_status validate_circuit(const qg_circuit *c, int n_params, std::string *err);

std::vector<Gate> load_gates(const qg_circuit *c);

// Execution-order gate list (reversed for adjoint sweeps).
std::vector<Gate> execution_order(const std::vector<Gate> &g, bool reverse);

// Fusion: partition execution-order gates into passes, in order.
std::vector<PassRange> fuse(const std::vector<Gate> &g, const PlanConfig &cfg);

// Commutation-aware greedy fusion: gates touching disjoint qubits commute, so a
// pass takes, in one scan, every not-yet-scheduled gate that fits its width and
// is not preceded by a skipped gate sharing one of its qubits.  `order` lists
// gate indices in execution order; ranges index into `order`.
struct Schedule {
    std::vector<int> order;
    std::vector<PassRange> ranges;
};
Schedule schedule(const std::vector<Gate> &g, const PlanConfig &cfg);
std::vector<Gate> permute(const std::vector<Gate> &g, const std::vector<int> &order);

// Device program for the given pass partition.
Program build_program(const std::vector<Gate> &g, const std::vector<PassRange> &passes,
                      const PlanConfig &cfg);

// All qubits a gate touches (targets, controls, diagonal qubits).
uint64_t touched_qubits(const Gate &g);
// Dense step of gates [begin, end) on block qubits `blk` (4..6 qubits, covering
// every touched qubit); appended to prog as a PASS_DENSE pass.
void append_dense(Program *prog, const std::vector<Gate> &g, int begin, int end, uint64_t blk, const PlanConfig &cfg);
// Block qubits of gates [r.g_begin, r.g_end) when the planner runs them as one
// dense block (at most 6 qubits, at least the break-even gate count), else 0.
uint64_t range_dense_block(const std::vector<Gate> &g, const PassRange &r, const PlanConfig &cfg);
// One pass of gates [r.g_begin, r.g_end) in the kernel the planner picks for it:
// the cross-lane gate or standalone SWAP kernels for those single gates, a dense
// block at or above the break-even gate count, else a tile pass.
void append_range(Program *prog, const std::vector<Gate> &g, const PassRange &r, const PlanConfig &cfg);
// Block qubits for a dense step of gates [begin, end), or 0 if they touch more than 6 qubits.
uint64_t dense_block_qubits(const std::vector<Gate> &g, int begin, int end, int n);
// Gates a run on `k` block qubits (4..6, after padding) needs to run as a dense block.
int dense_threshold(const PlanConfig &cfg, int k);

// Greedy plan (commutation-aware schedule) with the dense rule applied (cfg.dense_min_gates).
// *order (may be NULL) receives the execution order of the gates.
Program build_plan(const std::vector<Gate> &g, const PlanConfig &cfg, std::vector<int> *order = nullptr);

// Appends a program's passes, phases and ops (offsetting their indices); pass_of_gate is not merged.
void append_program(Program *dst, const Program &src);

// ---- learned fusion: features of one candidate pass
constexpr int kPlanFeatures = 24;
// Candidate strategies: k = 0..3 are tile passes with max_high = 4 + k (index 1 is
// the greedy default, width 5); k = kPlanDense is a dense block on the matrix cores.
constexpr int kPlanConfigs = 5;
constexpr int kPlanDense = 4;
PlanConfig candidate_config(int n, bool c64, int k);
// End of the pass the greedy rule would form starting at gate `begin`.
int first_block_end(const std::vector<Gate> &g, int begin, const PlanConfig &cfg);
// Features of gates [begin, end) executed as one pass under cfg (scaled, see the .cpp).
void pass_features(const std::vector<Gate> &g, int begin, int end, const PlanConfig &cfg, float *f);
// Features of gates [begin, end) executed as one dense block on qubits blk.
void dense_features(const std::vector<Gate> &g, int begin, int end, uint64_t blk, const PlanConfig &cfg, float *f);
// End of the longest run from `begin` whose gates touch at most 6 qubits (and at most max_gates).
int dense_block_end(const std::vector<Gate> &g, int begin, int max_gates);

// 2x2 matrix of a single-qubit gate (textbook forms, header of qg.h).
void gate_matrix(int op, const double *p, cd m[2][2]);

// Required tile qubits of a gate (targets of non-diagonal ops) as a bit mask.
uint64_t required_qubits(const Gate &g);

}  // namespace qg
