// qg_kernels.h -- host launchers of the gfx950 kernels (HIP runtime types only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/qg.h"
#include "qg_internal.h"

namespace qg {

// One pass of the tile kernel.  `dev` holds PassDesc[], PhaseDesc[] and DevOp[]
// at the given byte offsets; `host_pass` is the same pass on the host (launch
// shape).  ns = 1 (psi only) or 2 (psi and lam, adjoint sweep with gradient
// partials gpart[row * gstride + tile * waves + wave]).
// When `inl` is not NULL the pass travels by value as the kernel argument and
// `dev` is not read.
hipError_t launch_tile(bool c64, const PassDesc &host_pass, const InlineProg *inl, const void *dev,
                       const ProgOffsets &offs, int pass_idx, int ns, void *psi, void *lam, double *gpart,
                       int64_t gstride, hipStream_t st);

// psi <- |0...0>
hipError_t launch_zero_state(bool c64, void *psi, uint64_t dim, hipStream_t st);

// out[i] = |psi_i|^2 (idx == NULL) or out[k] = |psi_{idx[k]}|^2.
hipError_t launch_probs(bool c64, const void *psi, uint64_t dim, const uint64_t *idx, int64_t n,
                        double *out, hipStream_t st);

// Allocation-free expectations: masks and coefficients (host arrays) go to the
// device by value and every partial sum lives in a static device array of the
// library (kNoAllocMaxTerms terms at most).  noalloc_scratch_init looks up that
// array's address on the current device.
constexpr int kNoAllocMaxTerms = 256;
hipError_t noalloc_scratch_init();
hipError_t launch_expval_noalloc(bool c64, const void *psi, uint64_t dim, const uint64_t *masks, const double *coeff,
                                 int n_terms, double *out_terms, double *out_sum, hipStream_t st);

// Z-string expectations.  part: scratch of expval_partials(dim, n_terms) doubles.
int64_t expval_partials(uint64_t dim, int n_terms);
hipError_t launch_expval(bool c64, const void *psi, uint64_t dim, const uint64_t *masks,
                         const double *coeff, int n_terms, double *part, double *out_terms,
                         double *out_sum, hipStream_t st);

// Shot sampling over a 64-ary tree of probability sums.  tree: scratch of
// sample_tree_doubles(dim) doubles.
int64_t sample_tree_doubles(uint64_t dim);
hipError_t launch_sample(bool c64, const void *psi, uint64_t dim, int64_t shots, uint64_t seed,
                         double *tree, uint64_t *out, hipStream_t st);

// Adjoint helpers.
// lam_i = (sum_m coeff_m (-1)^{popcount(i & mask_m)}) psi_i
hipError_t launch_apply_observable(bool c64, const void *psi, void *lam, uint64_t dim,
                                   const uint64_t *masks, const double *coeff, int n_terms,
                                   hipStream_t st);
// rows[r] = sum_{k < count} gpart[r * gstride + k] for r in [0, n_rows)
hipError_t launch_grad_rows(const double *gpart, int64_t gstride, int64_t count, int n_rows,
                            double *rows, hipStream_t st);
// grad[s] = sum of rows[r] over r with row_slot[r] == s (in row order)
hipError_t launch_grad_slots(const double *rows, const int32_t *row_slot, int n_rows, double *grad,
                             int n_params, hipStream_t st);

// Dense block on the matrix cores; ut_re/ut_im: transposed 2^k x 2^k matrix (R precision).
hipError_t launch_dense(bool c64, const DenseDesc &D, const void *ut_re, const void *ut_im, void *psi,
                        hipStream_t st);

// SWAP of qubits a and b as a permutation of the amplitudes whose bits differ.
// xcd: deal contiguous eighths of the pair range to the 8 XCDs (blocks go to XCDs in turn).
hipError_t launch_swap2(bool c64, void *psi, int n, int a, int b, bool xcd, hipStream_t st);
// SWAP whose lower qubit is a lane bit (< 6); n >= 12.
hipError_t launch_swap_lane(bool c64, void *psi, int n, int a, int b, bool xcd, hipStream_t st);
// One-qubit gate m = {m00, m01, m10, m11} (re, im pairs) on target t < 6, or a
// CX with control c >= 0 (m unused); n >= 12.
struct LaneGateArgs {
    double m[8];
    int t, c;
};
hipError_t launch_lane_gate(bool c64, void *psi, int n, const LaneGateArgs &g, bool xcd, hipStream_t st);

// Batched form.  Circuits whose state is one tile run in one persistent
// launch, a workgroup per circuit.  Larger circuits run pass by pass: one launch
// applies the next pass of every such circuit of a group, a workgroup per
// (circuit, tile), over the group's states in device memory.
//
// A workgroup of a multi-tile launch finds its item through the launch's
// block map: item = items[map[blockIdx.x]], and its tile or chunk within the
// item is blockIdx.x - item.begin.
struct BatchItem {
    uint64_t begin;      // first workgroup of this (circuit, pass) in its launch
    uint64_t state_off;  // the circuit's state in the state buffer (amplitudes)
    int32_t pass;        // index into the batch's pass list
    int32_t zero_init;   // 1: the state is |0...0> before this pass: the item is its
                         // tile 0 alone, which starts from |0...0> in registers
};
// kBatchChunk amplitudes of a circuit's state: the unit of the fill and
// observable kernels.
constexpr int kBatchChunk = 4096;
struct BatchChunkItem {
    uint64_t begin;      // first workgroup of this circuit in its launch
    uint64_t state_off;
    int32_t circ;        // index into the batch's circuit list
    int32_t n;           // qubits (2^n / kBatchChunk chunks)
};
// Final sum of one multi-tile circuit's observable partials.
struct BatchObsSum {
    uint64_t partial_begin;
    int32_t count;
    int32_t circ;
};
enum BatchStepKind : int32_t { BATCH_FILL = 0, BATCH_PASS = 1, BATCH_OBS = 2 };
struct BatchStep {
    int32_t kind;
    uint32_t lds;          // dynamic LDS bytes (pass steps)
    uint64_t blocks;       // workgroups
    uint64_t map_off;      // first entry of this launch in the block map
    uint64_t partial_off;  // observable steps: first partial written
};
struct BatchLaunch {
    // one-tile circuits (all pointers are device pointers)
    const BatchCirc *circs;
    const int32_t *order;       // the one-tile circuits, longest first
    int n_circ;                 // entries of order
    const PassDesc *passes;
    const PhaseDesc *phases;
    const DevOp *ops;
    const uint64_t *masks;
    const double *coeff;
    int obs_kind;
    int *counter;               // work counter (reset by the launch)
    double *out;
    int grid;
    int tile_bits;
    // multi-tile circuits
    const BatchItem *items;
    const BatchChunkItem *chunks;
    const int32_t *map;
    const BatchObsSum *sums;
    int n_sums;
    double *partial;
    void *states;
    std::vector<BatchStep> steps;  // host: launches in stream order
};
hipError_t launch_batch(bool c64, int rb, const BatchLaunch &L, hipStream_t st);

// Cost-model MLP (FP32, hidden width kMlpHidden).  z1..z3, dz1..dz3: [B][H] scratch.
constexpr int kMlpHidden = 64;
int mlp_param_count(int n_in);
hipError_t launch_mlp_forward(const float *theta, const float *X, int B, int F, float *z1, float *z2, float *z3,
                              float *y, hipStream_t st);
// Forward, loss (mean squared error; added to loss_acc[loss_slot] when not NULL),
// backward: grad[P] for the batch.
hipError_t launch_mlp_grad(const float *theta, const float *X, const float *T, int B, int F, float *z1, float *z2,
                           float *z3, float *y, float *dy, float *dz1, float *dz2, float *dz3, float *grad,
                           double *loss_acc, int loss_slot, hipStream_t st);
hipError_t launch_mlp_adam(float *theta, const float *g, float *m, float *v, int n, float lr, int step,
                           hipStream_t st);
hipError_t launch_mlp_gather(const float *X, const float *T, const int32_t *idx, int B, int F, float *Xb, float *Tb,
                             hipStream_t st);

}  // namespace qg
