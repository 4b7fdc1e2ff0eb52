/*
 * qg_oracle.c -- FP64 CPU oracle for the state-vector simulation of Q-GEAR
 * (arXiv 2504.03967, Appendix A "Quantum state vector simulation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * calls it.  It shares no code, header or table with the GPU library.
 *
 * Everything here is the plain definition, written out gate by gate, with no
 * fusion, tiling or reordering:
 *   - the state is the 2^n complex vector of eq. (hilbert), initialised to
 *     |0...0>;
 *   - a single-qubit gate U on qubit t acts as I x ... x U x ... x I
 *     (eq. (tp)); written out, it mixes every pair of amplitudes whose indices
 *     differ only in bit t;
 *   - CX flips the target bit on every basis state whose control bit is 1
 *     (eq. (cx) and the 3-qubit worked example that follows it);
 *   - CP(lambda) is the CR1 matrix of eq. (cr1): a phase e^{i lambda} on the
 *     basis states where both qubits are 1; CZ is CP(pi);
 *   - SWAP exchanges two qubits.
 * Qubit q is bit q of the amplitude index (little-endian).
 * Gate matrices not printed in the paper are the textbook ones:
 *   H = [[1,1],[1,-1]]/sqrt2, X = [[0,1],[1,0]],
 *   RX(a) = [[c,-is],[-is,c]], RY(a) = [[c,-s],[s,c]],
 *   RZ(a) = diag(e^{-ia/2}, e^{+ia/2}),
 *   U3(a,b,l) = [[c, -e^{il}s],[e^{ib}s, e^{i(b+l)}c]],
 * with c = cos(a/2), s = sin(a/2).
 *
 * Probabilities are |alpha_i|^2 (eq. (hilbert)).  Shots are drawn by the
 * inverse CDF of those probabilities with the Philox4x32-10 counter-based
 * generator (Salmon, Moraes, Dror, Shaw, SC'11), keyed by the seed and counted
 * by the shot index.  Pauli-Z-string expectations are sums of p_i times the
 * parity sign of the masked index bits.  Gradients of a Z-string observable
 * follow the adjoint recursion (Jones & Gacon 2020; the paper names "adjoint
 * GPU modes" in its methods overview without describing them).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so qg_oracle.c -lm
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Gate codes of the circuit encoding (one row per gate: {code, q0, q1}). */
enum { G_H = 0, G_X, G_RX, G_RY, G_RZ, G_U3, G_CX, G_CZ, G_CP, G_SWAP, G_COUNT };

/* ---------------------------------------------------------------- gates */

/* 2x2 matrix of a single-qubit gate; m[r][c] acts on (alpha_{bit=0}, alpha_{bit=1}). */
static int one_qubit_matrix(int op, const double *p, cplx m[2][2])
{
    double c = cos(p[0] / 2), s = sin(p[0] / 2);
    switch (op) {
    case G_H:
        m[0][0] = 1 / sqrt(2.0); m[0][1] = 1 / sqrt(2.0);
        m[1][0] = 1 / sqrt(2.0); m[1][1] = -1 / sqrt(2.0);
        return 0;
    case G_X:
        m[0][0] = 0; m[0][1] = 1; m[1][0] = 1; m[1][1] = 0;
        return 0;
    case G_RX:
        m[0][0] = c; m[0][1] = -I * s; m[1][0] = -I * s; m[1][1] = c;
        return 0;
    case G_RY:
        m[0][0] = c; m[0][1] = -s; m[1][0] = s; m[1][1] = c;
        return 0;
    case G_RZ:
        m[0][0] = cexp(-I * p[0] / 2); m[0][1] = 0;
        m[1][0] = 0; m[1][1] = cexp(I * p[0] / 2);
        return 0;
    case G_U3:
        m[0][0] = c;
        m[0][1] = -cexp(I * p[2]) * s;
        m[1][0] = cexp(I * p[1]) * s;
        m[1][1] = cexp(I * (p[1] + p[2])) * c;
        return 0;
    }
    return -1;
}

static void apply_matrix(int n, cplx *psi, int t, cplx m[2][2])
{
    uint64_t dim = 1ull << n, bit = 1ull << t;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)dim; i++) {
        if (i & bit) continue;
        cplx a0 = psi[i], a1 = psi[i | bit];
        psi[i] = m[0][0] * a0 + m[0][1] * a1;
        psi[i | bit] = m[1][0] * a0 + m[1][1] * a1;
    }
}

static void apply_cx(int n, cplx *psi, int c, int t)
{
    uint64_t dim = 1ull << n, cb = 1ull << c, tb = 1ull << t;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)dim; i++) {
        if ((i & cb) && !(i & tb)) {
            cplx tmp = psi[i];
            psi[i] = psi[i | tb];
            psi[i | tb] = tmp;
        }
    }
}

/* Multiply every amplitude whose bits a and b are both 1 by phase. */
static void apply_both_ones_phase(int n, cplx *psi, int a, int b, cplx phase)
{
    uint64_t dim = 1ull << n, ab = 1ull << a, bb = 1ull << b;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)dim; i++)
        if ((i & ab) && (i & bb)) psi[i] *= phase;
}

static void apply_swap(int n, cplx *psi, int a, int b)
{
    uint64_t dim = 1ull << n, ab = 1ull << a, bb = 1ull << b;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)dim; i++) {
        if ((i & ab) && !(i & bb)) {
            uint64_t j = (i ^ ab) | bb;
            cplx tmp = psi[i];
            psi[i] = psi[j];
            psi[j] = tmp;
        }
    }
}

static int check_gate(int n, const int32_t *g)
{
    int op = g[0], q0 = g[1], q1 = g[2];
    if (op < 0 || op >= G_COUNT) return -1;
    if (q1 < 0 || q1 >= n) return -1;
    if (op >= G_CX) {
        if (q0 < 0 || q0 >= n || q0 == q1) return -1;
    }
    return 0;
}

/* Apply one gate row {op, q0, q1} with parameters p[3]; dagger != 0 applies U^dagger. */
static int apply_gate(int n, cplx *psi, const int32_t *g, const double *p, int dagger)
{
    int op = g[0], q0 = g[1], q1 = g[2];
    if (check_gate(n, g)) return -1;
    if (op <= G_U3) {
        cplx m[2][2];
        one_qubit_matrix(op, p, m);
        if (dagger) {
            cplx d[2][2] = {{conj(m[0][0]), conj(m[1][0])}, {conj(m[0][1]), conj(m[1][1])}};
            apply_matrix(n, psi, q1, d);
        } else {
            apply_matrix(n, psi, q1, m);
        }
        return 0;
    }
    switch (op) {
    case G_CX: apply_cx(n, psi, q0, q1); return 0;
    case G_CZ: apply_both_ones_phase(n, psi, q0, q1, -1.0); return 0;
    case G_CP: apply_both_ones_phase(n, psi, q0, q1, cexp((dagger ? -I : I) * p[0])); return 0;
    case G_SWAP: apply_swap(n, psi, q0, q1); return 0;
    }
    return -1;
}

/* ------------------------------------------------------------- public API */

/* psi <- |0...0>. */
void qgo_init(int n, cplx *psi)
{
    memset(psi, 0, sizeof(cplx) << n);
    psi[0] = 1;
}

/* Apply gates [0, n_gates) in order.  gate_type is [n_gates][3] = {op, q0, q1}
 * (q0 = control or first qubit, -1 for single-qubit gates; q1 = target or
 * second qubit); gate_param is [n_gates][3] = {theta, phi, lambda}.
 * Returns 0, or -1 - g for the first malformed gate g. */
int qgo_apply_circuit(int n, cplx *psi, int64_t n_gates, const int32_t *gate_type,
                      const double *gate_param)
{
    for (int64_t g = 0; g < n_gates; g++)
        if (apply_gate(n, psi, gate_type + 3 * g, gate_param + 3 * g, 0)) return (int)(-1 - g);
    return 0;
}

/* Apply the adjoint of gates [0, n_gates) in reverse order (U^dagger of the circuit). */
int qgo_apply_circuit_dagger(int n, cplx *psi, int64_t n_gates, const int32_t *gate_type,
                             const double *gate_param)
{
    for (int64_t g = n_gates - 1; g >= 0; g--)
        if (apply_gate(n, psi, gate_type + 3 * g, gate_param + 3 * g, 1)) return (int)(-1 - g);
    return 0;
}

/* p_i = |alpha_i|^2 for all i. */
void qgo_probs(int n, const cplx *psi, double *p)
{
    uint64_t dim = 1ull << n;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)dim; i++) p[i] = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
}

/* <Z_m> = sum_i p_i (-1)^{popcount(i & mask_m)} for each of n_terms masks. */
void qgo_expval(int n, const cplx *psi, int n_terms, const uint64_t *mask, double *out)
{
    uint64_t dim = 1ull << n;
    for (int m = 0; m < n_terms; m++) {
        double acc = 0;
        int64_t i;
#pragma omp parallel for schedule(static) reduction(+ : acc)
        for (i = 0; i < (int64_t)dim; i++) {
            double p = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
            acc += (__builtin_popcountll((uint64_t)i & mask[m]) & 1) ? -p : p;
        }
        out[m] = acc;
    }
}

/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 Philox S-box,
 * multipliers 0xD2511F53 and 0xCD9E8D57, key schedule bumped by the Weyl
 * constants 0x9E3779B9 and 0xBB67AE85 between rounds. */
void qgo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    memcpy(out, c, sizeof c);
}

/* The uniform double in [0,1) for shot s under seed: Philox4x32-10 with
 * key = (seed low 32, seed high 32), counter = (s low 32, s high 32, 0, 0);
 * x = out[1]:out[0] as a 64-bit word; u = (x >> 11) * 2^-53. */
double qgo_shot_uniform(uint64_t seed, uint64_t s)
{
    uint32_t ctr[4] = {(uint32_t)s, (uint32_t)(s >> 32), 0, 0};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    qgo_philox4x32_10(ctr, key, o);
    uint64_t x = ((uint64_t)o[1] << 32) | o[0];
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/* Inverse-CDF sampling.  C_i = p_0 + ... + p_i summed sequentially in index
 * order; T = C_{dim-1}.  Shot s returns the smallest i with C_i > u_s * T; if
 * rounding leaves no such i, the largest i with p_i > 0. */
int qgo_sample(int n, const cplx *psi, int64_t shots, uint64_t seed, uint64_t *out)
{
    uint64_t dim = 1ull << n;
    double *cdf = malloc(sizeof(double) * dim);
    if (!cdf) return -1;
    double acc = 0;
    uint64_t last_nz = 0;
    for (uint64_t i = 0; i < dim; i++) {
        double p = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        if (p > 0) last_nz = i;
        acc += p;
        cdf[i] = acc;
    }
    double total = acc;
    int64_t s;
#pragma omp parallel for schedule(static)
    for (s = 0; s < shots; s++) {
        double r = qgo_shot_uniform(seed, (uint64_t)s) * total;
        uint64_t lo = 0, hi = dim; /* first index with cdf > r lies in [lo, hi] */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > r) hi = mid;
            else lo = mid + 1;
        }
        out[s] = lo < dim ? lo : last_nz;
    }
    free(cdf);
    return 0;
}

/* Adjoint-method gradient of f = <psi|O|psi>, O = sum_m coeff_m Z_{mask_m}, for
 * the circuit applied to |0...0>.  Every gate with param_idx[g] >= 0 is
 * trainable in its first parameter: RX, RY, RZ (exp(-i a P / 2), P = X, Y, Z)
 * contribute Im<lambda|P|psi>, CP contributes -2 Im<lambda|P11|psi> (P11 the
 * projector on both qubits = 1), both taken with psi and lambda at the point
 * right after the gate, accumulated into grad[param_idx[g]].
 * Recursion: psi_G = U_G..U_1|0>, lambda_G = O psi_G, then for g = G..1 the
 * gradient term, psi <- U_g^dag psi, lambda <- U_g^dag lambda.
 * Returns 0, -1 on a malformed gate or an untrainable gate with an index,
 * -2 on allocation failure. */
int qgo_adjoint_grad(int n, int64_t n_gates, const int32_t *gate_type, const double *gate_param,
                     const int32_t *param_idx, int n_params, int n_terms, const uint64_t *mask,
                     const double *coeff, double *value, double *grad)
{
    uint64_t dim = 1ull << n;
    cplx *psi = malloc(sizeof(cplx) * dim), *lam = malloc(sizeof(cplx) * dim);
    if (!psi || !lam) { free(psi); free(lam); return -2; }
    for (int k = 0; k < n_params; k++) grad[k] = 0;
    qgo_init(n, psi);
    if (qgo_apply_circuit(n, psi, n_gates, gate_type, gate_param)) { free(psi); free(lam); return -1; }

    double f = 0;
    for (uint64_t i = 0; i < dim; i++) {
        double o = 0;
        for (int m = 0; m < n_terms; m++)
            o += (__builtin_popcountll(i & mask[m]) & 1) ? -coeff[m] : coeff[m];
        lam[i] = o * psi[i];
        f += creal(conj(psi[i]) * lam[i]);
    }
    *value = f;

    for (int64_t g = n_gates - 1; g >= 0; g--) {
        const int32_t *gt = gate_type + 3 * g;
        int k = param_idx ? param_idx[g] : -1;
        if (k >= n_params) { free(psi); free(lam); return -1; }
        if (k >= 0) {
            int op = gt[0], t = gt[2];
            uint64_t tb = 1ull << t;
            cplx acc = 0;
            if (op == G_RX || op == G_RY || op == G_RZ) {
                for (uint64_t i = 0; i < dim; i++) {
                    /* (P psi)_i for P = X, Y, Z on qubit t */
                    int bit = (i & tb) != 0;
                    cplx ppsi;
                    if (op == G_RX) ppsi = psi[i ^ tb];
                    else if (op == G_RY) ppsi = (bit ? I : -I) * psi[i ^ tb];
                    else ppsi = bit ? -psi[i] : psi[i];
                    acc += conj(lam[i]) * ppsi;
                }
                grad[k] += cimag(acc);
            } else if (op == G_CP) {
                uint64_t cb = 1ull << gt[1];
                for (uint64_t i = 0; i < dim; i++)
                    if ((i & cb) && (i & tb)) acc += conj(lam[i]) * psi[i];
                grad[k] += -2 * cimag(acc);
            } else {
                free(psi); free(lam);
                return -1;
            }
        }
        apply_gate(n, psi, gt, gate_param + 3 * g, 1);
        apply_gate(n, lam, gt, gate_param + 3 * g, 1);
    }
    free(psi);
    free(lam);
    return 0;
}

/* Independent circuits, as in the parallel ("batched") mode of Sec. 2.4: circuit c has
 * n[c] qubits and the gate rows [goff[c], goff[c + 1]) of gate_type / gate_param; each
 * starts from |0...0> and out[c] is the open-chain observable sum_{q < n-1} <Z_q Z_{q+1}>
 * of its final state.  One circuit per OpenMP thread at a time; the gate loops inside run
 * on that thread alone (the nested parallel regions are inactive).  Returns 0, -1 - c for
 * the first circuit c holding a malformed gate, or -(1 << 30) when a state cannot be
 * allocated. */
int qgo_batch_zz_chain(int n_circ, const int32_t *n, const int64_t *goff, const int32_t *gate_type,
                       const double *gate_param, double *out)
{
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_circ; c++) {
        int nq = n[c];
        cplx *psi = malloc(sizeof(cplx) << nq);
        if (!psi) {
#pragma omp critical
            err = -(1 << 30);
            continue;
        }
        qgo_init(nq, psi);
        if (qgo_apply_circuit(nq, psi, goff[c + 1] - goff[c], gate_type + 3 * goff[c],
                              gate_param + 3 * goff[c])) {
#pragma omp critical
            if (err == 0 || -1 - c > err) err = -1 - c;
        }
        double sum = 0;
        for (int q = 0; q + 1 < nq; q++) {
            uint64_t m = 3ull << q;
            double t;
            qgo_expval(nq, psi, 1, &m, &t);
            sum += t;
        }
        out[c] = sum;
        free(psi);
    }
    return err;
}

/* Number of OpenMP threads a parallel region of the oracle uses. */
int qgo_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
