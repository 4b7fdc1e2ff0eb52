// qg_plan.cpp -- validation, greedy fusion and tile/phase planning (host only).
//
// Every gate of the circuit becomes one or more ops of a pass (App. A gives the
// operators; the textbook matrices are listed in qg.h).  A pass is executed by
// the tile kernel: all tiles of the state are streamed once through registers,
// so a pass costs one read and one write of the (active part of the) state
// whatever the number of ops it holds.  That is the role the paper's backend
// gives to gate fusion (fusion width 5, App. D.2), carried out here without
// forming dense 2^k matrices.
#include "qg_plan.h"

#include <algorithm>
#include <queue>
#include <set>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace qg {

namespace {

inline int popcount64(uint64_t x) { return __builtin_popcountll(x); }

struct Item {
    int kind;
    int qa, qc;
    double m[8];
    int g;
};

bool is_one_qubit(int op) { return op >= QG_H && op <= QG_U3; }
bool is_two_qubit(int op) { return op >= QG_CX && op <= QG_SWAP; }

void put(double *m, int k, cd v) {
    m[2 * k] = v.real();
    m[2 * k + 1] = v.imag();
}

// Ops of one gate; `dagger` emits U^dagger.  In reverse sweeps a gradient op
// (taken at the state right after the gate) precedes the daggered gate.
void gate_items(const Gate &g, bool dagger, int grad_row, std::vector<Item> *out) {
    Item it{};
    it.g = -1;
    if (grad_row >= 0) {
        Item gi{};
        gi.g = grad_row;
        gi.qa = g.q1;
        gi.qc = g.q0;
        switch (g.op) {
        case QG_RX: gi.kind = OP_GRADX; break;
        case QG_RY: gi.kind = OP_GRADY; break;
        case QG_RZ: gi.kind = OP_GRADZ; break;
        case QG_CP: gi.kind = OP_GRADP11; break;
        }
        out->push_back(gi);
    }
    if (is_one_qubit(g.op) && g.op != QG_RZ) {
        cd m[2][2];
        gate_matrix(g.op, g.p, m);
        if (dagger) {
            cd d[2][2] = {{std::conj(m[0][0]), std::conj(m[1][0])}, {std::conj(m[0][1]), std::conj(m[1][1])}};
            std::memcpy(m, d, sizeof d);
        }
        it.kind = OP_MAT;
        it.qa = g.q1;
        put(it.m, 0, m[0][0]);
        put(it.m, 1, m[0][1]);
        put(it.m, 2, m[1][0]);
        put(it.m, 3, m[1][1]);
        out->push_back(it);
        return;
    }
    const double sgn = dagger ? -1.0 : 1.0;
    switch (g.op) {
    case QG_RZ:
        it.kind = OP_DIAG1;
        it.qa = g.q1;
        put(it.m, 0, std::polar(1.0, -0.5 * sgn * g.p[0]));
        put(it.m, 1, std::polar(1.0, 0.5 * sgn * g.p[0]));
        out->push_back(it);
        return;
    case QG_CX:
        it.kind = OP_CX;
        it.qc = g.q0;
        it.qa = g.q1;
        out->push_back(it);
        return;
    case QG_CZ:
    case QG_CP:
        it.kind = OP_DIAG2;
        it.qa = g.q0;
        it.qc = g.q1;
        put(it.m, 0, g.op == QG_CZ ? cd(-1.0, 0.0) : std::polar(1.0, sgn * g.p[0]));
        out->push_back(it);
        return;
    case QG_SWAP: {
        // SWAP(a, b) = CX(a->b) CX(b->a) CX(a->b)
        int a = g.q0, b = g.q1;
        int seq[3][2] = {{a, b}, {b, a}, {a, b}};
        for (auto &s : seq) {
            Item x{};
            x.kind = OP_CX;
            x.g = -1;
            x.qc = s[0];
            x.qa = s[1];
            out->push_back(x);
        }
        return;
    }
    }
}

int needs_register(const Item &it) {
    switch (it.kind) {
    case OP_MAT:
    case OP_CX:
    case OP_GRADX:
    case OP_GRADY:
        return it.qa;
    }
    return -1;
}

}  // namespace

Tuning &tuning() {
    static Tuning t;
    return t;
}

namespace {
struct Knob {
    const char *name;
    int *(*field)(Tuning &);
    int lo, hi;
};
const Knob kKnobs[] = {
    {"tile_bits_c128", [](Tuning &t) { return &t.tile_bits[0]; }, 2, 13},
    {"tile_bits_c64", [](Tuning &t) { return &t.tile_bits[1]; }, 2, 13},
    {"reg_bits_c128", [](Tuning &t) { return &t.reg_bits[0]; }, 1, 4},
    {"reg_bits_c64", [](Tuning &t) { return &t.reg_bits[1]; }, 1, 5},
    {"low_bits_c128", [](Tuning &t) { return &t.low_bits[0]; }, 0, 13},
    {"low_bits_c64", [](Tuning &t) { return &t.low_bits[1]; }, 0, 13},
    {"max_high_c128", [](Tuning &t) { return &t.max_high[0]; }, 1, 13},
    {"max_high_c64", [](Tuning &t) { return &t.max_high[1]; }, 1, 13},
    {"nt", [](Tuning &t) { return &t.nt; }, 0, 2},
    {"swz_bits", [](Tuning &t) { return &t.swz_bits; }, 0, 16},
    {"xcd", [](Tuning &t) { return &t.xcd; }, 0, 1},
    {"pipe", [](Tuning &t) { return &t.pipe; }, 0, 2},
    {"diag_run_min", [](Tuning &t) { return &t.diag_run_min; }, 0, 1 << 20},
    {"lane_swap", [](Tuning &t) { return &t.lane_swap; }, 0, 1},
    {"lane_gate", [](Tuning &t) { return &t.lane_gate; }, 0, 1},
    {"half_lds_c128", [](Tuning &t) { return &t.half_lds[0]; }, 0, 1},
    {"half_lds_c64", [](Tuning &t) { return &t.half_lds[1]; }, 0, 1},
    {"pipe_min_ops", [](Tuning &t) { return &t.pipe_min_ops; }, 1, 1 << 20},
    {"dense_min_gates", [](Tuning &t) { return &t.dense_min_gates; }, 0, 1 << 30},
    {"dense_tile_bits", [](Tuning &t) { return &t.dense_tile_bits; }, 10, 13},
    {"batch_group_mib", [](Tuning &t) { return &t.batch_group_mib; }, 1, 1 << 20},
    {"adjoint_tile_bits", [](Tuning &t) { return &t.adjoint_tile_bits; }, 8, 11},
    {"adjoint_low_bits", [](Tuning &t) { return &t.adjoint_low_bits; }, 3, 8},
};

// A phase of a pass: the tile positions held in registers (slot order) and
// the items it applies, in execution order.
struct PhasePlan {
    std::vector<int> S;
    std::vector<int> items;
};

// Fills S up to rb positions with the highest positions not yet in it.
void fill_slots(std::vector<int> *S, int b, int rb) {
    for (int p = b - 1; p >= 0 && (int)S->size() < rb; --p)
        if (std::find(S->begin(), S->end(), p) == S->end()) S->push_back(p);
}

// Items in their given order; a phase ends at the first item whose register
// qubit is not among the first rb distinct ones (adjoint sweeps keep this
// order: their gradient partials read the state at fixed points).
std::vector<PhasePlan> plan_phases_in_order(const std::vector<Item> &items, const int *pos_of, int b, int rb) {
    std::vector<PhasePlan> out;
    size_t i = 0;
    do {
        PhasePlan pp;
        for (size_t j = i; j < items.size() && (int)pp.S.size() < rb; ++j) {
            const int q = needs_register(items[j]);
            if (q < 0) continue;
            if (std::find(pp.S.begin(), pp.S.end(), pos_of[q]) == pp.S.end()) pp.S.push_back(pos_of[q]);
        }
        fill_slots(&pp.S, b, rb);
        for (; i < items.size(); ++i) {
            const int q = needs_register(items[i]);
            if (q >= 0 && std::find(pp.S.begin(), pp.S.end(), pos_of[q]) == pp.S.end()) break;
            pp.items.push_back((int)i);
        }
        out.push_back(pp);
    } while (i < items.size());
    return out;
}

// Qubits an item acts on, and whether it is diagonal on each (a CX is
// diagonal on its control).  Two items commute when every qubit they share is
// one on which both are diagonal.
int item_qubits(const Item &it, int *q, bool *diag) {
    switch (it.kind) {
    case OP_CX:
        q[0] = it.qa, diag[0] = false;
        q[1] = it.qc, diag[1] = true;
        return 2;
    case OP_DIAG1:
        q[0] = it.qa, diag[0] = true;
        return 1;
    case OP_DIAG2:
        q[0] = it.qa, diag[0] = true;
        q[1] = it.qc, diag[1] = true;
        return 2;
    default:
        q[0] = it.qa, diag[0] = false;
        return 1;
    }
}

bool items_commute(const Item &x, const Item &y) {
    int qx[2], qy[2];
    bool dx[2], dy[2];
    const int nx = item_qubits(x, qx, dx), ny = item_qubits(y, qy, dy);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            if (qx[i] == qy[j] && !(dx[i] && dy[j])) return false;
    return true;
}

// Fewer register layouts (each change is an LDS exchange of the whole tile):
// items may run in any order that keeps every non-commuting pair in its given
// order.  A phase runs every ready item it can (smallest index first); when
// none is left it takes the register qubit of the earliest ready item (for the
// first phase, one at or above the cache-line bits if any, so that the loads
// stay line-aligned), until rb qubits are held.
//
// The order constraints are kept as a graph whose transitive closure is the
// non-commuting pairs: per qubit, an item that is diagonal on it follows the
// last item that is not; an item that is not diagonal on it follows that item
// and every diagonal item since.  So planning a pass of thousands of gates
// (QCrank's) costs time linear in its items, not quadratic.
std::vector<PhasePlan> plan_phases(const std::vector<Item> &items, const int *pos_of, int b, int rb, int line_bits) {
    const int n = (int)items.size();
    std::vector<std::vector<int>> succ(n);
    std::vector<int> indeg(n, 0);
    {
        std::vector<int> last_nd(64, -1);
        std::vector<std::vector<int>> diag_since(64);
        for (int j = 0; j < n; ++j) {
            int qs[2];
            bool dg[2];
            const int nq = item_qubits(items[j], qs, dg);
            for (int k = 0; k < nq; ++k) {
                const int q = qs[k];
                auto edge = [&](int i) {
                    if (i >= 0 && i != j) {
                        succ[i].push_back(j);
                        ++indeg[j];
                    }
                };
                edge(last_nd[q]);
                if (dg[k]) {
                    diag_since[q].push_back(j);
                } else {
                    for (int i : diag_since[q]) edge(i);
                    diag_since[q].clear();
                    last_nd[q] = j;
                }
            }
        }
    }
    // Ready items that need a register qubit outside the current layout wait
    // in `waiting` (ordered by index) and in the bucket of their tile position.
    std::set<int> waiting;
    std::vector<std::vector<int>> bucket(64);
    std::priority_queue<int, std::vector<int>, std::greater<int>> runnable;
    std::vector<PhasePlan> out;
    PhasePlan pp;
    auto in_S = [&](int p) { return std::find(pp.S.begin(), pp.S.end(), p) != pp.S.end(); };
    auto make_ready = [&](int j) {
        const int q = needs_register(items[j]);
        if (q < 0 || in_S(pos_of[q])) {
            runnable.push(j);
        } else {
            waiting.insert(j);
            bucket[pos_of[q]].push_back(j);
        }
    };
    for (int j = 0; j < n; ++j)
        if (indeg[j] == 0) make_ready(j);
    int left = n;
    do {
        pp = PhasePlan();
        for (;;) {
            while (!runnable.empty()) {
                const int j = runnable.top();
                runnable.pop();
                pp.items.push_back(j);
                --left;
                for (int k : succ[j])
                    if (--indeg[k] == 0) make_ready(k);
            }
            if (left == 0 || (int)pp.S.size() >= rb || waiting.empty()) break;
            int pick = -1;
            if (out.empty()) {
                for (int j : waiting)
                    if (pos_of[needs_register(items[j])] >= line_bits) {
                        pick = j;
                        break;
                    }
            }
            if (pick < 0) pick = *waiting.begin();
            const int p = pos_of[needs_register(items[pick])];
            pp.S.push_back(p);
            for (int j : bucket[p]) {
                waiting.erase(j);
                runnable.push(j);
            }
            bucket[p].clear();
        }
        fill_slots(&pp.S, b, rb);
        out.push_back(pp);
    } while (left > 0);
    return out;
}
}  // namespace

int pass_class(uint64_t required, bool c64) {
    if (!required) return 4;
    const int top = 63 - __builtin_clzll(required);
    if (top < (c64 ? 4 : 3)) return 0;
    if (top < 12) return 1;
    if (top < 20) return 2;
    return 3;
}

namespace {
// "tgt<q>_<tile|reg|swz|xcd>_<c128|c64>"
int *target_knob(const char *key, int *lo, int *hi) {
    int q = -1;
    char what[8] = {0}, dt[8] = {0};
    if (std::sscanf(key, "tgt%d_%7[a-z]_%7[a-z0-9]", &q, what, dt) != 3) return nullptr;
    if (q < 0 || q >= 64) return nullptr;
    const int d = std::strcmp(dt, "c128") == 0 ? 0 : std::strcmp(dt, "c64") == 0 ? 1 : -1;
    if (d < 0) return nullptr;
    static const char *names[4] = {"tile", "reg", "swz", "xcd"};
    static const int los[4] = {0, 0, 0, 0}, his[4] = {13, 5, 16, 1};  // all 0: unset
    for (int f = 0; f < 4; ++f)
        if (std::strcmp(what, names[f]) == 0) {
            *lo = los[f];
            *hi = f == 1 && d == 0 ? 4 : his[f];
            return &tuning().tgt[d][q][f];
        }
    return nullptr;
}

// "cls<k>_<tile|reg|swz>_<c128|c64>"
int *class_knob(const char *key, int *lo, int *hi) {
    if (int *f = target_knob(key, lo, hi)) return f;
    int k = -1;
    char what[8] = {0}, dt[8] = {0};
    if (std::sscanf(key, "cls%d_%7[a-z]_%7[a-z0-9]", &k, what, dt) != 3) return nullptr;
    if (k < 0 || k >= kPassClasses) return nullptr;
    int d = std::strcmp(dt, "c128") == 0 ? 0 : std::strcmp(dt, "c64") == 0 ? 1 : -1;
    if (d < 0) return nullptr;
    Tuning &t = tuning();
    if (std::strcmp(what, "tile") == 0) {
        *lo = 4;
        *hi = 13;  // 8 thread bits + at most 5 register bits
        return &t.cls_tile[d][k];
    }
    if (std::strcmp(what, "reg") == 0) {
        *lo = 1;
        *hi = d ? 5 : 4;
        return &t.cls_reg[d][k];
    }
    if (std::strcmp(what, "swz") == 0) {
        *lo = 0;
        *hi = 16;
        return &t.cls_swz[d][k];
    }
    return nullptr;
}
}  // namespace

int set_tuning(const char *key, int64_t value) {
    int lo, hi;
    if (int *f = class_knob(key, &lo, &hi)) {
        if (value < lo || value > hi) return -1;
        *f = (int)value;
        return 0;
    }
    for (const Knob &k : kKnobs) {
        if (std::strcmp(k.name, key) == 0) {
            if (value < k.lo || value > k.hi) return -1;
            *k.field(tuning()) = (int)value;
            return 0;
        }
    }
    return -1;
}

int get_tuning(const char *key, int64_t *value) {
    int lo, hi;
    if (int *f = class_knob(key, &lo, &hi)) {
        *value = *f;
        return 0;
    }
    for (const Knob &k : kKnobs) {
        if (std::strcmp(k.name, key) == 0) {
            *value = *k.field(tuning());
            return 0;
        }
    }
    return -1;
}

PlanConfig default_config(int n, bool c64, int fusion) {
    const Tuning &t = tuning();
    const int d = c64 ? 1 : 0;
    PlanConfig c;
    c.n = n;
    c.c64 = c64;
    c.fusion = fusion;
    c.tile_bits = t.tile_bits[d];
    c.reg_bits = t.reg_bits[d];
    c.low_bits = std::min(t.low_bits[d], c.tile_bits);
    c.max_high = std::max(1, std::min(t.max_high[d], c.tile_bits - c.low_bits));
    c.flags = t.nt ? PASS_NT : 0;
    c.nt_mode = t.nt;
    c.swz_bits = t.swz_bits;
    c.dense_min_gates = t.dense_min_gates;
    c.diag_run_min = t.diag_run_min;
    c.half_lds = t.half_lds[d] != 0;
    return c;
}

void clamp_config(PlanConfig *c) {
    // Two complex128 states of 2^5 amplitudes per thread exceed the register
    // file, and with 2^4 the kernel runs one wave per SIMD: adjoint sweeps in
    // complex128 take 8 registers per thread (two waves per SIMD), 2^10-amplitude
    // tiles and a 5-qubit low block (the adjoint_* keys; the 24-qubit,
    // 480-parameter gradient measured 37.5 ms with 2^12 tiles and 16 registers,
    // 23.9 ms with 2^11 tiles and a 6-qubit low block, 23.1 ms now).
    if (c->reverse && !c->c64) {
        c->tile_bits = std::min(c->tile_bits, tuning().adjoint_tile_bits);
        c->reg_bits = std::min(c->reg_bits, 3);
        c->low_bits = std::min(c->low_bits, tuning().adjoint_low_bits);
    }
    c->low_bits = std::min(c->low_bits, c->tile_bits);
    c->max_high = std::max(1, std::min(c->max_high, c->tile_bits - c->low_bits));
}

void gate_matrix(int op, const double *p, cd m[2][2]) {
    const double c = std::cos(0.5 * p[0]), s = std::sin(0.5 * p[0]);
    const cd I(0.0, 1.0);
    switch (op) {
    case QG_H: {
        const double r = 1.0 / std::sqrt(2.0);
        m[0][0] = r; m[0][1] = r; m[1][0] = r; m[1][1] = -r;
        return;
    }
    case QG_X:
        m[0][0] = 0.0; m[0][1] = 1.0; m[1][0] = 1.0; m[1][1] = 0.0;
        return;
    case QG_RX:
        m[0][0] = c; m[0][1] = -I * s; m[1][0] = -I * s; m[1][1] = c;
        return;
    case QG_RY:
        m[0][0] = c; m[0][1] = -s; m[1][0] = s; m[1][1] = c;
        return;
    case QG_RZ:
        m[0][0] = std::polar(1.0, -0.5 * p[0]); m[0][1] = 0.0;
        m[1][0] = 0.0; m[1][1] = std::polar(1.0, 0.5 * p[0]);
        return;
    case QG_U3:
        m[0][0] = c;
        m[0][1] = -std::polar(1.0, p[2]) * s;
        m[1][0] = std::polar(1.0, p[1]) * s;
        m[1][1] = std::polar(1.0, p[1] + p[2]) * c;
        return;
    }
    m[0][0] = 1.0; m[0][1] = 0.0; m[1][0] = 0.0; m[1][1] = 1.0;
}

uint64_t required_qubits(const Gate &g) {
    switch (g.op) {
    case QG_H: case QG_X: case QG_RX: case QG_RY: case QG_U3: case QG_CX:
        return 1ull << g.q1;
    case QG_SWAP:
        return (1ull << g.q0) | (1ull << g.q1);
    }
    return 0;
}

qg_status validate_circuit(const qg_circuit *c, int n_params, std::string *err) {
    if (!c) { *err = "circuit is NULL"; return QG_EINVAL; }
    const int n = c->n_qubits;
    if (n < 1 || n > 34) { *err = "n_qubits must be in [1, 34], got " + std::to_string(n); return QG_EINVAL; }
    if (c->n_gates < 0) { *err = "n_gates < 0"; return QG_EINVAL; }
    if (c->n_gates > 0 && (!c->gate_type || !c->gate_param)) {
        *err = "gate_type / gate_param is NULL";
        return QG_EINVAL;
    }
    for (int g = 0; g < c->n_gates; ++g) {
        const int op = c->gate_type[3 * g], q0 = c->gate_type[3 * g + 1], q1 = c->gate_type[3 * g + 2];
        const double *p = c->gate_param + 3 * g;
        const std::string at = " at gate " + std::to_string(g);
        if (op < QG_H || op > QG_SWAP) { *err = "unknown gate code " + std::to_string(op) + at; return QG_EINVAL; }
        if (q1 < 0 || q1 >= n) { *err = "qubit " + std::to_string(q1) + " out of range" + at; return QG_EINVAL; }
        if (is_two_qubit(op)) {
            if (q0 < 0 || q0 >= n) { *err = "qubit " + std::to_string(q0) + " out of range" + at; return QG_EINVAL; }
            if (q0 == q1) { *err = "two-qubit gate with q0 == q1" + at; return QG_EINVAL; }
        }
        const int used = op == QG_U3 ? 3 : (op == QG_RX || op == QG_RY || op == QG_RZ || op == QG_CP) ? 1 : 0;
        for (int k = 0; k < used; ++k)
            if (!std::isfinite(p[k])) { *err = "non-finite parameter" + at; return QG_EINVAL; }
        if (c->param_idx && c->param_idx[g] >= 0) {
            if (!(op == QG_RX || op == QG_RY || op == QG_RZ || op == QG_CP)) {
                *err = "trainable slot on a gate other than RX/RY/RZ/CP" + at;
                return QG_EINVAL;
            }
            if (n_params >= 0 && c->param_idx[g] >= n_params) {
                *err = "param_idx " + std::to_string(c->param_idx[g]) + " >= n_params" + at;
                return QG_EINVAL;
            }
        }
    }
    return QG_OK;
}

std::vector<Gate> load_gates(const qg_circuit *c) {
    std::vector<Gate> v(c->n_gates);
    for (int g = 0; g < c->n_gates; ++g) {
        Gate &x = v[g];
        x.op = c->gate_type[3 * g];
        x.q0 = c->gate_type[3 * g + 1];
        x.q1 = c->gate_type[3 * g + 2];
        for (int k = 0; k < 3; ++k) x.p[k] = c->gate_param[3 * g + k];
        x.pidx = c->param_idx ? c->param_idx[g] : -1;
    }
    return v;
}

std::vector<Gate> execution_order(const std::vector<Gate> &g, bool reverse) {
    std::vector<Gate> v(g);
    if (reverse) std::reverse(v.begin(), v.end());
    return v;
}

std::vector<PassRange> fuse(const std::vector<Gate> &g, const PlanConfig &cfg) {
    std::vector<PassRange> out;
    const int G = (int)g.size();
    if (cfg.fusion == QG_FUSE_NONE) {
        for (int i = 0; i < G; ++i) out.push_back({i, i + 1});
        return out;
    }
    const int n = cfg.n;
    const int b = std::min(n, cfg.tile_bits);
    // Qubits below low_bits are always in a fused tile; when the whole state is one
    // tile every qubit is.
    const int low = n <= b ? n : std::min(cfg.low_bits, b);
    const uint64_t low_mask = low >= 64 ? ~0ull : ((1ull << low) - 1);
    const int max_high = n <= b ? 64 : std::min(cfg.max_high, b - low);
    const int kMaxGatesPerPass = cfg.max_gates_per_pass;
    const int kMaxGradPerPass = 64;  // bounds the adjoint partial-sum scratch
    int begin = 0, grads = 0;
    uint64_t high = 0;
    for (int i = 0; i < G; ++i) {
        const uint64_t req = required_qubits(g[i]) & ~low_mask;
        const int gr = (cfg.reverse && g[i].pidx >= 0) ? 1 : 0;
        if (i > begin && (popcount64(high | req) > max_high || i - begin >= kMaxGatesPerPass ||
                          grads + gr > kMaxGradPerPass)) {
            out.push_back({begin, i});
            begin = i;
            high = 0;
            grads = 0;
        }
        high |= req;
        grads += gr;
    }
    if (G > begin) out.push_back({begin, G});
    return out;
}

// Runs of consecutive gates (in the given order) that touch at most 6 qubits and
// hold at least dense_min_gates gates: each becomes a pass of its own, which the
// plan then executes as one dense block.  Greedy from the left, longest run
// from each start.  Empty when dense blocks are off or on the automatic
// threshold.
std::vector<PassRange> dense_runs(const std::vector<Gate> &g, const PlanConfig &cfg) {
    std::vector<PassRange> runs;
    const int G = (int)g.size();
    // Only an explicit threshold cuts runs out of the schedule.  Under the measured
    // break-even (dense_min_gates = 0) a greedy pass that happens to touch <= 6
    // qubits becomes a dense block instead, because a run cut out of a larger
    // pass adds a pass of its own (QCrank's Gray-code runs, for one, fit 6 qubits
    // for 62 gates inside passes of thousands).
    if (cfg.reverse || cfg.n < 8 || cfg.dense_min_gates <= 0 || cfg.dense_min_gates >= (1 << 30) ||
        cfg.fusion == QG_FUSE_NONE)
        return runs;
    for (int i = 0; i < G;) {
        uint64_t q = 0;
        int j = i;
        while (j < G && popcount64(q | touched_qubits(g[j])) <= 6) q |= touched_qubits(g[j++]);
        const uint64_t blk = j > i ? dense_block_qubits(g, i, j, cfg.n) : 0;
        if (blk && j - i >= dense_threshold(cfg, popcount64(blk))) {
            runs.push_back({i, j});
            i = j;
        } else {
            ++i;
        }
    }
    return runs;
}

int dense_threshold(const PlanConfig &cfg, int k) {
    if (cfg.dense_min_gates > 0) return cfg.dense_min_gates;
    const int kk = k < 4 ? 4 : k > 6 ? 6 : k;
    return tuning().dense_auto[cfg.c64 ? 1 : 0][kk - 4];
}

Schedule schedule(const std::vector<Gate> &g, const PlanConfig &cfg) {
    Schedule sc;
    const int G = (int)g.size();
    if (cfg.fusion == QG_FUSE_NONE || G == 0) {
        for (int i = 0; i < G; ++i) sc.order.push_back(i);
        sc.ranges = fuse(g, cfg);
        return sc;
    }
    const int n = cfg.n;
    const int b = std::min(n, cfg.tile_bits);
    const int low = n <= b ? n : std::min(cfg.low_bits, b);
    const uint64_t low_mask = low >= 64 ? ~0ull : ((1ull << low) - 1);
    const int max_high = n <= b ? 64 : std::min(cfg.max_high, b - low);
    const int kMaxGradPerPass = 64;  // bounds the adjoint partial-sum scratch
    // Gates between dense runs are scheduled greedily among themselves; a dense
    // run keeps its gates in order as one pass, and nothing moves across it.
    std::vector<PassRange> runs = dense_runs(g, cfg);
    runs.push_back({G, G});
    int seg = 0;
    for (const PassRange &dr : runs) {
        std::vector<int> pending;
        for (int i = seg; i < dr.g_begin; ++i) pending.push_back(i);
        while (!pending.empty()) {
            uint64_t high = 0, blocked = 0;
            int taken = 0, grads = 0;
            std::vector<int> rest;
            rest.reserve(pending.size());
            const int begin = (int)sc.order.size();
            for (int idx : pending) {
                const Gate &x = g[idx];
                const uint64_t touch = touched_qubits(x);
                const uint64_t req = required_qubits(x) & ~low_mask;
                const bool ready = (touch & blocked) == 0;
                const int gr = (cfg.reverse && x.pidx >= 0) ? 1 : 0;
                if (ready && taken < cfg.max_gates_per_pass && grads + gr <= kMaxGradPerPass &&
                    popcount64(high | req) <= max_high) {
                    high |= req;
                    sc.order.push_back(idx);
                    ++taken;
                    grads += gr;
                } else {
                    blocked |= touch;
                    rest.push_back(idx);
                }
            }
            sc.ranges.push_back({begin, (int)sc.order.size()});
            pending.swap(rest);
        }
        if (dr.g_end > dr.g_begin) {
            const int begin = (int)sc.order.size();
            for (int i = dr.g_begin; i < dr.g_end; ++i) sc.order.push_back(i);
            sc.ranges.push_back({begin, (int)sc.order.size()});
        }
        seg = dr.g_end;
    }
    return sc;
}

std::vector<Gate> permute(const std::vector<Gate> &g, const std::vector<int> &order) {
    std::vector<Gate> out;
    out.reserve(order.size());
    for (int i : order) out.push_back(g[i]);
    return out;
}

// Fuses the diagonal items `run` (in order) of a phase into one DiagRun: the
// uniform parts (register slots only) are multiplied out here in FP64, the
// parts that read thread bits or qubits outside the tile become entries.
template <typename SlotOf, typename Ref>
void append_diag_run(const std::vector<Item> &items, const std::vector<int> &run, int rb, SlotOf slot_of, Ref ref,
                     Program *prog) {
    cd s0[kMaxRegBits], s1[kMaxRegBits], q[kMaxRegBits * (kMaxRegBits - 1) / 2];
    for (auto &v : s0) v = 1.0;
    for (auto &v : s1) v = 1.0;
    for (auto &v : q) v = 1.0;
    std::vector<DiagEntry> thr, slot[kMaxRegBits];
    auto entry = [](int a, int c, cd f0, cd f1) {
        DiagEntry e{};
        for (int ref : {a, c}) {
            if (ref == kNoRef) continue;
            if (ref >= 0) e.tmask |= 1u << ref;                  // tile position (a thread bit here)
            else e.gmask |= 1ull << (-1 - ref);                 // qubit outside the tile
        }
        e.f0_one = f0 == cd(1.0) ? 1u : 0u;
        e.f0[0] = f0.real(), e.f0[1] = f0.imag();
        e.f1[0] = f1.real(), e.f1[1] = f1.imag();
        return e;
    };
    for (int ii : run) {
        const Item &it = items[ii];
        if (it.kind == OP_DIAG1) {
            const cd p0(it.m[0], it.m[1]), p1(it.m[2], it.m[3]);
            const int j = slot_of(it.qa);
            if (j >= 0) {
                s0[j] *= p0;
                s1[j] *= p1;
            } else {
                thr.push_back(entry(ref(it.qa), kNoRef, p0, p1));
            }
        } else {
            const cd phi(it.m[0], it.m[1]);
            const int ja = slot_of(it.qa), jc = slot_of(it.qc);
            if (ja >= 0 && jc >= 0) {
                const int lo = std::min(ja, jc), hi = std::max(ja, jc);
                q[hi * (hi - 1) / 2 + lo] *= phi;
            } else if (ja >= 0) {
                slot[ja].push_back(entry(ref(it.qc), kNoRef, 1.0, phi));
            } else if (jc >= 0) {
                slot[jc].push_back(entry(ref(it.qa), kNoRef, 1.0, phi));
            } else {
                thr.push_back(entry(ref(it.qa), ref(it.qc), 1.0, phi));
            }
        }
    }
    DiagRun d{};
    cd c0 = 1.0;
    for (int j = 0; j < rb; ++j) c0 *= s0[j];
    d.c0[0] = c0.real(), d.c0[1] = c0.imag();
    for (int j = 0; j < kMaxRegBits; ++j) {
        // every factor has modulus 1, so s1 / s0 = s1 conj(s0)
        const cd r = s1[j] * std::conj(s0[j]);
        d.r[j][0] = r.real(), d.r[j][1] = r.imag();
    }
    for (int k = 0; k < kMaxRegBits * (kMaxRegBits - 1) / 2; ++k) d.q[k][0] = q[k].real(), d.q[k][1] = q[k].imag();
    d.e_begin = (int)prog->entries.size();
    prog->entries.insert(prog->entries.end(), thr.begin(), thr.end());
    for (int j = 0; j <= kMaxRegBits; ++j) {
        d.s_begin[j] = (int)prog->entries.size();
        if (j < rb) prog->entries.insert(prog->entries.end(), slot[j].begin(), slot[j].end());
    }
    prog->runs.push_back(d);
}

Program build_program(const std::vector<Gate> &gates, const std::vector<PassRange> &ranges,
                      const PlanConfig &cfg) {
    Program prog;
    const int n = cfg.n;
    prog.pass_of_gate.assign(gates.size(), -1);
    int grad_rows = 0;
    for (size_t pi = 0; pi < ranges.size(); ++pi) {
        const PassRange &r = ranges[pi];
        std::vector<Item> items;
        uint64_t req = 0;
        const int grad_base = grad_rows;
        for (int gi = r.g_begin; gi < r.g_end; ++gi) {
            const Gate &g = gates[gi];
            prog.pass_of_gate[gi] = (int)pi;
            req |= required_qubits(g);
            int row = -1;  // gradient row, local to the pass
            if (cfg.reverse && g.pidx >= 0) {
                row = grad_rows++ - grad_base;
                prog.grad_row_slot.push_back(g.pidx);
            }
            gate_items(g, cfg.reverse, row, &items);
        }
        // ---- tile shape: single-gate passes take the tuned shape of their class
        const Tuning &tu = tuning();
        const int dcls = cfg.c64 ? 1 : 0;
        const int cls = pass_class(req, cfg.c64);
        int tile_bits = cfg.tile_bits, reg_bits = cfg.reg_bits, swz_bits = cfg.swz_bits;
        int xcd = tu.xcd;
        if (cfg.use_classes && !cfg.reverse) {
            if (r.g_end - r.g_begin == 1) {
                tile_bits = tu.cls_tile[dcls][cls];
                reg_bits = tu.cls_reg[dcls][cls];
            }
            swz_bits = tu.cls_swz[dcls][cls];
            const Gate &g0 = gates[r.g_begin];
            if (r.g_end - r.g_begin == 1 && is_one_qubit(g0.op) && g0.op != QG_RZ && tu.tgt[dcls][g0.q1][0] > 0 &&
                tu.tgt[dcls][g0.q1][1] > 0) {
                const int *e = tu.tgt[dcls][g0.q1];
                tile_bits = e[0];
                reg_bits = e[1];
                swz_bits = e[2];
                xcd = e[3];
            }
        }
        // ---- tile: required qubits, then the lowest remaining ones
        const int b = std::min(n, std::max(tile_bits, popcount64(req)));
        uint64_t tile = req;
        for (int q = 0; q < n && popcount64(tile) < b; ++q) tile |= 1ull << q;
        int tile_q[kMaxTileBits];
        int pos_of[64];
        for (int q = 0; q < 64; ++q) pos_of[q] = -1;
        int nb = 0;
        for (int q = 0; q < n; ++q)
            if (tile >> q & 1) { pos_of[q] = nb; tile_q[nb++] = q; }
        int rb = std::min(reg_bits, b);
        if (b - rb > kMaxThreadBits) rb = b - kMaxThreadBits;
        const int tb = b - rb;

        // ---- fixed bits: tiles on which every op is the identity are skipped
        uint64_t fixed = items.empty() ? 0 : ~0ull;
        for (const Item &it : items) {
            uint64_t cond = 0;
            if (it.kind == OP_CX && pos_of[it.qc] < 0) cond = 1ull << it.qc;
            if (it.kind == OP_DIAG2 || it.kind == OP_GRADP11) {
                if (pos_of[it.qa] < 0) cond |= 1ull << it.qa;
                if (pos_of[it.qc] < 0) cond |= 1ull << it.qc;
            }
            fixed &= cond;
        }

        PassDesc pd{};
        pd.b = b;
        pd.rb = rb;
        pd.tb = tb;
        pd.fixed_mask = fixed;
        pd.fixed_val = fixed;
        pd.flags = cfg.flags;
        int free_bits = 0;
        for (int q = 0; q < n; ++q) {
            if ((tile >> q & 1) || (fixed >> q & 1)) continue;
            if (pd.n_runs > 0 && pd.run_start[pd.n_runs - 1] + pd.run_len[pd.n_runs - 1] == q) {
                pd.run_len[pd.n_runs - 1]++;
            } else {
                pd.run_start[pd.n_runs] = q;
                pd.run_len[pd.n_runs] = 1;
                pd.n_runs++;
            }
            free_bits++;
        }
        pd.n_tiles = 1ull << free_bits;
        pd.swz_bits = std::min(swz_bits, free_bits / 2);
        if (xcd && free_bits >= 3) pd.flags |= PASS_XCD;
        pd.phase_begin = (int)prog.phases.size();

        // ---- phases: register positions must hold every mixing op's target
        const int line_bits = cfg.c64 ? 4 : 3;
        const std::vector<PhasePlan> plans =
            cfg.reverse ? plan_phases_in_order(items, pos_of, b, rb) : plan_phases(items, pos_of, b, rb, line_bits);
        auto ref = [&](int q) { return pos_of[q] >= 0 ? pos_of[q] : qref_global(q); };
        for (const PhasePlan &pp : plans) {
            const std::vector<int> &S = pp.S;
            PhaseDesc ph{};
            std::vector<int> thr;
            for (int p = 0; p < b; ++p)
                if (std::find(S.begin(), S.end(), p) == S.end()) thr.push_back(p);
            for (int k = 0; k < tb; ++k) {
                ph.thr_goff[k] = 1ull << tile_q[thr[k]];
                ph.thr_poff[k] = 1u << thr[k];
            }
            for (int j = 0; j < rb; ++j) {
                ph.reg_goff[j] = 1ull << tile_q[S[j]];
                ph.reg_poff[j] = 1u << S[j];
            }
            ph.op_begin = (int)prog.ops.size();
            // register slot of a qubit in this phase's layout, or -1
            auto slot_of = [&](int qq) {
                if (pos_of[qq] < 0) return -1;
                auto f = std::find(S.begin(), S.end(), pos_of[qq]);
                return f == S.end() ? -1 : (int)(f - S.begin());
            };
            auto is_diag = [&](int ii) { return items[ii].kind == OP_DIAG1 || items[ii].kind == OP_DIAG2; };
            for (size_t x = 0; x < pp.items.size(); ++x) {
                const int ii = pp.items[x];
                if (cfg.diag_run_min > 0 && !cfg.reverse && is_diag(ii)) {
                    size_t y = x;
                    while (y < pp.items.size() && is_diag(pp.items[y])) ++y;
                    if ((int)(y - x) >= cfg.diag_run_min) {
                        DevOp op{};
                        op.kind = OP_DIAGRUN;
                        op.g = -1;
                        op.a = (int)prog.runs.size();
                        std::vector<int> run(pp.items.begin() + x, pp.items.begin() + y);
                        append_diag_run(items, run, rb, slot_of, ref, &prog);
                        prog.ops.push_back(op);
                        x = y - 1;
                        continue;
                    }
                }
                const Item &it = items[ii];
                const int q = needs_register(it);
                const int slot = q >= 0 ? slot_of(q) : -1;
                DevOp op{};
                op.kind = it.kind;
                op.g = it.g;
                std::memcpy(op.m, it.m, sizeof op.m);
                switch (it.kind) {
                case OP_MAT:
                    op.a = slot;
                    // m = {m00, m01, m10, m11} as (re, im) pairs
                    if (it.m[1] == 0 && it.m[3] == 0 && it.m[5] == 0 && it.m[7] == 0)
                        op.kind = OP_MATR;
                    else if (it.m[1] == 0 && it.m[2] == 0 && it.m[4] == 0 && it.m[7] == 0)
                        op.kind = OP_MATRX;
                    break;
                case OP_GRADX: case OP_GRADY:
                    op.a = slot;
                    break;
                case OP_CX:
                    op.a = slot;
                    if (slot_of(it.qc) >= 0) {
                        op.kind = OP_CXRR;
                        op.c = slot_of(it.qc);
                    } else {
                        op.c = ref(it.qc);
                    }
                    break;
                case OP_DIAG1:
                    if (slot_of(it.qa) >= 0) {
                        op.kind = OP_DIAG1R;
                        op.a = slot_of(it.qa);
                    } else {
                        op.a = ref(it.qa);
                    }
                    break;
                case OP_GRADZ:
                    op.a = ref(it.qa);
                    break;
                case OP_DIAG2: {
                    const int sa = slot_of(it.qa), sc = slot_of(it.qc);
                    if (sa >= 0 && sc >= 0) {
                        op.kind = OP_DIAG2RR;
                        op.a = sa;
                        op.c = sc;
                    } else if (sa >= 0 || sc >= 0) {
                        op.kind = OP_DIAG2R;
                        op.a = sa >= 0 ? sa : sc;
                        op.c = ref(sa >= 0 ? it.qc : it.qa);
                    } else {
                        op.a = ref(it.qa);
                        op.c = ref(it.qc);
                    }
                    break;
                }
                case OP_GRADP11:
                    op.a = ref(it.qa);
                    op.c = ref(it.qc);
                    break;
                }
                prog.ops.push_back(op);
            }
            ph.op_end = (int)prog.ops.size();
            prog.phases.push_back(ph);
        }
        pd.n_phase = (int)prog.phases.size() - pd.phase_begin;
        const int n_ops = prog.phases.back().op_end - prog.phases[pd.phase_begin].op_begin;
        if (!cfg.reverse && (tu.pipe == 2 || (tu.pipe == 1 && (pd.n_phase > 1 || n_ops >= tu.pipe_min_ops))))
            pd.flags |= PASS_PIPE;
        if (pd.n_phase > 1 && cfg.half_lds) pd.flags |= PASS_HALFX;
        // Non-temporal state accesses only pay when every wavefront load/store
        // covers whole 128-byte lines: the first and last layouts must keep the
        // line-offset tile positions (3 for complex128, 4 for complex64) on lanes.
        if ((pd.flags & PASS_NT) && cfg.nt_mode == 1) {
            const uint32_t line_mask = (1u << std::min(line_bits, b)) - 1;
            for (int which : {pd.phase_begin, pd.phase_begin + pd.n_phase - 1}) {
                const PhaseDesc &ph = prog.phases[which];
                for (int j = 0; j < rb; ++j)
                    if (ph.reg_poff[j] & line_mask) pd.flags &= ~PASS_NT;
                if (tb < line_bits) pd.flags &= ~PASS_NT;
            }
        }
        pd.grad_base = grad_base;
        pd.n_grad = grad_rows - grad_base;
        const int64_t waves = std::max(1, (1 << tb) / 64);
        prog.max_grad_part = std::max<int64_t>(prog.max_grad_part, (int64_t)pd.n_tiles * waves * pd.n_grad);
        prog.passes.push_back(pd);
    }
    return prog;
}

uint64_t touched_qubits(const Gate &g) {
    uint64_t m = 1ull << g.q1;
    if (g.op >= QG_CX) m |= 1ull << g.q0;
    return m;
}

uint64_t dense_block_qubits(const std::vector<Gate> &g, int begin, int end, int n) {
    uint64_t q = 0;
    for (int i = begin; i < end; ++i) q |= touched_qubits(g[i]);
    if (popcount64(q) > 6 || n < 8 || n - std::max(4, popcount64(q)) < 4) return 0;
    // at least 4 block qubits (16-row matrix tiles): add the highest untouched qubits
    for (int b = n - 1; b >= 0 && popcount64(q) < 4; --b) q |= 1ull << b;
    return q;
}

namespace {

// Column-by-column product U <- G U on the k block qubits (local bit j = j-th block qubit).
void dense_apply(std::vector<cd> &U, int k, const Gate &g, const int *local_of) {
    const int dim = 1 << k;
    const int t = local_of[g.q1];
    const int c = g.op >= QG_CX ? local_of[g.q0] : -1;
    cd m[2][2];
    if (g.op <= QG_U3) gate_matrix(g.op, g.p, m);
    for (int col = 0; col < dim; ++col) {
        cd *v = U.data() + (size_t)col;  // element r of column col is U[r * dim + col]
        auto at = [&](int r) -> cd & { return v[(size_t)r * dim]; };
        for (int r = 0; r < dim; ++r) {
            const int bt = (r >> t) & 1;
            switch (g.op) {
            case QG_CX:
                if (((r >> c) & 1) && !bt) std::swap(at(r), at(r | (1 << t)));
                break;
            case QG_CZ:
                if (((r >> c) & 1) && bt) at(r) = -at(r);
                break;
            case QG_CP:
                if (((r >> c) & 1) && bt) at(r) *= std::polar(1.0, g.p[0]);
                break;
            case QG_SWAP:
                if (((r >> c) & 1) && !bt) std::swap(at(r), at((r ^ (1 << c)) | (1 << t)));
                break;
            default:
                if (!bt) {
                    const cd a0 = at(r), a1 = at(r | (1 << t));
                    at(r) = m[0][0] * a0 + m[0][1] * a1;
                    at(r | (1 << t)) = m[1][0] * a0 + m[1][1] * a1;
                }
            }
        }
    }
}

}  // namespace

void append_dense(Program *prog, const std::vector<Gate> &g, int begin, int end, uint64_t blk, const PlanConfig &cfg) {
    const int n = cfg.n;
    DenseDesc D{};
    int local_of[64];
    for (int q = 0; q < 64; ++q) local_of[q] = -1;
    int k = 0;
    for (int q = 0; q < n; ++q)
        if (blk >> q & 1) {
            local_of[q] = k;
            D.blk_q[k++] = (int8_t)q;
        }
    D.k = k;
    const int tile = std::min(n, tuning().dense_tile_bits);
    const int l = std::min(tile - k, n - k);
    int li = 0;
    uint64_t used = blk;
    for (int q = 0; q < n && li < l; ++q)
        if (!(blk >> q & 1)) {
            D.low_q[li++] = (int8_t)q;
            used |= 1ull << q;
        }
    D.l = li;
    int free_bits = 0;
    for (int q = 0; q < n; ++q) {
        if (used >> q & 1) continue;
        if (D.n_runs > 0 && D.run_start[D.n_runs - 1] + D.run_len[D.n_runs - 1] == q) {
            D.run_len[D.n_runs - 1]++;
        } else {
            D.run_start[D.n_runs] = q;
            D.run_len[D.n_runs] = 1;
            D.n_runs++;
        }
        free_bits++;
    }
    D.n_tiles = 1ull << free_bits;
    const int dim = 1 << k;
    std::vector<cd> U((size_t)dim * dim, 0.0);
    for (int r = 0; r < dim; ++r) U[(size_t)r * dim + r] = 1.0;
    for (int i = begin; i < end; ++i) dense_apply(U, k, g[i], local_of);
    D.u_index = (int64_t)prog->dense_ut.size();
    // transposed: UT[c][r] = U[r][c]; re block then im block
    for (int part = 0; part < 2; ++part)
        for (int c = 0; c < dim; ++c)
            for (int r = 0; r < dim; ++r) {
                const cd v = U[(size_t)r * dim + c];
                prog->dense_ut.push_back(part ? v.imag() : v.real());
            }
    PassDesc pd{};
    pd.flags = PASS_DENSE;
    pd.phase_begin = (int)prog->dense.size();
    pd.n_phase = 0;
    pd.n_tiles = D.n_tiles;
    pd.b = k + li;
    prog->dense.push_back(D);
    prog->passes.push_back(pd);
}

namespace {
// Standalone SWAPs run as permutations: half the state when both qubits are at
// or above the line bits, otherwise (lower qubit a lane bit) the whole state
// with a cross-lane exchange.
int swap_kind(const std::vector<Gate> &g, const PassRange &r, const PlanConfig &cfg) {
    if (cfg.reverse || r.g_end - r.g_begin != 1 || g[r.g_begin].op != QG_SWAP) return 0;
    const int line_bits = cfg.c64 ? 4 : 3;
    const int lo = std::min(g[r.g_begin].q0, g[r.g_begin].q1);
    if (lo >= line_bits) return PASS_SWAP2;
    return cfg.n >= 12 && tuning().lane_swap ? PASS_SWAPL : 0;
}

// A single one-qubit mixing gate or CX whose target lies inside a cache line
// runs as a cross-lane exchange with whole-line accesses.
bool lane_gate(const std::vector<Gate> &g, const PassRange &r, const PlanConfig &cfg) {
    if (cfg.reverse || r.g_end - r.g_begin != 1 || cfg.n < 12 || !tuning().lane_gate) return false;
    const int line_bits = cfg.c64 ? 4 : 3;
    const Gate &x = g[r.g_begin];
    return ((is_one_qubit(x.op) && x.op != QG_RZ) || x.op == QG_CX) && x.q1 < line_bits;
}
}  // namespace

uint64_t range_dense_block(const std::vector<Gate> &g, const PassRange &r, const PlanConfig &cfg) {
    if (cfg.reverse || cfg.n < 8 || cfg.dense_min_gates >= (1 << 30)) return 0;
    const uint64_t blk = dense_block_qubits(g, r.g_begin, r.g_end, cfg.n);
    return blk && r.g_end - r.g_begin >= dense_threshold(cfg, popcount64(blk)) ? blk : 0;
}

void append_range(Program *prog, const std::vector<Gate> &g, const PassRange &r, const PlanConfig &cfg) {
    const Gate &g1 = g[r.g_begin];
    if (lane_gate(g, r, cfg)) {
        std::vector<Item> its;
        gate_items(g1, false, -1, &its);
        DevOp op{};
        op.kind = its[0].kind;
        op.g = -1;
        std::memcpy(op.m, its[0].m, sizeof op.m);
        PassDesc pd{};
        pd.flags = PASS_LANE1 | (tuning().xcd ? PASS_XCD : 0);
        pd.run_start[0] = g1.q1;
        pd.run_start[1] = g1.op == QG_CX ? g1.q0 : -1;
        pd.n_tiles = 1ull << (cfg.n - 2);
        pd.phase_begin = (int)prog->ops.size();
        prog->ops.push_back(op);
        prog->passes.push_back(pd);
        return;
    }
    if (const int kind = swap_kind(g, r, cfg)) {
        PassDesc pd{};
        pd.flags = kind | (tuning().xcd ? PASS_XCD : 0);
        pd.run_start[0] = g1.q0;
        pd.run_start[1] = g1.q1;
        pd.n_tiles = 1ull << (cfg.n - 2);
        prog->passes.push_back(pd);
        return;
    }
    if (const uint64_t blk = range_dense_block(g, r, cfg)) {
        append_dense(prog, g, r.g_begin, r.g_end, blk, cfg);
    } else {
        std::vector<PassRange> one{r};
        append_program(prog, build_program(g, one, cfg));
    }
}

Program build_plan(const std::vector<Gate> &g0, const PlanConfig &cfg, std::vector<int> *order) {
    Schedule sc = schedule(g0, cfg);
    if (order) *order = sc.order;
    const std::vector<Gate> g = permute(g0, sc.order);
    const std::vector<PassRange> &ranges = sc.ranges;
    bool special = false;
    for (const PassRange &r : ranges) special |= swap_kind(g, r, cfg) != 0 || lane_gate(g, r, cfg);
    // Adjoint sweeps number their gradient rows across the whole program: one build.
    if (cfg.reverse || (!special && (cfg.dense_min_gates >= (1 << 30) || cfg.n < 8)))
        return build_program(g, ranges, cfg);
    Program prog;
    prog.pass_of_gate.assign(g.size(), -1);
    for (size_t p = 0; p < ranges.size(); ++p) {
        append_range(&prog, g, ranges[p], cfg);
        for (int i = ranges[p].g_begin; i < ranges[p].g_end; ++i) prog.pass_of_gate[i] = (int)p;
    }
    return prog;
}

void append_program(Program *dst, const Program &src) {
    const int ph0 = (int)dst->phases.size(), op0 = (int)dst->ops.size(), pass0 = (int)dst->passes.size();
    const int d0 = (int)dst->dense.size();
    const int64_t u0 = (int64_t)dst->dense_ut.size();
    for (PassDesc pd : src.passes) {
        if (pd.flags & PASS_LANE1) pd.phase_begin += op0;  // index of its matrix op
        else if (!(pd.flags & (PASS_SWAP2 | PASS_SWAPL))) pd.phase_begin += (pd.flags & PASS_DENSE) ? d0 : ph0;
        dst->passes.push_back(pd);
    }
    for (DenseDesc d : src.dense) {
        d.u_index += u0;
        dst->dense.push_back(d);
    }
    dst->dense_ut.insert(dst->dense_ut.end(), src.dense_ut.begin(), src.dense_ut.end());
    for (PhaseDesc ph : src.phases) {
        ph.op_begin += op0;
        ph.op_end += op0;
        dst->phases.push_back(ph);
    }
    const int r0 = (int)dst->runs.size(), e0 = (int)dst->entries.size();
    for (DevOp op : src.ops) {
        if (op.kind == OP_DIAGRUN) op.a += r0;
        dst->ops.push_back(op);
    }
    for (DiagRun d : src.runs) {
        d.e_begin += e0;
        for (int &b : d.s_begin) b += e0;
        dst->runs.push_back(d);
    }
    dst->entries.insert(dst->entries.end(), src.entries.begin(), src.entries.end());
    (void)pass0;
}

PlanConfig candidate_config(int n, bool c64, int k) {
    PlanConfig c = default_config(n, c64, QG_FUSE_GREEDY);
    // max_high = 4 + k; low_bits fills the rest of the tile
    c.max_high = 4 + k;
    c.low_bits = c.tile_bits - c.max_high;
    clamp_config(&c);
    return c;
}

int first_block_end(const std::vector<Gate> &g, int begin, const PlanConfig &cfg) {
    const int G = (int)g.size();
    const int n = cfg.n;
    const int b = std::min(n, cfg.tile_bits);
    const int low = n <= b ? n : std::min(cfg.low_bits, b);
    const uint64_t low_mask = low >= 64 ? ~0ull : ((1ull << low) - 1);
    const int max_high = n <= b ? 64 : std::min(cfg.max_high, b - low);
    uint64_t high = 0;
    int i = begin;
    for (; i < G; ++i) {
        const uint64_t req = required_qubits(g[i]) & ~low_mask;
        if (i > begin && (popcount64(high | req) > max_high || i - begin >= cfg.max_gates_per_pass)) break;
        high |= req;
    }
    return i;
}

// Scaled features (see the cost-model kernels): qubits, precision, log2 of the
// active fraction and of the bytes moved, gate / op / phase counts, required
// qubits (all, and outside the low block), tile shape, fusion knobs, and the
// count of each gate code.
void pass_features(const std::vector<Gate> &g, int begin, int end, const PlanConfig &cfg, float *f) {
    std::vector<Gate> sub(g.begin() + begin, g.begin() + end);
    std::vector<PassRange> one{{0, (int)sub.size()}};
    Program p = build_program(sub, one, cfg);
    const PassDesc &pd = p.passes[0];
    uint64_t req = 0;
    int counts[10] = {0};
    for (const Gate &x : sub) {
        req |= required_qubits(x);
        counts[x.op]++;
    }
    const int fixed = popcount64(pd.fixed_mask);
    const int sbits = cfg.c64 ? 3 : 4;
    const uint64_t low_mask = cfg.low_bits >= 64 ? ~0ull : ((1ull << cfg.low_bits) - 1);
    f[0] = cfg.n / 32.f;
    f[1] = cfg.c64 ? 0.f : 1.f;
    f[2] = -fixed / 4.f;
    f[3] = (cfg.n + sbits + 1 - fixed - 30) / 4.f;
    f[4] = sub.size() / 32.f;
    f[5] = p.ops.size() / 32.f;
    f[6] = pd.n_phase / 8.f;
    f[7] = 0.f;  // strategy: tile pass
    f[8] = popcount64(req) / 8.f;
    f[9] = popcount64(req & ~low_mask) / 8.f;
    f[10] = pd.b / 16.f;
    f[11] = pd.rb / 5.f;
    f[12] = cfg.low_bits / 16.f;
    f[13] = cfg.max_high / 8.f;
    for (int k = 0; k < 10; ++k) f[14 + k] = counts[k] / 16.f;
}

void dense_features(const std::vector<Gate> &g, int begin, int end, uint64_t blk, const PlanConfig &cfg, float *f) {
    int counts[10] = {0};
    uint64_t req = 0;
    for (int i = begin; i < end; ++i) {
        counts[g[i].op]++;
        req |= required_qubits(g[i]);
    }
    const int k = popcount64(blk);
    const int l = std::min(std::min(cfg.n, cfg.tile_bits) - k, cfg.n - k);
    const int sbits = cfg.c64 ? 3 : 4;
    const uint64_t low_mask = cfg.low_bits >= 64 ? ~0ull : ((1ull << cfg.low_bits) - 1);
    f[0] = cfg.n / 32.f;
    f[1] = cfg.c64 ? 0.f : 1.f;
    f[2] = 0.f;
    f[3] = (cfg.n + sbits + 1 - 30) / 4.f;
    f[4] = (end - begin) / 32.f;
    f[5] = (end - begin) / 32.f;
    f[6] = 1 / 8.f;
    f[7] = 1.f;  // strategy: dense block
    f[8] = k / 8.f;
    f[9] = popcount64(blk & ~low_mask) / 8.f;
    f[10] = (k + l) / 16.f;
    f[11] = 0.f;
    f[12] = l / 16.f;
    f[13] = k / 8.f;
    for (int j = 0; j < 10; ++j) f[14 + j] = counts[j] / 16.f;
    (void)req;
}

int dense_block_end(const std::vector<Gate> &g, int begin, int max_gates) {
    uint64_t q = 0;
    int i = begin;
    for (; i < (int)g.size() && i - begin < max_gates; ++i) {
        const uint64_t nq = q | touched_qubits(g[i]);
        if (popcount64(nq) > 6) break;
        q = nq;
    }
    return i;
}

}  // namespace qg
