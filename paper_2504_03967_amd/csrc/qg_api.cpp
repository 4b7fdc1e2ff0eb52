// qg_api.cpp -- the C ABI of libqg.so: validation, state handles, uploads and
// the launch sequences of each entry point (declared and documented in qg.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qg.h"
#include "qg_kernels.h"
#include "qg_plan.h"

using namespace qg;

namespace {

thread_local std::string g_err;

qg_status fail(qg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

qg_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? QG_ENOMEM : QG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Device buffer that only grows.  Shrinking never happens, so pointers handed
// to enqueued kernels stay valid until the next growth, which first waits for
// the stream.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes, hipStream_t st) {
        if (bytes <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) return e;
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = bytes + bytes / 4 + 4096;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Pinned host staging for uploads.  The next writer waits for the previous
// copy out of it (event), so host data can be reused as soon as a call returns.
struct Staging {
    void *h = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    hipError_t ready(size_t bytes) {
        if (pending) {
            hipError_t e = hipEventSynchronize(ev);
            if (e != hipSuccess) return e;
            pending = false;
        }
        if (!ev) {
            hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        if (bytes > cap) {
            if (h) (void)hipHostFree(h);
            h = nullptr;
            cap = 0;
            size_t want = bytes + bytes / 4 + 4096;
            hipError_t e = hipHostMalloc(&h, want, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            cap = want;
        }
        return hipSuccess;
    }
    void release() {
        if (pending && ev) (void)hipEventSynchronize(ev);
        if (h) (void)hipHostFree(h);
        if (ev) (void)hipEventDestroy(ev);
        h = nullptr;
        ev = nullptr;
        cap = 0;
        pending = false;
    }
};

// Packs several host arrays into one upload; offsets are 256-byte aligned.
struct Pack {
    std::vector<unsigned char> bytes;
    size_t add(const void *src, size_t n) {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + n);
        if (n) std::memcpy(bytes.data() + off, src, n);
        return off;
    }
    template <typename T>
    size_t add(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

struct Ctx {
    hipStream_t stream = nullptr;
    Staging stage;
    DevBuf upload;   // uploaded program / index / mask tables
    DevBuf work;     // partial sums, sampling tree
    DevBuf work2;    // gradient rows
    ~Ctx() {
        stage.release();
        upload.release();
        work.release();
        work2.release();
    }
    // Copies the pack to `upload` on the stream; returns the device base pointer.
    hipError_t push(const Pack &pk, unsigned char **dev) {
        const size_t n = pk.bytes.size();
        hipError_t e = upload.ensure(n ? n : 1, stream);
        if (e != hipSuccess) return e;
        *dev = static_cast<unsigned char *>(upload.p);
        if (!n) return hipSuccess;
        e = stage.ready(n);
        if (e != hipSuccess) return e;
        std::memcpy(stage.h, pk.bytes.data(), n);
        e = hipMemcpyAsync(upload.p, stage.h, n, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
        e = hipEventRecord(stage.ev, stream);
        if (e != hipSuccess) return e;
        stage.pending = true;
        return hipSuccess;
    }
};

size_t amp_bytes(qg_dtype dt) { return dt == QG_C64 ? 8 : 16; }
int max_qubits(qg_dtype dt) { return dt == QG_C64 ? 34 : 33; }

// Runs a program's passes on psi (and lam when ns == 2) with the uploaded copy at dev.
qg_status run_program(Ctx &cx, bool c64, const Program &prog, void *psi, void *lam, double *rows_out) {
    if (prog.passes.empty()) return QG_OK;
    Pack pk;
    const size_t pass_off = pk.add(prog.passes);
    const size_t phase_off = pk.add(prog.phases);
    const size_t op_off = pk.add(prog.ops);
    unsigned char *dev = nullptr;
    HIP_TRY(cx.push(pk, &dev), "upload program");
    const int ns = lam ? 2 : 1;
    double *gpart = nullptr;
    int64_t gstride = 0;
    if (ns == 2 && prog.max_grad_part > 0) {
        HIP_TRY(cx.work.ensure(prog.max_grad_part * sizeof(double), cx.stream), "allocate gradient partials");
        gpart = static_cast<double *>(cx.work.p);
    }
    for (size_t p = 0; p < prog.passes.size(); ++p) {
        const PassDesc &pd = prog.passes[p];
        const int64_t waves = pd.tb >= 6 ? (int64_t(1) << pd.tb) / 64 : 1;
        gstride = (int64_t)pd.n_tiles * waves;
        HIP_TRY(launch_tile(c64, pd, dev, pass_off, phase_off, op_off, (int)p, ns, psi, lam, gpart, gstride,
                            cx.stream),
                "tile kernel launch");
        if (ns == 2 && pd.n_grad > 0) {
            HIP_TRY(launch_grad_rows(gpart, gstride, gstride, pd.n_grad, rows_out + pd.grad_base, cx.stream),
                    "gradient row reduction");
        }
    }
    return QG_OK;
}

PlanConfig plan_config(int n, bool c64, int fusion) {
    PlanConfig cfg = default_config(n, c64, fusion == QG_FUSE_LEARNED ? QG_FUSE_GREEDY : fusion);
    return cfg;
}

qg_status check_masks(const uint64_t *m, int n_terms, int n) {
    if (n_terms < 0) return fail(QG_EINVAL, "n_terms < 0");
    if (n_terms > 0 && !m) return fail(QG_EINVAL, "zmask is NULL");
    for (int t = 0; t < n_terms; ++t)
        if (n < 64 && (m[t] >> n) != 0) return fail(QG_EINVAL, "zmask[%d] has bits at or above n = %d", t, n);
    return QG_OK;
}

}  // namespace

struct qg_state {
    int n = 0;
    qg_dtype dt = QG_C128;
    void *buf = nullptr;
    bool owned = false;
    Ctx cx;
    uint64_t dim() const { return 1ull << n; }
    bool c64() const { return dt == QG_C64; }
};

extern "C" {

const char *qg_last_error(void) { return g_err.c_str(); }

const char *qg_version(void) { return "qgear-mi355x 0.1 (gfx950)"; }

qg_status qg_state_alloc(int n_qubits, qg_dtype dtype, void *dev_buf, size_t buf_bytes, void *hip_stream,
                         qg_state **out) {
    if (!out) return fail(QG_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != QG_C64 && dtype != QG_C128) return fail(QG_EINVAL, "unknown dtype %d", (int)dtype);
    if (n_qubits < 1 || n_qubits > max_qubits(dtype))
        return fail(QG_EINVAL, "n_qubits = %d outside [1, %d] for this dtype", n_qubits, max_qubits(dtype));
    const size_t need = amp_bytes(dtype) << n_qubits;
    if (dev_buf && buf_bytes < need)
        return fail(QG_EINVAL, "buffer of %zu bytes is smaller than the %zu-byte state", buf_bytes, need);
    qg_state *s = new (std::nothrow) qg_state;
    if (!s) return fail(QG_ENOMEM, "host allocation failed");
    s->n = n_qubits;
    s->dt = dtype;
    s->cx.stream = static_cast<hipStream_t>(hip_stream);
    if (dev_buf) {
        s->buf = dev_buf;
    } else {
        hipError_t e = hipMalloc(&s->buf, need);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e, "state allocation");
        }
        s->owned = true;
    }
    hipError_t e = launch_zero_state(s->c64(), s->buf, s->dim(), s->cx.stream);
    if (e != hipSuccess) {
        if (s->owned) (void)hipFree(s->buf);
        delete s;
        return hip_fail(e, "state init");
    }
    *out = s;
    return QG_OK;
}

qg_status qg_state_free(qg_state *s) {
    if (!s) return QG_OK;
    hipError_t e = hipStreamSynchronize(s->cx.stream);
    if (s->owned) (void)hipFree(s->buf);
    delete s;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    return QG_OK;
}

qg_status qg_state_reset(qg_state *s) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    HIP_TRY(launch_zero_state(s->c64(), s->buf, s->dim(), s->cx.stream), "state init");
    return QG_OK;
}

qg_status qg_state_set_stream(qg_state *s, void *hip_stream) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    s->cx.stream = static_cast<hipStream_t>(hip_stream);
    return QG_OK;
}

qg_status qg_state_info(const qg_state *s, void **dev_ptr, int *n_qubits, qg_dtype *dtype) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    if (dev_ptr) *dev_ptr = s->buf;
    if (n_qubits) *n_qubits = s->n;
    if (dtype) *dtype = s->dt;
    return QG_OK;
}

qg_status qg_plan_passes(const qg_circuit *c, qg_dtype dtype, int fusion_mode, int32_t *pass_of_gate,
                         int32_t *n_passes) {
    std::string err;
    if (validate_circuit(c, -1, &err) != QG_OK) return fail(QG_EINVAL, "%s", err.c_str());
    if (fusion_mode < QG_FUSE_NONE || fusion_mode > QG_FUSE_LEARNED)
        return fail(QG_EINVAL, "unknown fusion mode %d", fusion_mode);
    if (dtype != QG_C64 && dtype != QG_C128) return fail(QG_EINVAL, "unknown dtype %d", (int)dtype);
    std::vector<Gate> g = load_gates(c);
    PlanConfig cfg = plan_config(c->n_qubits, dtype == QG_C64, fusion_mode);
    std::vector<PassRange> r = fuse(g, cfg);
    for (size_t p = 0; p < r.size(); ++p)
        for (int i = r[p].g_begin; i < r[p].g_end; ++i)
            if (pass_of_gate) pass_of_gate[i] = (int32_t)p;
    if (n_passes) *n_passes = (int32_t)r.size();
    return QG_OK;
}

qg_status qg_apply_circuit(qg_state *s, const qg_circuit *c, int fusion_mode) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    std::string err;
    if (validate_circuit(c, -1, &err) != QG_OK) return fail(QG_EINVAL, "%s", err.c_str());
    if (c->n_qubits != s->n)
        return fail(QG_EINVAL, "circuit has %d qubits, state has %d", c->n_qubits, s->n);
    if (fusion_mode < QG_FUSE_NONE || fusion_mode > QG_FUSE_LEARNED)
        return fail(QG_EINVAL, "unknown fusion mode %d", fusion_mode);
    if (c->n_gates == 0) return QG_OK;
    std::vector<Gate> g = load_gates(c);
    PlanConfig cfg = plan_config(s->n, s->c64(), fusion_mode);
    Program prog = build_program(g, fuse(g, cfg), cfg);
    return run_program(s->cx, s->c64(), prog, s->buf, nullptr, nullptr);
}

qg_status qg_probs(qg_state *s, const uint64_t *idx, int64_t n_idx, double *out) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    if (!out) return fail(QG_EINVAL, "out is NULL");
    if (idx) {
        if (n_idx < 0) return fail(QG_EINVAL, "n_idx < 0");
        for (int64_t k = 0; k < n_idx; ++k)
            if (idx[k] >= s->dim()) return fail(QG_EINVAL, "idx[%lld] = %llu >= 2^n", (long long)k, (unsigned long long)idx[k]);
        if (n_idx == 0) return QG_OK;
        Pack pk;
        pk.add(idx, n_idx * sizeof(uint64_t));
        unsigned char *dev = nullptr;
        HIP_TRY(s->cx.push(pk, &dev), "upload indices");
        HIP_TRY(launch_probs(s->c64(), s->buf, s->dim(), reinterpret_cast<const uint64_t *>(dev), n_idx, out,
                             s->cx.stream),
                "probs kernel");
        return QG_OK;
    }
    HIP_TRY(launch_probs(s->c64(), s->buf, s->dim(), nullptr, 0, out, s->cx.stream), "probs kernel");
    return QG_OK;
}

qg_status qg_sample(qg_state *s, int64_t shots, uint64_t seed, uint64_t *out_idx) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    if (shots < 0) return fail(QG_EINVAL, "shots < 0");
    if (shots == 0) return QG_OK;
    if (!out_idx) return fail(QG_EINVAL, "out_idx is NULL");
    HIP_TRY(s->cx.work.ensure(sample_tree_doubles(s->dim()) * sizeof(double), s->cx.stream), "sampling scratch");
    HIP_TRY(launch_sample(s->c64(), s->buf, s->dim(), shots, seed, static_cast<double *>(s->cx.work.p), out_idx,
                          s->cx.stream),
            "sampling kernels");
    return QG_OK;
}

qg_status qg_expval(qg_state *s, const uint64_t *zmask, const double *coeff, int n_terms, double *out_terms,
                    double *out_sum) {
    if (!s) return fail(QG_EINVAL, "state is NULL");
    qg_status st = check_masks(zmask, n_terms, s->n);
    if (st != QG_OK) return st;
    if (out_sum && !coeff && n_terms > 0) return fail(QG_EINVAL, "coeff is NULL but out_sum is requested");
    if (n_terms == 0) {
        if (out_sum) HIP_TRY(hipMemsetAsync(out_sum, 0, sizeof(double), s->cx.stream), "clear out_sum");
        return QG_OK;
    }
    Pack pk;
    const size_t mo = pk.add(zmask, n_terms * sizeof(uint64_t));
    std::vector<double> cf(n_terms, 0.0);
    if (coeff) std::memcpy(cf.data(), coeff, n_terms * sizeof(double));
    const size_t co = pk.add(cf);
    unsigned char *dev = nullptr;
    HIP_TRY(s->cx.push(pk, &dev), "upload masks");
    HIP_TRY(s->cx.work.ensure(expval_partials(s->dim(), n_terms) * sizeof(double), s->cx.stream), "expval scratch");
    HIP_TRY(launch_expval(s->c64(), s->buf, s->dim(), reinterpret_cast<const uint64_t *>(dev + mo),
                          reinterpret_cast<const double *>(dev + co), n_terms, static_cast<double *>(s->cx.work.p),
                          out_terms, out_sum, s->cx.stream),
            "expval kernels");
    return QG_OK;
}

qg_status qg_adjoint_grad(const qg_circuit *c, qg_dtype dtype, const uint64_t *zmask, const double *coeff,
                          int n_terms, int n_params, void *hip_stream, double *out_value, double *out_grad) {
    if (dtype != QG_C64 && dtype != QG_C128) return fail(QG_EINVAL, "unknown dtype %d", (int)dtype);
    if (n_params < 0) return fail(QG_EINVAL, "n_params < 0");
    std::string err;
    if (validate_circuit(c, n_params, &err) != QG_OK) return fail(QG_EINVAL, "%s", err.c_str());
    const int n = c->n_qubits;
    if (n > max_qubits(dtype)) return fail(QG_EINVAL, "n_qubits = %d too large for this dtype", n);
    qg_status st = check_masks(zmask, n_terms, n);
    if (st != QG_OK) return st;
    if (n_terms > 0 && !coeff) return fail(QG_EINVAL, "coeff is NULL");
    if (!out_value) return fail(QG_EINVAL, "out_value is NULL");
    if (n_params > 0 && !out_grad) return fail(QG_EINVAL, "out_grad is NULL");
    const bool c64 = dtype == QG_C64;
    const uint64_t dim = 1ull << n;
    const size_t sbytes = amp_bytes(dtype) << n;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && 2 * sbytes + (64u << 20) > free_b)
        return fail(QG_ENOMEM, "adjoint needs two %zu-byte states, %zu bytes free", sbytes, free_b);

    Ctx cx;
    cx.stream = static_cast<hipStream_t>(hip_stream);
    DevBuf states;
    HIP_TRY(states.ensure(2 * sbytes, cx.stream), "adjoint states");
    struct Release {
        DevBuf &b;
        hipStream_t s;
        ~Release() {
            (void)hipStreamSynchronize(s);
            b.release();
        }
    } release{states, cx.stream};
    void *psi = states.p;
    void *lam = static_cast<unsigned char *>(states.p) + sbytes;

    std::vector<Gate> g = load_gates(c);
    // Forward sweep
    HIP_TRY(launch_zero_state(c64, psi, dim, cx.stream), "state init");
    PlanConfig fcfg = plan_config(n, c64, QG_FUSE_GREEDY);
    Program fwd = build_program(g, fuse(g, fcfg), fcfg);
    st = run_program(cx, c64, fwd, psi, nullptr, nullptr);
    if (st != QG_OK) return st;
    // f and lambda = O psi
    std::vector<uint64_t> mk(zmask, zmask + n_terms);
    std::vector<double> cf(coeff, coeff + n_terms);
    Pack pk;
    const size_t mo = pk.add(mk);
    const size_t co = pk.add(cf);
    unsigned char *dev = nullptr;
    DevBuf obs;
    struct Release2 {
        DevBuf &b;
        hipStream_t s;
        ~Release2() {
            (void)hipStreamSynchronize(s);
            b.release();
        }
    } release2{obs, cx.stream};
    {
        HIP_TRY(cx.push(pk, &dev), "upload observable");
        HIP_TRY(obs.ensure(pk.bytes.size() + 1, cx.stream), "observable buffer");
        HIP_TRY(hipMemcpyAsync(obs.p, dev, pk.bytes.size(), hipMemcpyDeviceToDevice, cx.stream), "copy observable");
        dev = static_cast<unsigned char *>(obs.p);
    }
    const uint64_t *dmask = reinterpret_cast<const uint64_t *>(dev + mo);
    const double *dcoef = reinterpret_cast<const double *>(dev + co);
    if (n_terms > 0) {
        HIP_TRY(cx.work.ensure(expval_partials(dim, n_terms) * sizeof(double), cx.stream), "expval scratch");
        HIP_TRY(launch_expval(c64, psi, dim, dmask, dcoef, n_terms, static_cast<double *>(cx.work.p), nullptr,
                              out_value, cx.stream),
                "expval kernels");
    } else {
        HIP_TRY(hipMemsetAsync(out_value, 0, sizeof(double), cx.stream), "clear value");
    }
    HIP_TRY(launch_apply_observable(c64, psi, lam, dim, dmask, dcoef, n_terms, cx.stream), "observable");
    // Reverse sweep with gradient partials
    PlanConfig rcfg = fcfg;
    rcfg.reverse = true;
    std::vector<Gate> rg = execution_order(g, true);
    Program rev = build_program(rg, fuse(rg, rcfg), rcfg);
    const int n_rows = (int)rev.grad_row_slot.size();
    HIP_TRY(cx.work2.ensure((n_rows + 1) * sizeof(double) + (n_rows + 1) * sizeof(int32_t) + 512, cx.stream),
            "gradient rows");
    double *rows = static_cast<double *>(cx.work2.p);
    int32_t *dslot = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(cx.work2.p) +
                                                  ((n_rows + 1) * sizeof(double) + 255) / 256 * 256);
    if (n_rows > 0)
        HIP_TRY(hipMemcpyAsync(dslot, rev.grad_row_slot.data(), n_rows * sizeof(int32_t), hipMemcpyHostToDevice,
                               cx.stream),
                "upload gradient slots");
    st = run_program(cx, c64, rev, psi, lam, rows);
    if (st != QG_OK) return st;
    HIP_TRY(launch_grad_slots(rows, dslot, n_rows, out_grad, n_params, cx.stream), "gradient slots");
    HIP_TRY(hipStreamSynchronize(cx.stream), "adjoint sweep");
    return QG_OK;
}

qg_status qg_batch_expval(const qg_circuit *circs, int n_circ, qg_dtype dtype, int obs_kind, const int64_t *obs_off,
                          const uint64_t *zmask, const double *coeff, void *hip_stream, double *out) {
    (void)circs; (void)n_circ; (void)dtype; (void)obs_kind; (void)obs_off; (void)zmask; (void)coeff;
    (void)hip_stream; (void)out;
    return fail(QG_EUNSUPPORTED, "qg_batch_expval is not built yet");
}

}  // extern "C"
