// C ABI: plans, contexts, and the drivers of the blocked and per-gate paths.
//
// qsv_apply_circuit in blocked mode walks the plan like the chunk update loop
// of Sec. IV-C: a chunk_swap group (materialise mode only) is one permutation
// pass; a section (begin_blocking .. end_blocking) is one launch over all
// chunks; in remap mode chunk_swaps cost nothing because the next section
// simply gathers its chunk from other bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "device.hpp"
#include "qsv_internal.hpp"

struct qsv_plan {
    qsv::Plan p;
};

namespace qsv {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

static qsv_status hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return QSV_E_HIP;
}

struct DevPlanBuf {
    uint64_t uid = 0;
    void *block = nullptr;       // one allocation holding every table
    DevPlanView view{};
};

struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> pool;
    double total_ms = 0.0;
    int64_t launches = 0;
};

}  // namespace qsv

struct qsv_ctx {
    int device = 0;
    qsv_dtype dtype = QSV_C128;
    std::list<qsv::DevPlanBuf> plans;      // most recent first
    double *partials = nullptr;
    size_t partials_bytes = 0;
    qsv_zterm *terms = nullptr;
    size_t terms_cap = 0;
    bool timing = false;
    qsv::Timer timers[2];
    std::mutex mu;
};

using namespace qsv;

namespace {

size_t amp_bytes(qsv_dtype dt) { return dt == QSV_C128 ? 16 : 8; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

qsv_status upload_plan(qsv_ctx *ctx, const Plan &P, const DevPlanView **out) {
    for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it) {
        if (it->uid == P.uid) {
            ctx->plans.splice(ctx->plans.begin(), ctx->plans, it);
            *out = &ctx->plans.front().view;
            return QSV_OK;
        }
    }
    const size_t es = amp_bytes(ctx->dtype);
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t o_sec = 0;
    size_t o_ph = align(o_sec + P.dsec.size() * sizeof(DevSection));
    size_t o_op = align(o_ph + P.dphase.size() * sizeof(DevPhase));
    size_t o_m = align(o_op + P.dops.size() * sizeof(DevOp));
    size_t o_pg = align(o_m + P.dmats.size() * es);
    size_t total = align(o_pg + P.pg.size() * sizeof(PgOp)) + 256;
    std::vector<unsigned char> host(total, 0);
    std::memcpy(host.data() + o_sec, P.dsec.data(), P.dsec.size() * sizeof(DevSection));
    std::memcpy(host.data() + o_ph, P.dphase.data(), P.dphase.size() * sizeof(DevPhase));
    std::memcpy(host.data() + o_op, P.dops.data(), P.dops.size() * sizeof(DevOp));
    for (size_t i = 0; i < P.dmats.size(); ++i) {
        if (ctx->dtype == QSV_C128) {
            double v[2] = {P.dmats[i].real(), P.dmats[i].imag()};
            std::memcpy(host.data() + o_m + i * es, v, es);
        } else {
            float v[2] = {(float)P.dmats[i].real(), (float)P.dmats[i].imag()};
            std::memcpy(host.data() + o_m + i * es, v, es);
        }
    }
    std::memcpy(host.data() + o_pg, P.pg.data(), P.pg.size() * sizeof(PgOp));
    DevPlanBuf b;
    b.uid = P.uid;
    hipError_t e = hipMalloc(&b.block, total);
    if (e != hipSuccess) {
        set_error(std::string("plan table allocation: ") + hipGetErrorString(e));
        return QSV_E_NOMEM;
    }
    e = hipMemcpy(b.block, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(b.block);
        return hip_fail(e, "plan table upload");
    }
    unsigned char *base = (unsigned char *)b.block;
    b.view.secs = (const DevSection *)(base + o_sec);
    b.view.phases = (const DevPhase *)(base + o_ph);
    b.view.ops = (const DevOp *)(base + o_op);
    b.view.mats = base + o_m;
    b.view.pg = (const PgOp *)(base + o_pg);
    ctx->plans.push_front(b);
    while (ctx->plans.size() > 64) {
        (void)hipFree(ctx->plans.back().block);
        ctx->plans.pop_back();
    }
    *out = &ctx->plans.front().view;
    return QSV_OK;
}

qsv_status ensure_partials(qsv_ctx *ctx, size_t bytes) {
    if (ctx->partials_bytes >= bytes) return QSV_OK;
    if (ctx->partials) (void)hipFree(ctx->partials);
    ctx->partials = nullptr;
    ctx->partials_bytes = 0;
    hipError_t e = hipMalloc((void **)&ctx->partials, bytes);
    if (e != hipSuccess) {
        set_error(std::string("reduction workspace: ") + hipGetErrorString(e));
        return QSV_E_NOMEM;
    }
    ctx->partials_bytes = bytes;
    return QSV_OK;
}

hipEvent_t take_event(Timer &t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// launch wrapper that optionally brackets the launch with events
template <typename F>
qsv_status timed(qsv_ctx *ctx, int which, hipStream_t s, F &&launch, const char *what) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        e0 = take_event(ctx->timers[which]);
        e1 = take_event(ctx->timers[which]);
        (void)hipEventRecord(e0, s);
    }
    hipError_t e = launch();
    if (e != hipSuccess) return hip_fail(e, what);
    if (ctx->timing) {
        (void)hipEventRecord(e1, s);
        ctx->timers[which].pending.push_back({e0, e1});
    }
    return QSV_OK;
}

qsv_status check_state(qsv_ctx *ctx, const void *state, int n) {
    if (!ctx) {
        set_error("context is NULL");
        return QSV_E_INVALID;
    }
    if (!state) {
        set_error("state pointer is NULL");
        return QSV_E_INVALID;
    }
    if (n < 1 || n > QSV_MAX_QUBITS) {
        set_error("n out of range");
        return QSV_E_INVALID;
    }
    if (((uintptr_t)state) % 16 != 0) {
        set_error("state must be at least 16-byte aligned");
        return QSV_E_INVALID;
    }
    return QSV_OK;
}

size_t section_lds(const Plan &P, int s) {
    const DevSection &S = P.dsec[s];
    if (S.phase_end - S.phase_begin <= 1) return 0;
    return (size_t(1) << S.c) * amp_bytes(P.dtype);
}

qsv_status run_sections(qsv_ctx *ctx, const Plan &P, const DevPlanView &pv, void *state, int n,
                        int batch, int64_t s0, int64_t s1, const double *params, hipStream_t s) {
    const bool materialise = P.opt.swap_mode == QSV_SWAP_MATERIALIZE;
    for (int64_t si = s0; si < s1; ++si) {
        const HostSection &H = P.sections[si];
        if (materialise && !H.swaps_before.empty()) {
            std::vector<uint8_t> a, b;
            for (auto &pr : H.swaps_before) {
                a.push_back((uint8_t)pr.first);
                b.push_back((uint8_t)pr.second);
            }
            for (int bb = 0; bb < batch; ++bb) {
                void *st = (char *)state + ((size_t)bb << n) * amp_bytes(P.dtype);
                qsv_status rc = timed(ctx, 0, s, [&] {
                    return launch_swap_bits(P.dtype, st, n, a.data(), b.data(), (int)a.size(), s);
                }, "chunk_swap launch");
                if (rc != QSV_OK) return rc;
            }
        }
        size_t lds = section_lds(P, (int)si);
        qsv_status rc = timed(ctx, 0, s, [&] {
            return launch_section(P.dtype, P.r, P.kmax, state, n, batch, pv, (int)si, P.c, lds,
                                  params, (int)P.n_params, s);
        }, "section launch");
        if (rc != QSV_OK) return rc;
    }
    if (materialise && s1 == (int64_t)P.sections.size() && !P.restore_swaps.empty()) {
        // output in the original qubit order (Fig. "chunk_swap" case (b)): one pass per swap
        for (auto &pr : P.restore_swaps) {
            uint8_t a = (uint8_t)pr.first, b = (uint8_t)pr.second;
            for (int bb = 0; bb < batch; ++bb) {
                void *st = (char *)state + ((size_t)bb << n) * amp_bytes(P.dtype);
                qsv_status rc = timed(ctx, 0, s, [&] {
                    return launch_swap_bits(P.dtype, st, n, &a, &b, 1, s);
                }, "restore launch");
                if (rc != QSV_OK) return rc;
            }
        }
    }
    return QSV_OK;
}

}  // namespace

extern "C" {

const char *qsv_last_error(void) { return g_last_error.c_str(); }

qsv_status qsv_default_options(qsv_dtype dt, qsv_options *opt) {
    if (!opt || (dt != QSV_C64 && dt != QSV_C128)) {
        set_error("qsv_default_options: bad argument");
        return QSV_E_INVALID;
    }
    default_options(dt, *opt);
    return QSV_OK;
}

qsv_status qsv_plan_blocks(const qsv_options *opt, qsv_dtype dt, int n, const qsv_gate *g,
                           size_t ng, qsv_plan **plan) {
    if (!plan) {
        set_error("plan out-pointer is NULL");
        return QSV_E_INVALID;
    }
    *plan = nullptr;
    qsv_options o;
    if (opt) o = *opt;
    else default_options(dt, o);
    std::unique_ptr<qsv_plan> p(new (std::nothrow) qsv_plan);
    if (!p) {
        set_error("out of host memory");
        return QSV_E_NOMEM;
    }
    std::string err;
    qsv_status rc;
    try {
        rc = build_plan(o, dt, n, g, ng, p->p, err);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory while planning");
        return QSV_E_NOMEM;
    }
    if (rc != QSV_OK) {
        set_error(err);
        return rc;
    }
    *plan = p.release();
    return QSV_OK;
}

void qsv_plan_destroy(qsv_plan *plan) { delete plan; }

qsv_status qsv_plan_get_stats(const qsv_plan *plan, qsv_plan_stats *out) {
    if (!plan || !out) {
        set_error("qsv_plan_get_stats: NULL argument");
        return QSV_E_INVALID;
    }
    const Plan &P = plan->p;
    std::memset(out, 0, sizeof(*out));
    out->n = P.n;
    out->dtype = P.dtype;
    out->chunk_bits = P.c;
    out->register_bits = P.r;
    out->pinned_low_bits = P.opt.pinned_low_bits;
    out->fusion_max_qubits = P.opt.fusion_max_qubits;
    out->swap_mode = P.opt.swap_mode;
    out->diag_free = P.opt.diag_free;
    out->n_gates = (int64_t)P.gates.size();
    out->n_sections = (int64_t)P.sections.size();
    out->n_chunk_swaps = P.chunk_swaps;
    out->n_phases = (int64_t)P.dphase.size();
    out->n_device_ops = (int64_t)P.dops.size();
    out->n_params = P.n_params;
    out->section_flops = P.flops;
    for (int q = 0; q < P.n && q < 64; ++q) out->final_perm[q] = P.final_perm[q];
    return QSV_OK;
}

qsv_status qsv_plan_export(const qsv_plan *plan, qsv_op *ops, size_t cap, size_t *n_ops) {
    if (!plan || !n_ops || (cap > 0 && !ops)) {
        set_error("qsv_plan_export: NULL argument");
        return QSV_E_INVALID;
    }
    const Plan &P = plan->p;
    size_t k = 0;
    auto put = [&](const qsv_op &o) {
        if (k < cap) ops[k] = o;
        ++k;
    };
    for (const HostSection &S : P.sections) {
        for (auto &pr : S.swaps_before) {
            qsv_op o;
            std::memset(&o, 0, sizeof(o));
            o.tag = QSV_OP_CHUNK_SWAP;
            o.gate = -1;
            o.nq = 2;
            o.q[0] = pr.first;
            o.q[1] = pr.second;
            put(o);
        }
        qsv_op b;
        std::memset(&b, 0, sizeof(b));
        b.tag = QSV_OP_BEGIN;
        b.gate = -1;
        for (int p : S.phys_local) b.mask |= 1ull << p;
        put(b);
        for (int gi : S.gates) {
            const GateRec &g = P.gates[gi];
            qsv_op o;
            std::memset(&o, 0, sizeof(o));
            o.tag = QSV_OP_GATE;
            o.gate = gi;
            o.nq = g.nq;
            for (int j = 0; j < g.nq; ++j) o.q[j] = S.layout_at[g.q[j]];
            put(o);
        }
        qsv_op e;
        std::memset(&e, 0, sizeof(e));
        e.tag = QSV_OP_END;
        e.gate = -1;
        put(e);
    }
    *n_ops = k;
    return QSV_OK;
}

qsv_status qsv_create(qsv_ctx **ctx, int hip_device, qsv_dtype dt) {
    if (!ctx) {
        set_error("ctx out-pointer is NULL");
        return QSV_E_INVALID;
    }
    *ctx = nullptr;
    if (dt != QSV_C64 && dt != QSV_C128) {
        set_error("dtype must be QSV_C64 or QSV_C128");
        return QSV_E_INVALID;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        set_error(std::string("no HIP device available: ") + hipGetErrorString(e));
        return QSV_E_HIP;
    }
    if (hip_device < 0 || hip_device >= count) {
        set_error("hip_device out of range");
        return QSV_E_INVALID;
    }
    qsv_ctx *c = new (std::nothrow) qsv_ctx;
    if (!c) {
        set_error("out of host memory");
        return QSV_E_NOMEM;
    }
    c->device = hip_device;
    c->dtype = dt;
    *ctx = c;
    return QSV_OK;
}

void qsv_destroy(qsv_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &b : ctx->plans) (void)hipFree(b.block);
        if (ctx->partials) (void)hipFree(ctx->partials);
        if (ctx->terms) (void)hipFree(ctx->terms);
        for (auto &t : ctx->timers) {
            for (auto &pr : t.pending) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
            for (auto e : t.pool) (void)hipEventDestroy(e);
        }
    }
    delete ctx;
}

qsv_status qsv_init_basis(qsv_ctx *ctx, void *state, int n, uint64_t basis, void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if (n < 64 && basis >= (1ull << n)) {
        set_error("basis index out of range");
        return QSV_E_INVALID;
    }
    DeviceGuard g(ctx->device);
    hipError_t e = launch_fill_basis(ctx->dtype, state, n, 1, basis, (hipStream_t)stream);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "init launch");
}

static qsv_status check_plan(qsv_ctx *ctx, const qsv_plan *plan, int n) {
    if (!plan) {
        set_error("plan is NULL");
        return QSV_E_INVALID;
    }
    if (plan->p.dtype != ctx->dtype) {
        set_error("plan dtype differs from the context dtype");
        return QSV_E_INVALID;
    }
    if (plan->p.n != n) {
        set_error("plan qubit count differs from n");
        return QSV_E_INVALID;
    }
    return QSV_OK;
}

qsv_status qsv_apply_circuit(qsv_ctx *ctx, const qsv_plan *plan, void *state, int n, int mode,
                             void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_plan(ctx, plan, n)) != QSV_OK) return rc;
    const Plan &P = plan->p;
    if (P.n_params > 0) {
        set_error("plan has parameter-bound gates: use qsv_apply_params");
        return QSV_E_INVALID;
    }
    if (mode != QSV_MODE_BLOCKED && mode != QSV_MODE_PER_GATE) {
        set_error("mode must be QSV_MODE_BLOCKED or QSV_MODE_PER_GATE");
        return QSV_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    const DevPlanView *pv = nullptr;
    if ((rc = upload_plan(ctx, P, &pv)) != QSV_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (mode == QSV_MODE_BLOCKED)
        return run_sections(ctx, P, *pv, state, n, 1, 0, (int64_t)P.sections.size(), nullptr, s);
    for (const PgOp &op : P.pg) {
        rc = timed(ctx, 1, s, [&] {
            return launch_pergate_host(P.dtype, state, n, op, P.dmats.data(), pv->mats, s);
        }, "per-gate launch");
        if (rc != QSV_OK) return rc;
    }
    return QSV_OK;
}

qsv_status qsv_apply_sections(qsv_ctx *ctx, const qsv_plan *plan, void *state, int n, int64_t s0,
                              int64_t s1, void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_plan(ctx, plan, n)) != QSV_OK) return rc;
    const Plan &P = plan->p;
    if (P.opt.swap_mode != QSV_SWAP_REMAP) {
        set_error("section ranges need a remap-mode plan");
        return QSV_E_INVALID;
    }
    if (P.n_params > 0) {
        set_error("plan has parameter-bound gates: use qsv_apply_params");
        return QSV_E_INVALID;
    }
    if (s0 < 0 || s1 < s0 || s1 > (int64_t)P.sections.size()) {
        set_error("section range out of bounds");
        return QSV_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    const DevPlanView *pv = nullptr;
    if ((rc = upload_plan(ctx, P, &pv)) != QSV_OK) return rc;
    return run_sections(ctx, P, *pv, state, n, 1, s0, s1, nullptr, (hipStream_t)stream);
}

qsv_status qsv_apply_params(qsv_ctx *ctx, const qsv_plan *plan, void *states, int n, int batch,
                            const double *params_dev, void *stream) {
    qsv_status rc = check_state(ctx, states, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_plan(ctx, plan, n)) != QSV_OK) return rc;
    const Plan &P = plan->p;
    if (batch < 1 || batch > 65535) {
        set_error("batch must be in [1, 65535]");
        return QSV_E_INVALID;
    }
    if (P.n_params > 0 && !params_dev) {
        set_error("params_dev is NULL");
        return QSV_E_INVALID;
    }
    if (P.opt.swap_mode != QSV_SWAP_REMAP) {
        set_error("parameterised batches need a remap-mode plan");
        return QSV_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    const DevPlanView *pv = nullptr;
    if ((rc = upload_plan(ctx, P, &pv)) != QSV_OK) return rc;
    return run_sections(ctx, P, *pv, states, n, batch, 0, (int64_t)P.sections.size(), params_dev,
                        (hipStream_t)stream);
}

static qsv_status upload_terms(qsv_ctx *ctx, const qsv_zterm *terms, size_t nt, hipStream_t s) {
    if (nt > ctx->terms_cap) {
        if (ctx->terms) (void)hipFree(ctx->terms);
        ctx->terms = nullptr;
        ctx->terms_cap = 0;
        hipError_t e = hipMalloc((void **)&ctx->terms, nt * sizeof(qsv_zterm));
        if (e != hipSuccess) {
            set_error("observable table allocation failed");
            return QSV_E_NOMEM;
        }
        ctx->terms_cap = nt;
    }
    hipError_t e = hipMemcpyAsync(ctx->terms, terms, nt * sizeof(qsv_zterm), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "observable upload");
    e = hipStreamSynchronize(s);  // the host array may go away after return
    return e == hipSuccess ? QSV_OK : hip_fail(e, "observable upload sync");
}

static qsv_status reduce_common(qsv_ctx *ctx, int kind, const void *a, const void *b, int n,
                                int batch, const qsv_zterm *terms, size_t nt, double *out,
                                hipStream_t s) {
    const int nblk = reduce_blocks(n);
    const int W = kind == 1 ? 4 : 1;
    qsv_status rc = ensure_partials(ctx, (size_t)nblk * W * batch * sizeof(double));
    if (rc != QSV_OK) return rc;
    if (kind == 2) {
        if ((rc = upload_terms(ctx, terms, nt, s)) != QSV_OK) return rc;
    }
    hipError_t e = launch_reduce(ctx->dtype, kind, a, b, n, batch, ctx->terms, (int)nt,
                                 ctx->partials, nblk, out, s);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "reduction launch");
}

qsv_status qsv_norm(qsv_ctx *ctx, const void *state, int n, double *out_dev, void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if (!out_dev) {
        set_error("out_dev is NULL");
        return QSV_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    return reduce_common(ctx, 0, state, nullptr, n, 1, nullptr, 0, out_dev, (hipStream_t)stream);
}

qsv_status qsv_overlap(qsv_ctx *ctx, const void *a, const void *b, int n, double *out_dev,
                       void *stream) {
    qsv_status rc = check_state(ctx, a, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_state(ctx, b, n)) != QSV_OK) return rc;
    if (!out_dev) {
        set_error("out_dev is NULL");
        return QSV_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    return reduce_common(ctx, 1, a, b, n, 1, nullptr, 0, out_dev, (hipStream_t)stream);
}

qsv_status qsv_expval(qsv_ctx *ctx, const void *state, int n, const qsv_zterm *terms,
                      size_t n_terms, double *out_dev, void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if (!out_dev || (n_terms > 0 && !terms)) {
        set_error("NULL argument");
        return QSV_E_INVALID;
    }
    if (n_terms == 0 || n_terms > 4096) {
        set_error("n_terms must be in [1, 4096]");
        return QSV_E_INVALID;
    }
    for (size_t t = 0; t < n_terms; ++t)
        if (n < 64 && (terms[t].zmask >> n) != 0) {
            set_error("Z-string acts on a qubit >= n");
            return QSV_E_INVALID;
        }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    return reduce_common(ctx, 2, state, nullptr, n, 1, terms, n_terms, out_dev, (hipStream_t)stream);
}

qsv_status qsv_normalize(qsv_ctx *ctx, void *state, int n, double *norm_out_dev, void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if (!norm_out_dev) {
        set_error("norm_out_dev is NULL");
        return QSV_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    rc = reduce_common(ctx, 0, state, nullptr, n, 1, nullptr, 0, norm_out_dev, s);
    if (rc != QSV_OK) return rc;
    hipError_t e = launch_scale_by_norm(ctx->dtype, state, n, 1, norm_out_dev, s);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "scale launch");
}

qsv_status qsv_copy(qsv_ctx *ctx, void *dst, const void *src, int n, void *stream) {
    qsv_status rc = check_state(ctx, dst, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_state(ctx, src, n)) != QSV_OK) return rc;
    DeviceGuard g(ctx->device);
    hipError_t e = launch_copy(ctx->dtype, dst, src, n, (hipStream_t)stream);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "copy launch");
}

qsv_status qsv_timing_enable(qsv_ctx *ctx, int enable) {
    if (!ctx) {
        set_error("context is NULL");
        return QSV_E_INVALID;
    }
    ctx->timing = enable != 0;
    return QSV_OK;
}

qsv_status qsv_timing_read(qsv_ctx *ctx, int which, double *total_ms, int64_t *launches,
                           int reset) {
    if (!ctx || which < 0 || which > 1) {
        set_error("qsv_timing_read: bad argument");
        return QSV_E_INVALID;
    }
    DeviceGuard g(ctx->device);
    Timer &t = ctx->timers[which];
    for (auto &pr : t.pending) {
        hipError_t e = hipEventSynchronize(pr.second);
        if (e != hipSuccess) return hip_fail(e, "timing event");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return hip_fail(e, "timing elapsed");
        t.total_ms += ms;
        t.launches += 1;
        t.pool.push_back(pr.first);
        t.pool.push_back(pr.second);
    }
    t.pending.clear();
    if (total_ms) *total_ms = t.total_ms;
    if (launches) *launches = t.launches;
    if (reset) {
        t.total_ms = 0.0;
        t.launches = 0;
    }
    return QSV_OK;
}

}  // extern "C"

// placeholders replaced by adjoint.hip / batch.hip
