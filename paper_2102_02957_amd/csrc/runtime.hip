// C ABI: plans, contexts, and the drivers of the blocked and per-gate paths.
//
// qsv_apply_circuit in blocked mode walks the plan like the chunk update loop
// of Sec. IV-C: a chunk_swap group (materialise mode only) is one permutation
// pass; a section (begin_blocking .. end_blocking) is one launch over all
// chunks; in remap mode chunk_swaps cost nothing because the next section
// simply gathers its chunk from other bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "batch.hpp"
#include "device.hpp"
#include "qsv_internal.hpp"


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

struct BatchEntry {
    std::vector<uint64_t> uids, offsets;
    void *states = nullptr;
    double *norms = nullptr;
    BatchLaunch launch;
};

// A device workspace owned by a context.  Calls may come from several streams:
// each use records an event on its stream, and a use from another stream first
// makes its stream wait for that event, so device work on one workspace never
// overlaps.  Under graph capture no event is recorded or waited for (a
// captured context is used from the capturing stream only).
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t last = nullptr;       // recorded after the last use
    hipStream_t last_stream = nullptr;
    bool used = false;
};

// Host-resident states: device slice buffers, copy/compute streams and the
// per-plan tables of sections rewritten for slices (see qsv_apply_host).
constexpr int HOST_NBUF = 3;
struct HostStream {
    void *buf[HOST_NBUF] = {nullptr, nullptr, nullptr};
    size_t buf_bytes = 0;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    hipEvent_t ev_in[HOST_NBUF] = {}, ev_comp[HOST_NBUF] = {}, ev_out[HOST_NBUF] = {};
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
    uint64_t tab_uid = 0;
    int tab_o = -1;
    void *tab = nullptr;             // DevSection[S] rewritten for slices
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
    qsv::Workspace partials;               // reduction / gradient partials (double)
    qsv::Workspace ptab;                   // per-state parameter tables
    qsv::Workspace terms;                  // observable Z-strings (qsv_zterm)
    double *noalloc_partials = nullptr;    // this device's fixed array (qsv_overlap_noalloc)
    size_t noalloc_cap = 0;                // its size in doubles
    bool timing = false;
    qsv::Timer timers[2];
    std::list<qsv::BatchEntry> batches;    // prepared batch launches, most recent first
    qsv::HostStream host;                  // qsv_apply_host resources
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
    size_t o_ps = align(o_pg + P.pg.size() * sizeof(PgOp));
    size_t o_po = align(o_ps + P.pslots.size() * sizeof(PSlot));
    size_t o_pl = align(o_po + P.poff.size() * sizeof(int32_t));
    size_t total = align(o_pl + P.plist.size() * sizeof(int32_t)) + 256;
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
    std::memcpy(host.data() + o_ps, P.pslots.data(), P.pslots.size() * sizeof(PSlot));
    std::memcpy(host.data() + o_po, P.poff.data(), P.poff.size() * sizeof(int32_t));
    std::memcpy(host.data() + o_pl, P.plist.data(), P.plist.size() * sizeof(int32_t));
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
    b.view.pslots = (const PSlot *)(base + o_ps);
    b.view.poff = (const int32_t *)(base + o_po);
    b.view.plist = (const int32_t *)(base + o_pl);
    ctx->plans.push_front(b);
    while (ctx->plans.size() > 64) {
        (void)hipFree(ctx->plans.back().block);
        ctx->plans.pop_back();
    }
    *out = &ctx->plans.front().view;
    return QSV_OK;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// Grow `w` to at least `bytes` and order stream `s` after the workspace's last
// user.  Growing frees the old buffer after its last use has completed.
qsv_status ws_acquire(Workspace &w, size_t bytes, hipStream_t s, const char *what) {
    const bool cap = capturing(s);
    if (w.bytes < bytes) {
        if (cap) {
            set_error(std::string(what) + ": workspace must grow during graph capture "
                      "(call qsv_reserve before capturing)");
            return QSV_E_STATE;
        }
        if (w.used && w.last) {
            hipError_t e = hipEventSynchronize(w.last);
            if (e != hipSuccess) return hip_fail(e, what);
        }
        if (w.ptr) (void)hipFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
        w.used = false;
        hipError_t e = hipMalloc(&w.ptr, bytes);
        if (e != hipSuccess) {
            w.ptr = nullptr;
            set_error(std::string(what) + ": " + hipGetErrorString(e));
            return QSV_E_NOMEM;
        }
        w.bytes = bytes;
    }
    if (!w.last) {
        if (cap) {
            set_error(std::string(what) + ": first use of a workspace during graph capture "
                      "(call qsv_reserve before capturing)");
            return QSV_E_STATE;
        }
        hipError_t e = hipEventCreateWithFlags(&w.last, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    if (!cap && w.used && w.last_stream != s) {
        hipError_t e = hipStreamWaitEvent(s, w.last, 0);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return QSV_OK;
}

// Mark the end of a use of `w` on stream `s` (after the launches that read or write it).
qsv_status ws_release(Workspace &w, hipStream_t s, const char *what) {
    if (capturing(s)) return QSV_OK;
    hipError_t e = hipEventRecord(w.last, s);
    if (e != hipSuccess) return hip_fail(e, what);
    w.last_stream = s;
    w.used = true;
    return QSV_OK;
}

void ws_free(Workspace &w) {
    if (w.ptr) (void)hipFree(w.ptr);
    if (w.last) (void)hipEventDestroy(w.last);
    w = Workspace{};
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
    if (((uintptr_t)state) % 256 != 0) {
        set_error("state must be 256-byte aligned");
        return QSV_E_INVALID;
    }
    return QSV_OK;
}

size_t section_lds(const Plan &P, int s) {
    const DevSection &S = P.dsec[s];
    if (S.phase_end - S.phase_begin <= 1) return 0;
    return transpose_lds_bytes(S.c, amp_bytes(P.dtype));
}

// per-state parameter tables of `batch` states: 2 values per parameterised op
size_t ptab_bytes(const Plan &P, int batch, size_t es) {
    return (size_t)batch * 2 * std::max<int64_t>(1, P.n_param_ops) * es;
}

// adjoint workspace: per-(state, op, chunk) gradient partials + per-(state, op)
// sums, and the energy reduction's partials (doubles)
size_t adjoint_partials_bytes(const Plan &P, int batch) {
    const uint64_t nchunks = 1ull << (P.n - P.c);
    const size_t nslots = (size_t)P.n_param_ops;
    const size_t d = std::max<size_t>((size_t)reduce_blocks(P.n) * batch,
                                      (size_t)batch * nslots * nchunks + (size_t)batch * nslots);
    return d * sizeof(double);
}

// reverse-sweep LDS of section s: transposition area + per-wave partials
size_t adjoint_section_lds(const Plan &P, int s) {
    const size_t waves = ((size_t(1) << (P.dsec[s].c - P.r)) + 63) / 64;
    return section_lds(P, s) + P.dsec[s].n_params_used * waves * sizeof(double);
}


// ptab: per-state parameter tables already filled (or NULL for plans without parameters)
qsv_status run_sections(qsv_ctx *ctx, const Plan &P, const DevPlanView &pv, void *state, int n,
                        int batch, int64_t s0, int64_t s1, const void *ptab, hipStream_t s) {
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
        const size_t lds = section_lds(P, (int)si);
        const bool dense_only = (P.dsec[si].flags & SEC_DENSE_ONLY) != 0;
        qsv_status rc = timed(ctx, 0, s, [&] {
            if (lds_resident(P.opt))
                return launch_section_lds(P.dtype, P.kmax, P.opt.section_kernel == QSV_KERNEL_MFMA,
                                          state, n, batch, pv, (int)si, P.c, s);
            if (P.dsec[si].flags & SEC_PAIRED)
                return launch_section_paired(P.dtype, state, n, batch, pv, (int)si, P.c, lds, s);
            return launch_section(P.dtype, P.r, P.kmax, dense_only, state, n, batch, pv, (int)si,
                                  P.c, lds, ptab, (int)P.n_param_ops, s);
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

static qsv_status check_plan(qsv_ctx *ctx, const qsv_plan *plan, int n);

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

qsv_status qsv_plan_density(const qsv_options *opt, qsv_dtype dt, int n, const qsv_gate *g,
                            size_t ng, qsv_plan **plan) {
    if (!plan) {
        set_error("plan out-pointer is NULL");
        return QSV_E_INVALID;
    }
    *plan = nullptr;
    std::vector<qsv_gate> g2;
    std::vector<std::vector<double>> store;
    std::string err;
    qsv_status rc;
    try {
        rc = density_gates(n, g, ng, g2, store, err);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory while expanding the density circuit");
        return QSV_E_NOMEM;
    }
    if (rc != QSV_OK) {
        set_error("qsv_plan_density: " + err);
        return rc;
    }
    return qsv_plan_blocks(opt, dt, 2 * n, g2.data(), g2.size(), plan);
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
    out->fusion_max_qubits = P.fusion_eff;
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
    double *scr = nullptr;
    size_t scr_cap = 0;
    {
        DeviceGuard g(hip_device);
        e = noalloc_scratch(hip_device, &scr, &scr_cap);
        if (e != hipSuccess) return hip_fail(e, "fixed reduction array lookup");
    }
    qsv_ctx *c = new (std::nothrow) qsv_ctx;
    if (!c) {
        set_error("out of host memory");
        return QSV_E_NOMEM;
    }
    c->noalloc_partials = scr;
    c->noalloc_cap = scr_cap;
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
        for (auto &b : ctx->batches) batch_release(b.launch);
        {
            HostStream &h = ctx->host;
            for (void *b : h.buf)
                if (b) (void)hipFree(b);
            if (h.tab) (void)hipFree(h.tab);
            for (hipStream_t st : {h.s_in, h.s_comp, h.s_out})
                if (st) (void)hipStreamDestroy(st);
            for (int i = 0; i < HOST_NBUF; ++i)
                for (hipEvent_t e : {h.ev_in[i], h.ev_comp[i], h.ev_out[i]})
                    if (e) (void)hipEventDestroy(e);
            if (h.ev_start) (void)hipEventDestroy(h.ev_start);
            if (h.ev_done) (void)hipEventDestroy(h.ev_done);
        }
        ws_free(ctx->partials);
        ws_free(ctx->ptab);
        ws_free(ctx->terms);
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

}  // extern "C"

namespace {

// The o highest physical bits that are not local in section si (0 if fewer).
uint64_t stream_bits(const Plan &P, int si, int o) {
    uint64_t local = 0;
    for (int p : P.sections[si].phys_local) local |= 1ull << p;
    uint64_t m = 0;
    int k = 0;
    for (int b = P.n - 1; b >= 0 && k < o; --b)
        if (!((local >> b) & 1)) {
            m |= 1ull << b;
            ++k;
        }
    return k == o ? m : 0;
}

// position of physical bit p once the bits of O are removed from the index
uint8_t squeeze(uint8_t p, uint64_t O) {
    return (uint8_t)(p - __builtin_popcountll(O & ((1ull << p) - 1)));
}

// A section rewritten for one slice of the state (the amplitudes whose bits in O
// hold fixed values), stored compactly with the O bits removed from the index.
DevSection slice_section(const DevSection &S, uint64_t O) {
    DevSection T = S;
    for (uint32_t i = 0; i < S.c; ++i) {
        T.slot_phys[i] = squeeze(S.slot_phys[i], O);
        T.gather_phys[i] = squeeze(S.gather_phys[i], O);
        T.scatter_phys[i] = squeeze(S.scatter_phys[i], O);
    }
    uint32_t t = 0;
    for (uint32_t i = 0; i < S.n_nl; ++i)
        if (!((O >> S.nl_phys[i]) & 1)) T.nl_phys[t++] = squeeze(S.nl_phys[i], O);
    T.n_nl = t;
    return T;
}

// plans whose ops read non-local qubits (diag_free) cannot run on slices
bool reads_global_bits(const Plan &P) {
    for (const DevOp &op : P.dops) {
        if (op.type == OP_DIAG)
            for (int j = 0; j < op.k; ++j)
                if (op.a[j] >= SRC_GLOBAL) return true;
        if (op.type == OP_CX && op.a[1] >= SRC_GLOBAL) return true;
        if (op.type == OP_PDIAG && op.a[0] >= SRC_GLOBAL) return true;
    }
    return false;
}

qsv_status host_setup(qsv_ctx *ctx, size_t buf_bytes) {
    HostStream &h = ctx->host;
    hipError_t e = hipSuccess;
    if (!h.s_in) {
        for (hipStream_t *st : {&h.s_in, &h.s_comp, &h.s_out})
            if ((e = hipStreamCreateWithFlags(st, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "host streaming: stream creation");
        for (int i = 0; i < HOST_NBUF; ++i)
            for (hipEvent_t *ev : {&h.ev_in[i], &h.ev_comp[i], &h.ev_out[i]})
                if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess)
                    return hip_fail(e, "host streaming: event creation");
        if ((e = hipEventCreateWithFlags(&h.ev_start, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&h.ev_done, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "host streaming: event creation");
    }
    if (h.buf_bytes < buf_bytes) {
        if ((e = hipStreamSynchronize(h.s_out)) != hipSuccess) return hip_fail(e, "host streaming");
        for (void *&b : h.buf) {
            if (b) (void)hipFree(b);
            b = nullptr;
        }
        h.buf_bytes = 0;
        for (void *&b : h.buf)
            if ((e = hipMalloc(&b, buf_bytes)) != hipSuccess) {
                set_error(std::string("host streaming: slice buffer: ") + hipGetErrorString(e));
                return QSV_E_NOMEM;
            }
        h.buf_bytes = buf_bytes;
    }
    return QSV_OK;
}

}  // namespace

extern "C" {

qsv_status qsv_plan_stream_bits(const qsv_plan *plan, int o, uint64_t *mask_out) {
    if (!plan || !mask_out || o < 1 || o > 30) {
        set_error("qsv_plan_stream_bits: bad argument");
        return QSV_E_INVALID;
    }
    const Plan &P = plan->p;
    for (size_t si = 0; si < P.sections.size(); ++si) {
        mask_out[si] = stream_bits(P, (int)si, o);
        if (!mask_out[si] || P.n - o < (int)P.dsec[si].c) {
            set_error("section " + std::to_string(si) + " has fewer than " + std::to_string(o) +
                      " non-local bits to slice on");
            return QSV_E_UNSUPPORTED;
        }
    }
    return QSV_OK;
}

qsv_status qsv_apply_host(qsv_ctx *ctx, const qsv_plan *plan, void *host_state, int n,
                          size_t hbm_budget, int64_t s0, int64_t s1, void *stream) {
    if (!ctx || !plan || !host_state) {
        set_error("qsv_apply_host: NULL argument");
        return QSV_E_INVALID;
    }
    qsv_status rc = check_plan(ctx, plan, n);
    if (rc != QSV_OK) return rc;
    const Plan &P = plan->p;
    if (((uintptr_t)host_state) % 256 != 0) {
        set_error("host state must be 256-byte aligned");
        return QSV_E_INVALID;
    }
    if (P.opt.swap_mode != QSV_SWAP_REMAP || P.n_params > 0) {
        set_error("qsv_apply_host needs a remap-mode plan without bound parameters");
        return QSV_E_UNSUPPORTED;
    }
    if (reads_global_bits(P)) {
        set_error("qsv_apply_host: the plan reads non-local qubits (plan with diag_free = 0)");
        return QSV_E_UNSUPPORTED;
    }
    if (s0 < 0 || s1 < s0 || s1 > (int64_t)P.sections.size()) {
        set_error("section range out of bounds");
        return QSV_E_INVALID;
    }
    const size_t es = amp_bytes(ctx->dtype);
    // slices: 2^o of 2^(n-o) amplitudes; HOST_NBUF of them fit the budget
    int o = 1;
    while (o < n && (size_t)HOST_NBUF * ((size_t(1) << (n - o)) * es) > hbm_budget) ++o;
    std::vector<uint64_t> omask(P.sections.size());
    if ((rc = qsv_plan_stream_bits(plan, o, omask.data())) != QSV_OK) {
        set_error(std::string("qsv_apply_host: HBM budget too small for this plan: ") + qsv_last_error());
        return QSV_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t caller = (hipStream_t)stream;
    const size_t slice_amps = size_t(1) << (n - o);
    if ((rc = host_setup(ctx, slice_amps * es)) != QSV_OK) return rc;
    const DevPlanView *pv = nullptr;
    if ((rc = upload_plan(ctx, P, &pv)) != QSV_OK) return rc;
    HostStream &h = ctx->host;
    hipError_t e = hipSuccess;
    if (h.tab_uid != P.uid || h.tab_o != o) {
        if ((e = hipStreamSynchronize(h.s_comp)) != hipSuccess) return hip_fail(e, "host streaming");
        if (h.tab) (void)hipFree(h.tab);
        h.tab = nullptr;
        h.tab_uid = 0;
        std::vector<DevSection> T(P.dsec.size());
        for (size_t si = 0; si < T.size(); ++si) T[si] = slice_section(P.dsec[si], omask[si]);
        if ((e = hipMalloc(&h.tab, T.size() * sizeof(DevSection))) != hipSuccess) {
            h.tab = nullptr;
            set_error("host streaming: section table allocation");
            return QSV_E_NOMEM;
        }
        if ((e = hipMemcpy(h.tab, T.data(), T.size() * sizeof(DevSection), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "host streaming: section table upload");
        h.tab_uid = P.uid;
        h.tab_o = o;
    }
    DevPlanView sv = *pv;
    sv.secs = (const DevSection *)h.tab;
    // the state is the caller's until its stream reaches this point, and the slice
    // buffers are free once the previous call's copies back have finished
    if ((e = hipEventRecord(h.ev_start, caller)) != hipSuccess ||
        (e = hipStreamWaitEvent(h.s_in, h.ev_start, 0)) != hipSuccess ||
        (e = hipStreamWaitEvent(h.s_in, h.ev_done, 0)) != hipSuccess)
        return hip_fail(e, "host streaming: ordering");
    char *host = (char *)host_state;
    int64_t k_all = 0;
    for (int64_t si = s0; si < s1; ++si) {
        const uint64_t O = omask[si];
        const int minO = __builtin_ctzll(O);
        const size_t run = (size_t(1) << minO) * es;             // bytes per contiguous run
        std::vector<int> upper;                                   // free bits above min O
        for (int b = minO + 1; b < n; ++b)
            if (!((O >> b) & 1)) upper.push_back(b);
        const uint64_t nruns = 1ull << upper.size();
        std::vector<int> obits;
        for (int b = 0; b < n; ++b)
            if ((O >> b) & 1) obits.push_back(b);
        const size_t lds = section_lds(P, (int)si);
        const bool dense_only = (P.dsec[si].flags & SEC_DENSE_ONLY) != 0;
        for (uint64_t k = 0; k < (1ull << o); ++k, ++k_all) {
            const int b = (int)(k_all % HOST_NBUF);
            uint64_t fixed = 0;
            for (int j = 0; j < o; ++j)
                if ((k >> j) & 1) fixed |= 1ull << obits[j];
            // the buffer is free once its previous slice went back to the host
            if (k_all >= HOST_NBUF && (e = hipStreamWaitEvent(h.s_in, h.ev_out[b], 0)) != hipSuccess)
                return hip_fail(e, "host streaming: ordering");
            char *dev = (char *)h.buf[b];
            for (uint64_t j = 0; j < nruns; ++j) {
                uint64_t x = fixed;
                for (size_t t = 0; t < upper.size(); ++t)
                    if ((j >> t) & 1) x |= 1ull << upper[t];
                if ((e = hipMemcpyAsync(dev + j * run, host + x * es, run, hipMemcpyHostToDevice,
                                        h.s_in)) != hipSuccess)
                    return hip_fail(e, "host streaming: copy to device");
            }
            if ((e = hipEventRecord(h.ev_in[b], h.s_in)) != hipSuccess ||
                (e = hipStreamWaitEvent(h.s_comp, h.ev_in[b], 0)) != hipSuccess)
                return hip_fail(e, "host streaming: ordering");
            rc = timed(ctx, 0, h.s_comp, [&] {
                if (lds_resident(P.opt))
                    return launch_section_lds(P.dtype, P.kmax, P.opt.section_kernel == QSV_KERNEL_MFMA,
                                              dev, n - o, 1, sv, (int)si, P.c, h.s_comp);
                if (P.dsec[si].flags & SEC_PAIRED)
                    return launch_section_paired(P.dtype, dev, n - o, 1, sv, (int)si, P.c, lds, h.s_comp);
                return launch_section(P.dtype, P.r, P.kmax, dense_only, dev, n - o, 1, sv, (int)si,
                                      P.c, lds, nullptr, 0, h.s_comp);
            }, "section launch");
            if (rc != QSV_OK) return rc;
            if ((e = hipEventRecord(h.ev_comp[b], h.s_comp)) != hipSuccess ||
                (e = hipStreamWaitEvent(h.s_out, h.ev_comp[b], 0)) != hipSuccess)
                return hip_fail(e, "host streaming: ordering");
            for (uint64_t j = 0; j < nruns; ++j) {
                uint64_t x = fixed;
                for (size_t t = 0; t < upper.size(); ++t)
                    if ((j >> t) & 1) x |= 1ull << upper[t];
                if ((e = hipMemcpyAsync(host + x * es, dev + j * run, run, hipMemcpyDeviceToHost,
                                        h.s_out)) != hipSuccess)
                    return hip_fail(e, "host streaming: copy to host");
            }
            if ((e = hipEventRecord(h.ev_out[b], h.s_out)) != hipSuccess)
                return hip_fail(e, "host streaming: ordering");
        }
        // the next section's slices cut the state along other bits: every slice of
        // this one is back in host memory before the next section reads any
        if ((e = hipEventRecord(h.ev_done, h.s_out)) != hipSuccess ||
            (e = hipStreamWaitEvent(h.s_in, h.ev_done, 0)) != hipSuccess)
            return hip_fail(e, "host streaming: ordering");
    }
    if ((e = hipEventRecord(h.ev_done, h.s_out)) != hipSuccess ||
        (e = hipStreamWaitEvent(caller, h.ev_done, 0)) != hipSuccess)
        return hip_fail(e, "host streaming: ordering");
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
    hipStream_t s = (hipStream_t)stream;
    const size_t es = amp_bytes(ctx->dtype);
    if ((rc = ws_acquire(ctx->ptab, ptab_bytes(P, batch, es), s, "parameter table workspace")) != QSV_OK)
        return rc;
    hipError_t e = launch_param_table(ctx->dtype, params_dev, (int)P.n_params, pv->pslots,
                                      (int)P.n_param_ops, batch, ctx->ptab.ptr, s);
    if (e != hipSuccess) return hip_fail(e, "parameter table launch");
    rc = run_sections(ctx, P, *pv, states, n, batch, 0, (int64_t)P.sections.size(), ctx->ptab.ptr, s);
    qsv_status rr = ws_release(ctx->ptab, s, "parameter table workspace");
    return rc != QSV_OK ? rc : rr;
}

// Observable terms to the context's device table.  The terms travel by value
// in kernel arguments: no host staging, no synchronisation, so the host array
// may go away as soon as the call returns.  The caller holds the terms
// workspace (ws_acquire) around the launches that read it.
static qsv_status upload_terms(qsv_ctx *ctx, const qsv_zterm *terms, size_t nt, hipStream_t s) {
    hipError_t e = launch_store_terms(terms, nt, (qsv_zterm *)ctx->terms.ptr, s);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "observable upload");
}

static qsv_status check_terms(const qsv_zterm *terms, size_t nt, int n) {
    if (nt == 0 || nt > QSV_MAX_TERMS) {
        set_error("n_terms must be in [1, " + std::to_string(QSV_MAX_TERMS) + "]");
        return QSV_E_INVALID;
    }
    for (size_t t = 0; t < nt; ++t) {
        if (n < 64 && (terms[t].zmask >> n) != 0) {
            set_error("Z-string acts on a qubit >= n");
            return QSV_E_INVALID;
        }
        if (!std::isfinite(terms[t].coeff)) {
            set_error("Z-string coefficient is not finite");
            return QSV_E_NUMERIC;
        }
    }
    return QSV_OK;
}

static qsv_status reduce_common(qsv_ctx *ctx, int kind, const void *a, const void *b, int n,
                                int batch, const qsv_zterm *terms, size_t nt, double *out,
                                hipStream_t s) {
    const int nblk = reduce_blocks(n);
    const int W = kind == 1 ? 4 : 1;
    qsv_status rc = ws_acquire(ctx->partials, (size_t)nblk * W * batch * sizeof(double), s,
                               "reduction workspace");
    if (rc != QSV_OK) return rc;
    if (kind == 2) {
        if ((rc = ws_acquire(ctx->terms, QSV_MAX_TERMS * sizeof(qsv_zterm), s, "observable table")) != QSV_OK)
            return rc;
        if ((rc = upload_terms(ctx, terms, nt, s)) != QSV_OK) return rc;
    }
    hipError_t e = launch_reduce(ctx->dtype, kind, a, b, n, batch, (const qsv_zterm *)ctx->terms.ptr,
                                 (int)nt, (double *)ctx->partials.ptr, nblk, out, s);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    if (kind == 2 && (rc = ws_release(ctx->terms, s, "observable table")) != QSV_OK) return rc;
    return ws_release(ctx->partials, s, "reduction workspace");
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

qsv_status qsv_overlap_noalloc(qsv_ctx *ctx, const void *a, const void *b, int n,
                               double *out_dev, void *stream) {
    qsv_status rc = check_state(ctx, a, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_state(ctx, b, n)) != QSV_OK) return rc;
    if (!out_dev) {
        set_error("out_dev is NULL");
        return QSV_E_INVALID;
    }
    const int nblk = reduce_blocks(n);
    if ((size_t)nblk * 4 > ctx->noalloc_cap || !ctx->noalloc_partials) {
        set_error("qsv_overlap_noalloc: " + std::to_string(nblk) + " reduction blocks exceed the "
                  "fixed array of " + std::to_string(ctx->noalloc_cap / 4));
        return QSV_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipError_t e = launch_reduce(ctx->dtype, 1, a, b, n, 1, nullptr, 0, ctx->noalloc_partials,
                                 nblk, out_dev, (hipStream_t)stream);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "reduction launch");
}

qsv_status qsv_expval(qsv_ctx *ctx, const void *state, int n, const qsv_zterm *terms,
                      size_t n_terms, double *out_dev, void *stream) {
    qsv_status rc = check_state(ctx, state, n);
    if (rc != QSV_OK) return rc;
    if (!out_dev || (n_terms > 0 && !terms)) {
        set_error("NULL argument");
        return QSV_E_INVALID;
    }
    if ((rc = check_terms(terms, n_terms, n)) != QSV_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    return reduce_common(ctx, 2, state, nullptr, n, 1, terms, n_terms, out_dev, (hipStream_t)stream);
}

static qsv_status dm_reduce(qsv_ctx *ctx, int kind, const void *rho, int n,
                            const qsv_zterm *terms, size_t nt, double *out_dev, void *stream) {
    if (n < 1 || 2 * n > QSV_MAX_QUBITS) {
        set_error("density matrices need n in [1, " + std::to_string(QSV_MAX_QUBITS / 2) + "]");
        return QSV_E_INVALID;
    }
    qsv_status rc = check_state(ctx, rho, 2 * n);
    if (rc != QSV_OK) return rc;
    if (!out_dev || (nt > 0 && !terms)) {
        set_error("NULL argument");
        return QSV_E_INVALID;
    }
    if (kind == 1 && (rc = check_terms(terms, nt, n)) != QSV_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int nblk = reduce_blocks(n);
    if ((rc = ws_acquire(ctx->partials, (size_t)nblk * sizeof(double), s, "reduction workspace")) != QSV_OK)
        return rc;
    if (kind == 1) {
        if ((rc = ws_acquire(ctx->terms, QSV_MAX_TERMS * sizeof(qsv_zterm), s, "observable table")) != QSV_OK)
            return rc;
        if ((rc = upload_terms(ctx, terms, nt, s)) != QSV_OK) return rc;
    }
    hipError_t e = launch_dm_reduce(ctx->dtype, kind, rho, n, (const qsv_zterm *)ctx->terms.ptr,
                                    (int)nt, (double *)ctx->partials.ptr, nblk, out_dev, s);
    if (e != hipSuccess) return hip_fail(e, "density reduction launch");
    if (kind == 1 && (rc = ws_release(ctx->terms, s, "observable table")) != QSV_OK) return rc;
    return ws_release(ctx->partials, s, "reduction workspace");
}

qsv_status qsv_dm_trace(qsv_ctx *ctx, const void *rho, int n, double *out_dev, void *stream) {
    return dm_reduce(ctx, 0, rho, n, nullptr, 0, out_dev, stream);
}

qsv_status qsv_dm_expval(qsv_ctx *ctx, const void *rho, int n, const qsv_zterm *terms,
                         size_t n_terms, double *out_dev, void *stream) {
    return dm_reduce(ctx, 1, rho, n, terms, n_terms, out_dev, stream);
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

qsv_status qsv_reserve(qsv_ctx *ctx, const qsv_plan *plan, int n, int batch, void *stream) {
    if (!ctx) {
        set_error("context is NULL");
        return QSV_E_INVALID;
    }
    if (plan) n = plan->p.n;
    if (n < 1 || n > QSV_MAX_QUBITS) {
        set_error("n out of range");
        return QSV_E_INVALID;
    }
    if (batch < 1 || batch > 65535) {
        set_error("batch must be in [1, 65535]");
        return QSV_E_INVALID;
    }
    qsv_status rc;
    if (plan && (rc = check_plan(ctx, plan, n)) != QSV_OK) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) {
        set_error("qsv_reserve must be called before graph capture");
        return QSV_E_STATE;
    }
    size_t part = (size_t)reduce_blocks(n) * 4 * batch * sizeof(double);
    size_t pt = 0;
    if (plan) {
        const Plan &P = plan->p;
        const DevPlanView *pv = nullptr;
        if ((rc = upload_plan(ctx, P, &pv)) != QSV_OK) return rc;
        pt = ptab_bytes(P, batch, amp_bytes(ctx->dtype));
        if (P.n_param_ops > 0) part = std::max(part, adjoint_partials_bytes(P, batch));
    }
    struct { Workspace *w; size_t bytes; } need[3] = {
        {&ctx->partials, part}, {&ctx->ptab, std::max<size_t>(pt, 1)},
        {&ctx->terms, QSV_MAX_TERMS * sizeof(qsv_zterm)}};
    for (auto &x : need) {
        if ((rc = ws_acquire(*x.w, x.bytes, s, "qsv_reserve")) != QSV_OK) return rc;
        if ((rc = ws_release(*x.w, s, "qsv_reserve")) != QSV_OK) return rc;
    }
    return QSV_OK;
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

extern "C" qsv_status qsv_batch_run(qsv_ctx *ctx, int count, const qsv_plan *const *plans,
                                    const uint64_t *offsets, void *states, double *norms_dev,
                                    void *stream) {
    if (!ctx || !plans || !offsets || !states || !norms_dev) {
        set_error("qsv_batch_run: NULL argument");
        return QSV_E_INVALID;
    }
    if (count < 1 || count > (1 << 20)) {
        set_error("qsv_batch_run: count must be in [1, 2^20]");
        return QSV_E_INVALID;
    }
    std::vector<const Plan *> ps(count);
    std::vector<uint64_t> uids(count), offs(offsets, offsets + count);
    for (int b = 0; b < count; ++b) {
        if (!plans[b]) {
            set_error("qsv_batch_run: NULL plan");
            return QSV_E_INVALID;
        }
        ps[b] = &plans[b]->p;
        uids[b] = ps[b]->uid;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    BatchEntry *hit = nullptr;
    for (auto it = ctx->batches.begin(); it != ctx->batches.end(); ++it) {
        if (it->uids == uids && it->offsets == offs && it->states == states &&
            it->norms == norms_dev) {
            ctx->batches.splice(ctx->batches.begin(), ctx->batches, it);
            hit = &ctx->batches.front();
            break;
        }
    }
    if (!hit) {
        BatchEntry e;
        e.uids = uids;
        e.offsets = offs;
        e.states = states;
        e.norms = norms_dev;
        std::string err;
        qsv_status rc = batch_prepare(ctx->dtype, count, ps.data(), offsets, states, norms_dev,
                                      e.launch, err);
        if (rc != QSV_OK) {
            batch_release(e.launch);
            set_error("qsv_batch_run: " + err);
            return rc;
        }
        ctx->batches.push_front(std::move(e));
        hit = &ctx->batches.front();
        while (ctx->batches.size() > 8) {
            batch_release(ctx->batches.back().launch);
            ctx->batches.pop_back();
        }
    }
    hipStream_t s = (hipStream_t)stream;
    qsv_status rc = timed(ctx, 0, s, [&] { return batch_replay(hit->launch, s); }, "batch graph launch");
    return rc;
}

// Forward pass, energies, lambda = H psi and the reverse sweep, on workspaces
// already held by the caller.
static qsv_status adjoint_body(qsv_ctx *ctx, const Plan &P, const DevPlanView &pv,
                               const qsv_zterm *terms, size_t n_terms, const double *params_dev,
                               int batch, void *psi_dev, void *lambda_dev, double *energy_dev,
                               double *grad_dev, int nslots, int nblk, uint64_t nchunks,
                               hipStream_t s) {
    const int n = P.n;
    hipError_t e = hipSuccess;
    if (nslots > 0) {
        e = launch_param_table(ctx->dtype, params_dev, (int)P.n_params, pv.pslots, nslots, batch,
                               ctx->ptab.ptr, s);
        if (e != hipSuccess) return hip_fail(e, "parameter table launch");
    }
    // forward
    e = launch_fill_basis(ctx->dtype, psi_dev, n, batch, 0, s);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    qsv_status rc = run_sections(ctx, P, pv, psi_dev, n, batch, 0, (int64_t)P.sections.size(),
                                 ctx->ptab.ptr, s);
    if (rc != QSV_OK) return rc;
    // energies and lambda = H psi
    if ((rc = upload_terms(ctx, terms, n_terms, s)) != QSV_OK) return rc;
    double *partials = (double *)ctx->partials.ptr;
    const qsv_zterm *tdev = (const qsv_zterm *)ctx->terms.ptr;
    e = launch_reduce(ctx->dtype, 2, psi_dev, nullptr, n, batch, tdev, (int)n_terms, partials,
                      nblk, energy_dev, s);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    e = launch_apply_zsum(ctx->dtype, psi_dev, lambda_dev, n, batch, tdev, (int)n_terms, s);
    if (e != hipSuccess) return hip_fail(e, "observable launch");
    if (nslots == 0) return QSV_OK;
    // reverse sweep over the sections
    double *part = partials;
    double *ssum = partials + (size_t)batch * nslots * nchunks;
    for (int64_t si = (int64_t)P.sections.size() - 1; si >= 0; --si) {
        // transposition area + per-wave gradient partials of the section's ops
        const size_t lds = adjoint_section_lds(P, (int)si);
        if (lds > 159 * 1024) {
            set_error("adjoint: section " + std::to_string(si) + " has too many parameterised "
                      "ops for the reverse sweep's LDS (use smaller chunks)");
            return QSV_E_UNSUPPORTED;
        }
        rc = timed(ctx, 0, s, [&] {
            return launch_adjoint_section(P.dtype, P.r, psi_dev, lambda_dev, n, batch, pv, (int)si,
                                          P.c, lds, ctx->ptab.ptr, nslots, part, s);
        }, "adjoint section launch");
        if (rc != QSV_OK) return rc;
    }
    e = launch_grad_reduce(part, nslots, batch, nchunks, ssum, pv.poff, pv.plist,
                           (int)P.n_params, grad_dev, s);
    return e == hipSuccess ? QSV_OK : hip_fail(e, "gradient reduction launch");
}

extern "C" qsv_status qsv_adjoint_grad(qsv_ctx *ctx, const qsv_plan *plan, const qsv_zterm *terms,
                                       size_t n_terms, const double *params_dev, int batch,
                                       void *psi_dev, void *lambda_dev, double *energy_dev,
                                       double *grad_dev, void *stream) {
    if (!ctx || !plan || !terms || !psi_dev || !lambda_dev || !energy_dev) {
        set_error("qsv_adjoint_grad: NULL argument");
        return QSV_E_INVALID;
    }
    const Plan &P = plan->p;
    const int n = P.n;
    qsv_status rc = check_state(ctx, psi_dev, n);
    if (rc != QSV_OK) return rc;
    if ((rc = check_state(ctx, lambda_dev, n)) != QSV_OK) return rc;
    if ((rc = check_plan(ctx, plan, n)) != QSV_OK) return rc;
    if (batch < 1 || batch > 65535) {
        set_error("batch must be in [1, 65535]");
        return QSV_E_INVALID;
    }
    if (P.n_params > 0 && (!params_dev || !grad_dev)) {
        set_error("params_dev / grad_dev is NULL");
        return QSV_E_INVALID;
    }
    if ((rc = check_terms(terms, n_terms, n)) != QSV_OK) return rc;
    if (P.opt.swap_mode != QSV_SWAP_REMAP || P.kmax > 2 || P.c - P.r > 8 ||
        (P.dtype == QSV_C128 && P.r > 4)) {
        set_error("adjoint plans need remap mode, fusion of at most 2 qubits, "
                  "chunk_bits - register_bits <= 8 and register_bits <= 4 (complex128)");
        return QSV_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const DevPlanView *pv = nullptr;
    if ((rc = upload_plan(ctx, P, &pv)) != QSV_OK) return rc;
    const size_t es = amp_bytes(ctx->dtype);
    const int nslots = (int)P.n_param_ops;
    const int nblk = reduce_blocks(n);
    const uint64_t nchunks = 1ull << (n - P.c);
    if ((rc = ws_acquire(ctx->ptab, ptab_bytes(P, batch, es), s, "parameter table workspace")) != QSV_OK)
        return rc;
    if ((rc = ws_acquire(ctx->partials, adjoint_partials_bytes(P, batch), s, "gradient workspace")) != QSV_OK)
        return rc;
    if ((rc = ws_acquire(ctx->terms, QSV_MAX_TERMS * sizeof(qsv_zterm), s, "observable table")) != QSV_OK)
        return rc;
    rc = adjoint_body(ctx, P, *pv, terms, n_terms, params_dev, batch, psi_dev, lambda_dev,
                      energy_dev, grad_dev, nslots, nblk, nchunks, s);
    qsv_status r1 = ws_release(ctx->ptab, s, "parameter table workspace");
    qsv_status r2 = ws_release(ctx->partials, s, "gradient workspace");
    qsv_status r3 = ws_release(ctx->terms, s, "observable table");
    if (rc != QSV_OK) return rc;
    return r1 != QSV_OK ? r1 : r2 != QSV_OK ? r2 : r3;
}
