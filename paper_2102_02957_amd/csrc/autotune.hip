// Autotuner: chunk size, pinned low bits, fusion width and register bits are
// chosen by timing candidate option sets on the caller's own workload.
//
// For each candidate the circuit is planned (host), then run once untimed and
// `reps` times between HIP events on the caller's stream; the candidate with
// the smallest mean wins.  Candidates the planner rejects get +inf.  With a
// section budget m > 0 only the first m sections of a plan run and the time is
// scaled by S / m (S = the candidate's section count): candidates are compared
// on their own section counts without running whole large circuits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "device.hpp"
#include "qsv_internal.hpp"


extern "C" {

qsv_status qsv_autotune(qsv_ctx *ctx, qsv_dtype dt, int n, const qsv_gate *g, size_t ng,
                        const qsv_options *cands, int n_cands, void *state, int reps,
                        int max_sections, int refine, void *stream, int *best, double *ms_out) {
    if (!ctx || !cands || n_cands < 1 || !state || !best || reps < 1) {
        qsv::set_error("qsv_autotune: bad argument");
        return QSV_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        qsv::set_error("qsv_autotune: event creation failed");
        return QSV_E_HIP;
    }
    double best_ms = std::numeric_limits<double>::infinity();
    *best = -1;
    qsv_status rc = QSV_OK;
    std::vector<double> est(n_cands, std::numeric_limits<double>::infinity());
    // time candidate k with a section budget (0 = whole applies)
    auto time_one = [&](int k, int budget) {
        double ms = std::numeric_limits<double>::infinity();
        qsv_plan *plan = nullptr;
        if (qsv_plan_blocks(&cands[k], dt, n, g, ng, &plan) == QSV_OK) {
            const int64_t S = (int64_t)plan->p.sections.size();
            const int max_sections = budget;
            const bool prefix = max_sections > 0 && max_sections < S &&
                                plan->p.opt.swap_mode == QSV_SWAP_REMAP;
            const int64_t m = prefix ? max_sections : S;
            auto run = [&]() {
                return prefix ? qsv_apply_sections(ctx, plan, state, n, 0, m, stream)
                              : qsv_apply_circuit(ctx, plan, state, n, QSV_MODE_BLOCKED, stream);
            };
            qsv_status r = qsv_init_basis(ctx, state, n, 0, stream);
            if (r == QSV_OK) r = run();
            if (r == QSV_OK && hipEventRecord(e0, s) == hipSuccess) {
                for (int t = 0; t < reps && r == QSV_OK; ++t) r = run();
                float f = 0.0f;
                if (r == QSV_OK && hipEventRecord(e1, s) == hipSuccess &&
                    hipEventSynchronize(e1) == hipSuccess &&
                    hipEventElapsedTime(&f, e0, e1) == hipSuccess)
                    ms = f / reps * (double)S / (double)m;
            }
            if (r == QSV_E_HIP) rc = r;
            qsv_plan_destroy(plan);
        }
        return ms;
    };
    for (int k = 0; k < n_cands && rc == QSV_OK; ++k) est[k] = time_one(k, max_sections);
    // refine: the best `refine` estimates are re-timed on whole applies
    std::vector<double> fin = est;
    if (rc == QSV_OK && max_sections > 0 && refine > 0) {
        std::vector<int> order(n_cands);
        for (int k = 0; k < n_cands; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return est[a] < est[b]; });
        for (int j = 0; j < std::min(refine, n_cands) && rc == QSV_OK; ++j)
            if (std::isfinite(est[order[j]])) fin[order[j]] = time_one(order[j], 0);
        // candidates left on estimates cannot win over whole-run times
        for (int k = 0; k < n_cands; ++k) {
            bool refined = false;
            for (int j = 0; j < std::min(refine, n_cands); ++j) refined = refined || order[j] == k;
            if (!refined) fin[k] = std::numeric_limits<double>::infinity();
        }
    }
    for (int k = 0; k < n_cands; ++k) {
        if (ms_out) ms_out[k] = (max_sections > 0 && refine > 0 && std::isinf(fin[k])) ? est[k] : fin[k];
        if (fin[k] < best_ms) {
            best_ms = fin[k];
            *best = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == QSV_OK && *best < 0) {
        qsv::set_error("qsv_autotune: no candidate could be planned and run");
        return QSV_E_INVALID;
    }
    return rc;
}

qsv_status qsv_autotune_batch(qsv_ctx *ctx, qsv_dtype dt, int count, const int *ns,
                              const qsv_gate *const *gates, const size_t *ngs,
                              const uint64_t *offsets, const qsv_options *cands, int n_cands,
                              void *states, double *norms_dev, int reps, void *stream, int *best,
                              double *ms_out) {
    if (!ctx || count < 1 || !ns || !gates || !ngs || !offsets || !cands || n_cands < 1 ||
        !states || !norms_dev || !best || reps < 1) {
        qsv::set_error("qsv_autotune_batch: bad argument");
        return QSV_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        qsv::set_error("qsv_autotune_batch: event creation failed");
        return QSV_E_HIP;
    }
    double best_ms = std::numeric_limits<double>::infinity();
    *best = -1;
    qsv_status rc = QSV_OK;
    for (int k = 0; k < n_cands; ++k) {
        double ms = std::numeric_limits<double>::infinity();
        std::vector<qsv_plan *> plans(count, nullptr);
        bool ok = true;
        for (int b = 0; b < count && ok; ++b)
            ok = qsv_plan_blocks(&cands[k], dt, ns[b], gates[b], ngs[b], &plans[b]) == QSV_OK;
        if (ok) {
            qsv_status r = qsv_batch_run(ctx, count, plans.data(), offsets, states, norms_dev, stream);
            if (r == QSV_OK && hipEventRecord(e0, s) == hipSuccess) {
                for (int t = 0; t < reps && r == QSV_OK; ++t)
                    r = qsv_batch_run(ctx, count, plans.data(), offsets, states, norms_dev, stream);
                float f = 0.0f;
                if (r == QSV_OK && hipEventRecord(e1, s) == hipSuccess &&
                    hipEventSynchronize(e1) == hipSuccess &&
                    hipEventElapsedTime(&f, e0, e1) == hipSuccess)
                    ms = f / reps;
            }
            if (r == QSV_E_HIP) rc = r;
        }
        (void)hipStreamSynchronize(s);
        for (qsv_plan *p : plans) qsv_plan_destroy(p);
        if (ms_out) ms_out[k] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            *best = k;
        }
        if (rc != QSV_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == QSV_OK && *best < 0) {
        qsv::set_error("qsv_autotune_batch: no candidate could be planned and run");
        return QSV_E_INVALID;
    }
    return rc;
}

qsv_status qsv_autotune_adjoint(qsv_ctx *ctx, qsv_dtype dt, int n, const qsv_gate *g, size_t ng,
                                const qsv_zterm *terms, size_t n_terms, const double *params_dev,
                                int batch, void *psi_dev, void *lambda_dev, double *energy_dev,
                                double *grad_dev, const qsv_options *cands, int n_cands, int reps,
                                void *stream, int *best, double *ms_out) {
    if (!ctx || !cands || n_cands < 1 || !best || reps < 1) {
        qsv::set_error("qsv_autotune_adjoint: bad argument");
        return QSV_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        qsv::set_error("qsv_autotune_adjoint: event creation failed");
        return QSV_E_HIP;
    }
    double best_ms = std::numeric_limits<double>::infinity();
    *best = -1;
    qsv_status rc = QSV_OK;
    for (int k = 0; k < n_cands; ++k) {
        double ms = std::numeric_limits<double>::infinity();
        qsv_plan *plan = nullptr;
        if (qsv_plan_blocks(&cands[k], dt, n, g, ng, &plan) == QSV_OK) {
            auto run = [&]() {
                return qsv_adjoint_grad(ctx, plan, terms, n_terms, params_dev, batch, psi_dev,
                                        lambda_dev, energy_dev, grad_dev, stream);
            };
            qsv_status r = run();
            if (r == QSV_OK && hipEventRecord(e0, s) == hipSuccess) {
                for (int t = 0; t < reps && r == QSV_OK; ++t) r = run();
                float f = 0.0f;
                if (r == QSV_OK && hipEventRecord(e1, s) == hipSuccess &&
                    hipEventSynchronize(e1) == hipSuccess &&
                    hipEventElapsedTime(&f, e0, e1) == hipSuccess)
                    ms = f / reps;
            }
            if (r == QSV_E_HIP) rc = r;
            (void)hipStreamSynchronize(s);
            qsv_plan_destroy(plan);
        }
        if (ms_out) ms_out[k] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            *best = k;
        }
        if (rc != QSV_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == QSV_OK && *best < 0) {
        qsv::set_error("qsv_autotune_adjoint: no candidate could be planned and run");
        return QSV_E_INVALID;
    }
    return rc;
}

}  // extern "C"
