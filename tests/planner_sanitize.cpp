// Host planner under AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure, CPU only).  Built with g++ from the planner's host sources
// (planner.cpp, gates.cpp, density.cpp), it plans many circuits and option
// sets -- valid, invalid and adversarial -- and prints "ok <plans>" when every
// call returned (any sanitizer report aborts the run).  Invalid inputs must
// come back as error statuses, never as a crash.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2102_02957_amd/csrc/qsv_internal.hpp"

namespace {

struct Rng {  // splitmix64
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int below(int m) { return (int)(next() % (uint64_t)m); }
    double unit() { return (double)(next() >> 11) * 0x1.0p-53; }
};

const int ONE_Q[] = {QSV_H, QSV_X, QSV_Y, QSV_Z, QSV_S, QSV_SDG, QSV_T, QSV_TDG,
                     QSV_RX, QSV_RY, QSV_RZ, QSV_P, QSV_U3};
const int TWO_Q[] = {QSV_CX, QSV_CZ, QSV_CP, QSV_SWAP};

struct Circuit {
    std::vector<qsv_gate> g;
    std::vector<std::vector<double>> store;
};

void pick_qubits(Rng &r, int n, int k, int32_t *q) {
    for (int j = 0; j < k; ++j) {
        int v;
        bool dup;
        do {
            v = r.below(n);
            dup = false;
            for (int t = 0; t < j; ++t) dup = dup || q[t] == v;
        } while (dup);
        q[j] = v;
    }
}

Circuit random_circuit(Rng &r, int n, int ng, int maxk, bool params) {
    Circuit c;
    c.store.reserve(ng);
    for (int i = 0; i < ng; ++i) {
        qsv_gate g;
        std::memset(&g, 0, sizeof(g));
        g.param = -1;
        const int pick = r.below(10);
        if (pick < 5 || n < 2) {
            g.kind = ONE_Q[r.below(13)];
            g.nq = 1;
        } else if (pick < 8) {
            g.kind = TWO_Q[r.below(4)];
            g.nq = 2;
        } else {
            g.kind = QSV_UNITARY;
            g.nq = 1 + r.below(std::min(maxk, n));
            c.store.emplace_back(size_t(2) << (2 * g.nq));
            for (double &v : c.store.back()) v = r.unit() - 0.5;
            g.m = c.store.back().data();
        }
        pick_qubits(r, n, g.nq, g.q);
        for (double &p : g.p) p = 6.283185307179586 * r.unit();
        if (params && (g.kind == QSV_RX || g.kind == QSV_RY || g.kind == QSV_RZ || g.kind == QSV_P))
            g.param = r.below(8);
        c.g.push_back(g);
    }
    return c;
}

int plans = 0, failures = 0;

qsv_status plan(const qsv_options &o, qsv_dtype dt, int n, const std::vector<qsv_gate> &g) {
    qsv::Plan P;
    std::string err;
    const qsv_status st = qsv::build_plan(o, dt, n, g.data(), g.size(), P, err);
    ++plans;
    return st;
}

void expect_error(const char *what, const qsv_options &o, int n, const std::vector<qsv_gate> &g) {
    if (plan(o, QSV_C128, n, g) == QSV_OK) {
        std::printf("FAIL accepted invalid input: %s\n", what);
        ++failures;
    }
}

}  // namespace

int main() {
    Rng r{12345};
    // valid circuits over the option space (statuses other than OK are allowed where a
    // shape is unsupported; the point is that every call returns)
    const int ns[] = {1, 2, 3, 5, 8, 11, 14, 20, 26};
    for (int n : ns) {
        for (int rep = 0; rep < 3; ++rep) {
            const bool params = rep == 2;
            Circuit c = random_circuit(r, n, 6 * n + 5, 3, params);
            for (int kernel = 0; kernel <= 3; ++kernel)
                for (int planner = 0; planner <= 3; ++planner) {
                    if (planner == 3 && (n > 12 || c.g.size() > 64)) continue;
                    for (int dt = 1; dt <= 2; ++dt) {
                        qsv_options o;
                        qsv::default_options((qsv_dtype)dt, o);
                        o.section_kernel = kernel;
                        o.planner = planner;
                        o.chunk_bits = 1 + r.below(13);
                        o.register_bits = 1 + r.below(5);
                        o.pinned_low_bits = r.below(5) - 1;
                        o.fusion_max_qubits = r.below(6);
                        o.swap_mode = planner >= 2 ? QSV_SWAP_REMAP : r.below(2);
                        o.diag_free = r.below(2);
                        o.io_phases = r.below(2);
                        (void)plan(o, (qsv_dtype)dt, n, c.g);
                    }
                }
        }
    }
    // density-matrix lowering of a noisy circuit, then its 2n-qubit plan
    {
        const int n = 6;
        Circuit c = random_circuit(r, n, 30, 2, false);
        for (int q = 0; q < n; ++q) {
            qsv_gate g;
            std::memset(&g, 0, sizeof(g));
            g.param = -1;
            g.kind = (q % 3 == 0) ? QSV_AMP_DAMP : (q % 3 == 1) ? QSV_PHASE_DAMP : QSV_DEPOLARIZE;
            g.nq = 1;
            g.q[0] = q;
            g.p[0] = 0.05;
            c.g.push_back(g);
        }
        std::vector<qsv_gate> dg;
        std::vector<std::vector<double>> store;
        std::string err;
        if (qsv::density_gates(n, c.g.data(), c.g.size(), dg, store, err) != QSV_OK) {
            std::printf("FAIL density lowering: %s\n", err.c_str());
            ++failures;
        } else {
            qsv_options o;
            qsv::default_options(QSV_C128, o);
            o.chunk_bits = 8;
            if (plan(o, QSV_C128, 2 * n, dg) != QSV_OK) {
                std::printf("FAIL density plan\n");
                ++failures;
            }
        }
    }
    // invalid inputs come back as errors
    {
        qsv_options o;
        qsv::default_options(QSV_C128, o);
        o.chunk_bits = 4;
        qsv_gate g;
        std::memset(&g, 0, sizeof(g));
        g.param = -1;
        g.kind = QSV_CX;
        g.nq = 2;
        g.q[0] = 1;
        g.q[1] = 1;
        expect_error("duplicate qubits", o, 6, {g});
        g.q[1] = 6;
        expect_error("qubit out of range", o, 6, {g});
        g.q[1] = 2;
        g.nq = 3;
        expect_error("arity mismatch", o, 6, {g});
        g.nq = 1;
        g.kind = QSV_RX;
        g.p[0] = std::nan("");
        expect_error("NaN angle", o, 6, {g});
        g.kind = 999;
        g.p[0] = 0.0;
        expect_error("unknown kind", o, 6, {g});
        g.kind = QSV_UNITARY;
        g.nq = 2;
        g.m = nullptr;
        expect_error("missing matrix", o, 6, {g});
        g.kind = QSV_H;
        g.nq = 1;
        expect_error("n = 0", o, 0, {g});
        expect_error("n = 35", o, 35, {g});
        qsv_options bad = o;
        bad.chunk_bits = 0;
        bad.fusion_max_qubits = 9;
        expect_error("fusion width 9", bad, 6, {g});
        bad = o;
        bad.section_kernel = 7;
        expect_error("unknown section kernel", bad, 6, {g});
        bad = o;
        bad.chunk_bits = 1;
        expect_error("grid beyond the hardware limit", bad, 34, {g});
    }
    // adversarial circuits: every gate on one pair, long SWAP chains, wide gates only
    {
        qsv_options o;
        qsv::default_options(QSV_C64, o);
        std::vector<qsv_gate> same, swaps;
        for (int i = 0; i < 3000; ++i) {
            qsv_gate g;
            std::memset(&g, 0, sizeof(g));
            g.param = -1;
            g.kind = (i & 1) ? QSV_CX : QSV_H;
            g.nq = (i & 1) ? 2 : 1;
            g.q[0] = 0;
            g.q[1] = 1;
            same.push_back(g);
            g.kind = QSV_SWAP;
            g.nq = 2;
            g.q[0] = i % 24;
            g.q[1] = (i * 7 + 5) % 24 == i % 24 ? (i % 24 + 1) % 24 : (i * 7 + 5) % 24;
            swaps.push_back(g);
        }
        if (plan(o, QSV_C64, 24, same) != QSV_OK || plan(o, QSV_C64, 24, swaps) != QSV_OK) {
            std::printf("FAIL adversarial circuits\n");
            ++failures;
        }
        Circuit wide = random_circuit(r, 16, 200, 5, false);
        o.fusion_max_qubits = 5;
        o.section_kernel = QSV_KERNEL_MFMA;
        o.chunk_bits = 12;
        (void)plan(o, QSV_C64, 16, wide.g);
    }
    if (failures) return 1;
    std::printf("ok %d\n", plans);
    return 0;
}
