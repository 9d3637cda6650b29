// Density-matrix plans: the n-qubit density matrix as a 2n-qubit state.
//
// rho[i][j] sits at amplitude index i | (j << n).  The map rho -> K rho K^dagger
// acts on that vector as K on the row qubits and conj(K) on the column qubits:
// (K rho K^dagger)[i][j] = sum_{i', j'} K[i][i'] conj(K[j][j']) rho[i'][j'].
// A gate U therefore becomes two gates (U on Q, conj(U) on Q + n) and a channel
// with Kraus operators {K_m} becomes one dense gate on (Q, Q + n) whose matrix
// is sum_m K_m (x) conj(K_m) in the local-index order (Q bits low).  The rest
// (blocking, sections, kernels) is the state-vector path unchanged: the paper's
// cache blocking needs nothing else (Sec. III-A lists the density-matrix and
// super-operator methods beside the state vector).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "qsv_internal.hpp"

namespace qsv {

namespace {

// Kraus operators of a channel gate (k-qubit, row-major 2^k x 2^k each)
bool kraus_of(const qsv_gate &g, int k, std::vector<std::vector<cd>> &out, std::string &err) {
    out.clear();
    const cd I(0.0, 1.0);
    const double x = g.p[0];
    auto prob = [&](const char *name) {
        if (!(x >= 0.0 && x <= 1.0)) {
            err = std::string(name) + ": probability must be in [0, 1]";
            return false;
        }
        return true;
    };
    switch (g.kind) {
        case QSV_AMP_DAMP:
            if (!prob("amplitude damping")) return false;
            out.push_back({1.0, 0.0, 0.0, std::sqrt(1.0 - x)});
            out.push_back({0.0, std::sqrt(x), 0.0, 0.0});
            return true;
        case QSV_PHASE_DAMP:
            if (!prob("phase damping")) return false;
            out.push_back({1.0, 0.0, 0.0, std::sqrt(1.0 - x)});
            out.push_back({0.0, 0.0, 0.0, std::sqrt(x)});
            return true;
        case QSV_DEPOLARIZE: {
            if (!prob("depolarizing")) return false;
            const double a = std::sqrt(1.0 - x), b = std::sqrt(x / 3.0);
            out.push_back({a, 0.0, 0.0, a});
            out.push_back({0.0, b, b, 0.0});
            out.push_back({0.0, -I * b, I * b, 0.0});
            out.push_back({b, 0.0, 0.0, -b});
            return true;
        }
        case QSV_KRAUS: {
            const int M = g.param;
            if (M < 1 || M > 16 || !g.m) {
                err = "kraus: param must give 1..16 operators and m must be set";
                return false;
            }
            const size_t d = size_t(1) << k;
            for (int mi = 0; mi < M; ++mi) {
                std::vector<cd> K(d * d);
                for (size_t e = 0; e < d * d; ++e) {
                    const double re = g.m[2 * (mi * d * d + e)], im = g.m[2 * (mi * d * d + e) + 1];
                    if (!std::isfinite(re) || !std::isfinite(im)) {
                        err = "kraus: non-finite entry";
                        return false;
                    }
                    K[e] = cd(re, im);
                }
                out.push_back(std::move(K));
            }
            return true;
        }
    }
    err = "not a channel";
    return false;
}

bool is_channel(int kind) {
    return kind == QSV_AMP_DAMP || kind == QSV_PHASE_DAMP || kind == QSV_DEPOLARIZE ||
           kind == QSV_KRAUS;
}

}  // namespace

// Expand an n-qubit circuit with channels into the 2n-qubit gate list of its
// density-matrix evolution.  `store` owns the matrices the returned gates point to.
qsv_status density_gates(int n, const qsv_gate *g, size_t ng, std::vector<qsv_gate> &out,
                         std::vector<std::vector<double>> &store, std::string &err) {
    out.clear();
    store.clear();
    store.reserve(2 * ng);
    if (n < 1 || 2 * n > QSV_MAX_QUBITS) {
        err = "density plans need n in [1, " + std::to_string(QSV_MAX_QUBITS / 2) + "]";
        return QSV_E_INVALID;
    }
    if (ng > 0 && !g) {
        err = "gates pointer is NULL";
        return QSV_E_INVALID;
    }
    auto keep = [&](const std::vector<cd> &m) {
        std::vector<double> v(2 * m.size());
        for (size_t e = 0; e < m.size(); ++e) {
            v[2 * e] = m[e].real();
            v[2 * e + 1] = m[e].imag();
        }
        store.push_back(std::move(v));
        return (const double *)store.back().data();
    };
    for (size_t i = 0; i < ng; ++i) {
        const qsv_gate &s = g[i];
        const std::string at = "gate " + std::to_string(i) + ": ";
        if (is_channel(s.kind)) {
            const int k = s.kind == QSV_KRAUS ? s.nq : 1;
            if (k < 1 || k > 2 || s.nq != k) {
                err = at + "channels act on 1 qubit (QSV_KRAUS: 1 or 2)";
                return QSV_E_INVALID;
            }
            for (int j = 0; j < k; ++j)
                if (s.q[j] < 0 || s.q[j] >= n) {
                    err = at + "qubit out of range";
                    return QSV_E_INVALID;
                }
            if (k == 2 && s.q[0] == s.q[1]) {
                err = at + "repeated qubit";
                return QSV_E_INVALID;
            }
            if (!std::isfinite(s.p[0])) {
                err = at + "non-finite channel parameter";
                return QSV_E_NUMERIC;
            }
            std::vector<std::vector<cd>> K;
            std::string e2;
            if (!kraus_of(s, k, K, e2)) {
                err = at + e2;
                return e2.find("non-finite") != std::string::npos ? QSV_E_NUMERIC : QSV_E_INVALID;
            }
            const size_t d = size_t(1) << k, D = d * d;
            std::vector<cd> S(D * D, cd(0.0, 0.0));
            for (const auto &Km : K)
                for (size_t a = 0; a < d; ++a)
                    for (size_t b = 0; b < d; ++b)
                        for (size_t c = 0; c < d; ++c)
                            for (size_t e = 0; e < d; ++e)
                                S[(a | (b << k)) * D + (c | (e << k))] +=
                                    Km[a * d + c] * std::conj(Km[b * d + e]);
            qsv_gate t;
            std::memset(&t, 0, sizeof(t));
            t.kind = QSV_UNITARY;
            t.nq = 2 * k;
            for (int j = 0; j < k; ++j) {
                t.q[j] = s.q[j];
                t.q[k + j] = s.q[j] + n;
            }
            t.param = -1;
            t.m = keep(S);
            out.push_back(t);
            continue;
        }
        if (s.param >= 0) {
            err = at + "density plans take no bound parameters";
            return QSV_E_UNSUPPORTED;
        }
        int nq = 0;
        if (!gate_arity(s.kind, nq)) {
            err = at + "unknown kind " + std::to_string(s.kind);
            return QSV_E_INVALID;
        }
        if (nq < 0) nq = s.nq;
        if (s.nq != nq || nq < 1 || nq > QSV_MAX_GATE_QUBITS) {
            err = at + "nq does not match its kind";
            return QSV_E_INVALID;
        }
        for (int j = 0; j < nq; ++j)
            if (s.q[j] < 0 || s.q[j] >= n) {
                err = at + "qubit out of range";
                return QSV_E_INVALID;
            }
        // row copy: the gate itself
        out.push_back(s);
        // column copy: the complex conjugate on the shifted qubits
        qsv_gate c = s;
        for (int j = 0; j < nq; ++j) c.q[j] = s.q[j] + n;
        switch (s.kind) {
            case QSV_H: case QSV_X: case QSV_Z: case QSV_RY: case QSV_CX: case QSV_CZ:
            case QSV_SWAP:
                break;  // real matrices
            case QSV_S: c.kind = QSV_SDG; break;
            case QSV_SDG: c.kind = QSV_S; break;
            case QSV_T: c.kind = QSV_TDG; break;
            case QSV_TDG: c.kind = QSV_T; break;
            case QSV_RX: case QSV_RZ: case QSV_P: case QSV_CP:
                c.p[0] = -s.p[0];
                break;
            case QSV_U3:
                c.p[1] = -s.p[1];
                c.p[2] = -s.p[2];
                break;
            default: {  // QSV_Y and explicit matrices: conjugate entry by entry
                std::vector<cd> m;
                if (s.kind == QSV_UNITARY) {
                    if (!s.m) {
                        err = at + "unitary without matrix";
                        return QSV_E_INVALID;
                    }
                    const size_t d = size_t(1) << nq;
                    m.resize(d * d);
                    for (size_t e = 0; e < d * d; ++e) m[e] = cd(s.m[2 * e], s.m[2 * e + 1]);
                } else if (!named_matrix(s.kind, s.p, m)) {
                    err = at + "no matrix for kind";
                    return QSV_E_INVALID;
                }
                for (cd &v : m) v = std::conj(v);
                c.kind = QSV_UNITARY;
                c.m = keep(m);
            }
        }
        out.push_back(c);
    }
    return QSV_OK;
}

}  // namespace qsv
