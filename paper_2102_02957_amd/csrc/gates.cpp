// FP64 gate matrices, built on the host once per plan.
//
// u3 follows Eq. (1) of the paper (second angle = OpenQASM's phi); CNOT follows
// Eq. (2), whose "higher bit is the control" order is (target, control) in the
// local-index rule used here (local index = sum_j bit(q[j]) << j), so the
// matrix below, in this library's (control, target) order, swaps rows 1 and 3.
// Every other gate is its textbook definition.
#include <cmath>

#include "qsv_internal.hpp"

namespace qsv {

bool gate_arity(int kind, int &nq) {
    switch (kind) {
        case QSV_H: case QSV_X: case QSV_Y: case QSV_Z: case QSV_S: case QSV_SDG:
        case QSV_T: case QSV_TDG: case QSV_RX: case QSV_RY: case QSV_RZ: case QSV_P:
        case QSV_U3:
            nq = 1;
            return true;
        case QSV_CX: case QSV_CZ: case QSV_CP: case QSV_SWAP:
            nq = 2;
            return true;
        case QSV_UNITARY:
            nq = -1;  // caller-provided
            return true;
        default:
            return false;
    }
}

bool kind_is_diagonal(int kind) {
    switch (kind) {
        case QSV_Z: case QSV_S: case QSV_SDG: case QSV_T: case QSV_TDG:
        case QSV_RZ: case QSV_P: case QSV_CZ: case QSV_CP:
            return true;
        default:
            return false;
    }
}

static cd expi(double a) { return cd(std::cos(a), std::sin(a)); }

bool named_matrix(int kind, const double *p, std::vector<cd> &m) {
    const double h = 1.0 / std::sqrt(2.0);
    const cd I(0.0, 1.0);
    switch (kind) {
        case QSV_H: m = {h, h, h, -h}; return true;
        case QSV_X: m = {0.0, 1.0, 1.0, 0.0}; return true;
        case QSV_Y: m = {0.0, -I, I, 0.0}; return true;
        case QSV_Z: m = {1.0, 0.0, 0.0, -1.0}; return true;
        case QSV_S: m = {1.0, 0.0, 0.0, I}; return true;
        case QSV_SDG: m = {1.0, 0.0, 0.0, -I}; return true;
        case QSV_T: m = {1.0, 0.0, 0.0, expi(M_PI / 4)}; return true;
        case QSV_TDG: m = {1.0, 0.0, 0.0, expi(-M_PI / 4)}; return true;
        case QSV_RX: {
            double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
            m = {c, -I * s, -I * s, c};
            return true;
        }
        case QSV_RY: {
            double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
            m = {c, -s, s, c};
            return true;
        }
        case QSV_RZ: m = {expi(-p[0] / 2), 0.0, 0.0, expi(p[0] / 2)}; return true;
        case QSV_P: m = {1.0, 0.0, 0.0, expi(p[0])}; return true;
        case QSV_U3: {
            // Eq. (1): [[cos, -e^{i lam} sin], [e^{i phi} sin, e^{i(phi+lam)} cos]] at theta/2
            double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
            m = {c, -expi(p[2]) * s, expi(p[1]) * s, expi(p[1] + p[2]) * c};
            return true;
        }
        case QSV_CX: {
            // (control, target) order: local index = x_c + 2 x_t; x_c = 1 rows 1 and 3 swap.
            m.assign(16, 0.0);
            m[0 * 4 + 0] = 1.0;
            m[2 * 4 + 2] = 1.0;
            m[1 * 4 + 3] = 1.0;
            m[3 * 4 + 1] = 1.0;
            return true;
        }
        case QSV_CZ:
            m.assign(16, 0.0);
            m[0] = m[5] = m[10] = 1.0;
            m[15] = -1.0;
            return true;
        case QSV_CP:
            m.assign(16, 0.0);
            m[0] = m[5] = m[10] = 1.0;
            m[15] = expi(p[0]);
            return true;
        case QSV_SWAP:
            m.assign(16, 0.0);
            m[0] = m[15] = 1.0;
            m[1 * 4 + 2] = m[2 * 4 + 1] = 1.0;
            return true;
        default:
            return false;
    }
}

}  // namespace qsv
