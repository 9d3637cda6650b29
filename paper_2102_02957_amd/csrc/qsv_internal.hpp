// Internal data structures shared by the host planner and the HIP runtime.
//
// A plan is the paper's transpiled op list (Sec. IV-A) lowered one more level:
// every section (begin_blocking .. end_blocking) holds the chunk's physical bit
// set and a list of register "phases".  Inside a section one GPU workgroup owns
// one chunk of 2^c amplitudes; each thread keeps 2^r of them in registers.  A
// phase fixes which c-r chunk qubits are spread over the threads and which r
// sit in each thread's registers; gates whose qubits are register qubits are
// applied without communication, and a phase change is an LDS transposition.
// This is the cache-blocking idea of Sec. IV-A applied once more, one level
// down (registers as the cache of the LDS-held chunk).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qsv.h"

namespace qsv {

using cd = std::complex<double>;

// The section and adjoint kernels transpose one real component at a time
// (real parts, then imaginary parts), so their transposition buffer holds 2^c
// components: half the chunk's bytes.  (The batch kernel moves whole
// amplitudes and sizes its buffer itself.)
inline size_t transpose_lds_bytes(int c, size_t amp_bytes) { return (size_t(1) << c) * (amp_bytes / 2); }

// ---- device-side plan records (plain data, copied to the GPU) -------------

// Bit source of a diagonal gate / CX control, resolved per section:
//   0 .. 31   : data position (0..r-1 register bit, r..c-1 thread-index bit + r)
//   64 + b    : physical bit b of the chunk's base index (non-local qubit)
constexpr uint8_t SRC_GLOBAL = 64;

enum OpType : uint8_t {
    OP_DENSE = 1,   // dense 2^k x 2^k on register positions a[0] < ... < a[k-1]; mats[arg]
    OP_XREG = 2,    // Pauli X on register position a[0]: a register permutation
    OP_CX = 3,      // X on register position a[0] where bit source a[1] is 1
    OP_DIAG = 4,    // diagonal with 2^k entries mats[arg + sum_j bit(a[j]) << j]
    OP_PROT = 5,    // parameterised RX/RY on register position a[0]; (cos, sin) of half the
                    // angle params[arg] precomputed at ptab[2 slot], ptab[2 slot + 1]
    OP_PDIAG = 6,   // parameterised RZ/P on bit source a[0]; its two diagonal entries
                    // precomputed at ptab[2 slot], ptab[2 slot + 1]
};

enum RotKind : uint8_t { ROT_RX = 1, ROT_RY = 2, ROT_RZ = 3, ROT_P = 4 };

struct DevOp {               // 16 bytes
    uint8_t type;
    uint8_t k;
    uint8_t a[5];
    uint8_t rot;
    int32_t arg;             // matrix offset (dense, diag) or parameter index (param ops)
    int32_t slot;            // param ops: index into the per-state parameter table; else -1
};
static_assert(sizeof(DevOp) == 16, "DevOp layout");

struct DevPhase {            // 128 bytes
    uint8_t rd[16];          // data position -> chunk slot at the phase start
    uint8_t wr[16];          // data position -> chunk slot at the phase end
    // The LDS transposition into the next phase, as element-index masks per data
    // position: element index = XOR of the masks of the set position bits.  xw
    // from this phase's wr map, xr from the next phase's rd map, both with the
    // transposition's swizzle applied (its bank-conflict-free layout).
    uint16_t xw[16];
    uint16_t xr[16];
    uint32_t op_begin, op_end;
    uint32_t pad[6];
};
static_assert(sizeof(DevPhase) == 128, "DevPhase layout");

struct DevSection {          // 128 bytes
    uint8_t slot_phys[16];   // chunk slot -> physical bit (ascending)
    uint8_t nl_phys[40];     // i-th bit of the chunk id -> physical bit (ascending)
    uint32_t phase_begin, phase_end;
    uint32_t n_nl;           // number of non-local bits (n - c)
    uint32_t c;              // chunk bits of this section
    uint32_t n_params_used;  // parameterised ops in this section
    uint32_t param_slot;     // first adjoint partial slot of this section
    uint32_t flags;          // SEC_DENSE_ONLY: every op is OP_DENSE
    uint8_t gather_phys[16]; // data position -> physical bit at the section start
    uint8_t scatter_phys[16];// data position -> physical bit at the section end
    uint8_t pad[12];
};
constexpr uint32_t SEC_DENSE_ONLY = 1;
// single-phase section whose scatter sends amplitudes to other threads: without
// a transposition in between, a workgroup barrier must separate every wave's
// gather from any wave's scatter (the update is in place)
constexpr uint32_t SEC_SYNC_SCATTER = 2;
// paired phases: every phase is ops[2p] on register positions (0, 1) and
// ops[2p + 1] on (2, 3), dense 4 x 4 (4 register bits)
constexpr uint32_t SEC_PAIRED = 4;
static_assert(sizeof(DevSection) == 128, "DevSection layout");

// one parameterised op: which parameter drives it and how
struct PSlot {
    int32_t param;
    int32_t rot;             // RotKind
};

// ---- per-gate path records ------------------------------------------------

enum PgKind : uint8_t {
    PG_DENSE = 1,   // dense k-qubit, matrix at mats[arg] (qubits sorted ascending in q[])
    PG_DIAG1 = 2,   // 1q diagonal, both entries (rz):  mats[arg], mats[arg+1]
    PG_PHASE1 = 3,  // 1q diagonal with d0 == 1 (z, s, t, p): only bit=1 half
    PG_CPHASE = 4,  // 2q diag(1,1,1,d): only the 11 quarter (cz, cp)
    PG_X = 5,       // pauli X: swap halves (full pass)
    PG_CX = 6,      // swap (c=1,t=0)<->(c=1,t=1): half pass
    PG_SWAP = 7,    // swap (a=0,b=1)<->(a=1,b=0): half pass
};

struct PgOp {
    uint8_t kind, k;
    uint8_t q[5];
    uint8_t pad;
    int32_t arg;
    int32_t gate;
};

// ---- host plan ------------------------------------------------------------

struct GateRec {
    int kind = 0, nq = 0;
    int q[QSV_MAX_GATE_QUBITS] = {0, 0, 0, 0, 0};
    int param = -1;
    double p[3] = {0, 0, 0};
    std::vector<cd> m;        // 2^nq x 2^nq, row-major, gate's own qubit order (param gates: empty)
    bool diagonal = false;    // matrix is diagonal (phase gate)
    bool is_swap = false;     // relabelling gate
    uint64_t qmask = 0;       // every qubit it touches
};

struct HostSection {
    std::vector<int> phys_local;   // ascending physical bits held in the chunk
    std::vector<int> gates;        // circuit gate indices in execution order
    std::vector<std::pair<int, int>> swaps_before;  // materialise mode: chunk_swaps (physical)
    std::vector<int> layout_at;    // logical -> physical at this section
};

struct Plan {
    int n = 0;
    qsv_dtype dtype = QSV_C128;
    qsv_options opt{};
    int c = 0, r = 0;
    int kmax = 1;                           // widest dense in-section op (after fusion)
    int fusion_eff = 0;                     // fusion width actually applied (<= requested)
    std::vector<GateRec> gates;
    std::vector<HostSection> sections;
    std::vector<int> final_perm;                      // logical -> physical after the last section
    std::vector<std::pair<int, int>> restore_swaps;   // materialise mode: back to identity order

    // device tables
    std::vector<DevSection> dsec;
    std::vector<DevPhase> dphase;
    std::vector<DevOp> dops;
    std::vector<cd> dmats;                  // matrices and diagonal tables (FP64; cast at upload)
    std::vector<PgOp> pg;                   // per-gate path ops
    int64_t n_params = 0;
    int64_t n_param_ops = 0;                // parameterised ops over all sections
    std::vector<PSlot> pslots;              // [n_param_ops]
    std::vector<int32_t> poff, plist;       // CSR: the param ops driven by parameter p
    double flops = 0.0;
    int64_t chunk_swaps = 0;
    uint64_t uid = 0;                       // identity for device-side caching
};

// plans whose sections keep the chunk in LDS (one phase, op positions = LDS bits)
inline bool lds_resident(const qsv_options &o) {
    return o.section_kernel == QSV_KERNEL_LDS || o.section_kernel == QSV_KERNEL_MFMA;
}

// planner.cpp
qsv_status build_plan(const qsv_options &opt, qsv_dtype dt, int n, const qsv_gate *g, size_t ng,
                      Plan &out, std::string &err);
void default_options(qsv_dtype dt, qsv_options &opt);
// density.cpp: the 2n-qubit gate list of an n-qubit circuit's density-matrix
// evolution (channels become dense gates on (Q, Q + n)); `store` owns matrices
qsv_status density_gates(int n, const qsv_gate *g, size_t ng, std::vector<qsv_gate> &out,
                         std::vector<std::vector<double>> &store, std::string &err);
// gates.cpp
bool gate_arity(int kind, int &nq);
bool named_matrix(int kind, const double *p, std::vector<cd> &m);
bool kind_is_diagonal(int kind);

void set_error(const std::string &msg);

}  // namespace qsv

// the opaque plan handle of the C ABI
struct qsv_plan {
    qsv::Plan p;
};
