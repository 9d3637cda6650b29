// Lowering check (test infrastructure, CPU only): executes a plan's device
// tables -- sections, register phases, ops, matrices, the LDS layouts of the
// transpositions -- with plain complex<double> arithmetic, the way the section
// kernels interpret them, and prints the final state.  The test compares that
// state with the oracle.  It checks the planner's lowering (phase maps, op
// positions, fused matrices, gather/scatter maps, swizzle tables) without a
// GPU; it is not a second oracle (it runs the library's own plan).
//
// stdin:  n dtype(1 = c64, 2 = c128)
//         chunk_bits pinned fusion swap_mode diag_free register_bits io_phases planner kernel
//         ngates, then per gate: kind nq q[0..nq-1] p0 p1 p2 has_matrix [2 * 4^nq reals]
//         2^n amplitudes (re im)
// stdout: 2^n amplitudes (re im), or "ERROR <reason>" and exit status 1
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../paper_2102_02957_amd/csrc/qsv_internal.hpp"

using cdbl = std::complex<double>;
using qsv::DevOp;
using qsv::DevPhase;
using qsv::DevSection;

static int fail(const std::string &why) {
    std::printf("ERROR %s\n", why.c_str());
    return 1;
}

// value of a bit source (data position, or physical bit of the chunk base)
static int src_bit(uint8_t src, uint32_t x, uint64_t base) {
    if (src >= qsv::SRC_GLOBAL) return (int)((base >> (src - qsv::SRC_GLOBAL)) & 1ull);
    return (int)((x >> src) & 1u);
}

// data index under map `from` (position -> slot) to data index under map `to`
static uint32_t remap(uint32_t x, const uint8_t *from, const uint8_t *to, int C) {
    uint32_t z = 0, y = 0;
    for (int p = 0; p < C; ++p)
        if ((x >> p) & 1u) z |= 1u << from[p];
    for (int p = 0; p < C; ++p)
        if ((z >> to[p]) & 1u) y |= 1u << p;
    return y;
}

static bool is_perm(const uint8_t *m, int C) {
    uint32_t seen = 0;
    for (int p = 0; p < C; ++p) {
        if (m[p] >= C || ((seen >> m[p]) & 1u)) return false;
        seen |= 1u << m[p];
    }
    return true;
}

// applies one op to the chunk (data index bits = positions)
static bool apply_op(const qsv::Plan &P, const DevOp &op, std::vector<cdbl> &d, int C,
                     uint64_t base) {
    const uint32_t N = 1u << C;
    const cdbl *mats = P.dmats.data();
    switch (op.type) {
        case qsv::OP_DENSE: {
            const int k = op.k;
            const uint32_t D = 1u << k;
            uint32_t mask = 0;
            for (int j = 0; j < k; ++j) mask |= 1u << op.a[j];
            std::vector<cdbl> in(D), out(D);
            for (uint32_t x = 0; x < N; ++x) {
                if (x & mask) continue;
                for (uint32_t r = 0; r < D; ++r) {
                    uint32_t xi = x;
                    for (int j = 0; j < k; ++j)
                        if ((r >> j) & 1u) xi |= 1u << op.a[j];
                    in[r] = d[xi];
                }
                for (uint32_t r = 0; r < D; ++r) {
                    cdbl acc = 0;
                    for (uint32_t cc = 0; cc < D; ++cc) acc += mats[op.arg + r * D + cc] * in[cc];
                    out[r] = acc;
                }
                for (uint32_t r = 0; r < D; ++r) {
                    uint32_t xi = x;
                    for (int j = 0; j < k; ++j)
                        if ((r >> j) & 1u) xi |= 1u << op.a[j];
                    d[xi] = out[r];
                }
            }
            return true;
        }
        case qsv::OP_XREG:
        case qsv::OP_CX: {
            const uint32_t t = 1u << op.a[0];
            for (uint32_t x = 0; x < N; ++x) {
                if (x & t) continue;
                if (op.type == qsv::OP_CX && !src_bit(op.a[1], x, base)) continue;
                std::swap(d[x], d[x | t]);
            }
            return true;
        }
        case qsv::OP_DIAG: {
            for (uint32_t x = 0; x < N; ++x) {
                uint32_t sel = 0;
                for (int j = 0; j < op.k; ++j) sel |= (uint32_t)src_bit(op.a[j], x, base) << j;
                d[x] *= mats[op.arg + sel];
            }
            return true;
        }
        default:
            return false;  // parameterised ops are not emulated
    }
}

int main() {
    int n, dt;
    qsv_options o;
    std::memset(&o, 0, sizeof(o));
    if (std::scanf("%d %d", &n, &dt) != 2) return fail("input");
    if (std::scanf("%d %d %d %d %d %d %d %d %d", &o.chunk_bits, &o.pinned_low_bits,
                   &o.fusion_max_qubits, &o.swap_mode, &o.diag_free, &o.register_bits,
                   &o.io_phases, &o.planner, &o.section_kernel) != 9)
        return fail("options");
    size_t ng;
    if (std::scanf("%zu", &ng) != 1) return fail("ngates");
    std::vector<qsv_gate> g(ng);
    std::vector<std::vector<double>> store(ng);
    for (size_t i = 0; i < ng; ++i) {
        std::memset(&g[i], 0, sizeof(qsv_gate));
        int has_m;
        if (std::scanf("%d %d", &g[i].kind, &g[i].nq) != 2) return fail("gate");
        for (int j = 0; j < g[i].nq; ++j)
            if (std::scanf("%d", &g[i].q[j]) != 1) return fail("qubit");
        if (std::scanf("%lf %lf %lf %d", &g[i].p[0], &g[i].p[1], &g[i].p[2], &has_m) != 4)
            return fail("params");
        g[i].param = -1;
        if (has_m) {
            store[i].resize(2u << (2 * g[i].nq));
            for (double &v : store[i])
                if (std::scanf("%lf", &v) != 1) return fail("matrix");
            g[i].m = store[i].data();
        }
    }
    const uint64_t NS = 1ull << n;
    std::vector<cdbl> st(NS);
    for (uint64_t i = 0; i < NS; ++i) {
        double re, im;
        if (std::scanf("%lf %lf", &re, &im) != 2) return fail("state");
        st[i] = cdbl(re, im);
    }

    qsv_plan *pl = nullptr;
    if (qsv_plan_blocks(&o, (qsv_dtype)dt, n, g.data(), ng, &pl) != QSV_OK)
        return fail(std::string("plan: ") + qsv_last_error());
    const qsv::Plan &P = pl->p;
    const bool materialise = P.opt.swap_mode == QSV_SWAP_MATERIALIZE;
    const bool split = !qsv::lds_resident(P.opt);  // kernels whose transpositions use xw / xr

    auto swap_bits = [&](int a, int b) {
        for (uint64_t i = 0; i < NS; ++i)
            if (((i >> a) & 1ull) && !((i >> b) & 1ull)) std::swap(st[i], st[i ^ (1ull << a) ^ (1ull << b)]);
    };

    for (size_t si = 0; si < P.dsec.size(); ++si) {
        if (materialise)
            for (auto &pr : P.sections[si].swaps_before) swap_bits(pr.first, pr.second);
        const DevSection &S = P.dsec[si];
        const int C = (int)S.c;
        const uint32_t N = 1u << C;
        const bool paired = (S.flags & qsv::SEC_PAIRED) != 0;
        const int R = paired ? 4 : std::min(P.r, C);
        // tables: maps are permutations; consecutive transpositions address LDS consistently
        for (uint32_t ph = S.phase_begin; ph < S.phase_end; ++ph) {
            const DevPhase &F = P.dphase[ph];
            if (!is_perm(F.rd, C) || !is_perm(F.wr, C)) return fail("phase map not a permutation");
            if (paired) {
                const uint32_t nops = F.op_end - F.op_begin;
                if (nops != 2) return fail("paired phase without two ops");
                const DevOp &A = P.dops[F.op_begin], &B2 = P.dops[F.op_begin + 1];
                if (A.type != qsv::OP_DENSE || A.k != 2 || A.a[0] != 0 || A.a[1] != 1 ||
                    B2.type != qsv::OP_DENSE || B2.k != 2 || B2.a[0] != 2 || B2.a[1] != 3)
                    return fail("paired op positions");
            }
            for (uint32_t k = F.op_begin; k < F.op_end; ++k) {
                const DevOp &op = P.dops[k];
                if (op.type == qsv::OP_DENSE)
                    for (int j = 0; j < op.k; ++j)
                        if (op.a[j] >= R || (j && op.a[j] <= op.a[j - 1]))
                            return fail("dense op outside the registers or unsorted");
            }
            if (split && ph + 1 < S.phase_end) {
                const DevPhase &G = P.dphase[ph + 1];
                std::vector<char> hit(N, 0);
                for (uint32_t x = 0; x < N; ++x) {
                    uint32_t aw = 0, ar = 0;
                    const uint32_t y = remap(x, F.wr, G.rd, C);
                    for (int p = 0; p < C; ++p) {
                        if ((x >> p) & 1u) aw ^= F.xw[p];
                        if ((y >> p) & 1u) ar ^= F.xr[p];
                    }
                    if (aw != ar) return fail("LDS write and read addresses differ");
                    if (aw >= N || hit[aw]) return fail("LDS layout not a bijection");
                    hit[aw] = 1;
                }
            }
        }
        // every chunk: gather, phases, scatter
        std::vector<cdbl> d(N);
        const uint64_t nchunks = 1ull << (n - C);
        for (uint64_t ch = 0; ch < nchunks; ++ch) {
            uint64_t base = 0;
            for (int t = 0; t < (int)S.n_nl; ++t)
                if ((ch >> t) & 1ull) base |= 1ull << S.nl_phys[t];
            auto addr = [&](uint32_t x, const uint8_t *phys) {
                uint64_t a = base;
                for (int p = 0; p < C; ++p)
                    if ((x >> p) & 1u) a |= 1ull << phys[p];
                return a;
            };
            for (uint32_t x = 0; x < N; ++x) d[x] = st[addr(x, S.gather_phys)];
            for (uint32_t ph = S.phase_begin; ph < S.phase_end; ++ph) {
                const DevPhase &F = P.dphase[ph];
                for (uint32_t k = F.op_begin; k < F.op_end; ++k)
                    if (!apply_op(P, P.dops[k], d, C, base)) return fail("unsupported op");
                if (ph + 1 < S.phase_end) {
                    std::vector<cdbl> e(N);
                    for (uint32_t x = 0; x < N; ++x) e[remap(x, F.wr, P.dphase[ph + 1].rd, C)] = d[x];
                    d.swap(e);
                }
            }
            for (uint32_t x = 0; x < N; ++x) st[addr(x, S.scatter_phys)] = d[x];
        }
    }
    if (materialise)
        for (auto &pr : P.restore_swaps) swap_bits(pr.first, pr.second);
    for (uint64_t i = 0; i < NS; ++i) std::printf("%.17g %.17g\n", st[i].real(), st[i].imag());
    qsv_plan_destroy(pl);
    return 0;
}
