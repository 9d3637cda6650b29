// Host planner: the cache-blocking transpiler of Sec. IV-A and its lowering to
// device tables.
//
// Steps (all host, deterministic, no GPU):
//   1. validate the gates and build FP64 matrices (Eq. (1), Eq. (2), textbook);
//   2. blocking (the transpiler listing of Sec. IV-A, made precise):
//        repeat until no gate remains:
//          choose the chunk's qubit set (c qubits) from the remaining gates;
//          emit chunk_swaps (materialise mode) or just switch the chunk's bit set
//          (remap mode: nothing moves, the next section gathers other bits);
//          scan the remaining gates in order: a gate whose qubits are all in
//          the chunk and none of whose qubits is blocked joins the section;
//          otherwise all its qubits become blocked and it waits for the next
//          round (gates on disjoint qubits commute, so this only reorders
//          commuting gates; Sec. IV-A);
//      readings where the listing is loose: the chunk holds c qubits (not c-1),
//      a deferred gate blocks all of its qubits, and the first remaining gate
//      is always admitted so that every section makes progress;
//   3. per section, the same greedy step one level down: register phases
//      (which r chunk qubits sit in each thread's registers), then fusion of
//      consecutive register gates into dense matrices of at most f qubits;
//   4. the per-gate op list (one kernel per gate, the unblocked baseline).
#include <algorithm>
#include <functional>
#include <atomic>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "qsv_internal.hpp"

namespace qsv {

static inline int popc(uint64_t x) { return __builtin_popcountll(x); }
static inline uint64_t bit(int q) { return 1ull << q; }

void default_options(qsv_dtype dt, qsv_options &o) {
    std::memset(&o, 0, sizeof(o));
    o.chunk_bits = dt == QSV_C64 ? 13 : 12;
    o.pinned_low_bits = dt == QSV_C64 ? 4 : 3;
    o.fusion_max_qubits = 2;
    o.swap_mode = QSV_SWAP_REMAP;
    o.diag_free = 1;
    o.register_bits = dt == QSV_C64 ? 5 : 4;
    o.io_phases = 0;
    o.planner = QSV_PLANNER_DEFAULT;
}

// ---------------------------------------------------------------------------
// gate classification

namespace {

bool is_param_rot(const GateRec &g) { return g.param >= 0; }

// qubits that must be inside the chunk for the gate to run in a section
uint64_t need_local(const GateRec &g, bool diag_free) {
    if (g.is_swap) return g.qmask;
    if (diag_free) {
        if (g.diagonal) return 0;
        if (g.kind == QSV_CX) return bit(g.q[1]);
    }
    return g.qmask;
}

// qubits that must sit in register positions for the gate to run in a phase
uint64_t need_reg(const GateRec &g) {
    if (g.is_swap || g.diagonal) return 0;
    if (g.kind == QSV_CX) return bit(g.q[1]);
    return g.qmask;
}

// ---------------------------------------------------------------------------
// chunk choice (remap mode): several greedy candidates, keep the one whose
// section admits the most gates.

struct Blocker {
    const std::vector<GateRec> &G;
    bool diag_free;
};

uint64_t choose_inorder(const Blocker &B, const std::vector<int> &rem, uint64_t start, int cap,
                        int min_arity) {
    uint64_t chosen = start, blocked = 0;
    for (int idx : rem) {
        const GateRec &g = B.G[idx];
        uint64_t nm = need_local(g, B.diag_free);
        if (g.qmask & blocked) {
            blocked |= g.qmask;
            continue;
        }
        if (popc(nm) < min_arity) {
            // the first pass of the listing looks at multi-qubit gates only; a
            // 1-qubit gate on a qubit not yet chosen would be deferred by the
            // scan and so blocks its qubit
            if ((nm & ~chosen) != 0) blocked |= g.qmask;
            continue;
        }
        if (popc(chosen | nm) <= cap)
            chosen |= nm;
        else
            blocked |= g.qmask;
    }
    return chosen;
}

int scan_count(const Blocker &B, const std::vector<int> &rem, uint64_t local) {
    uint64_t blocked = 0;
    int cnt = 0;
    for (int idx : rem) {
        const GateRec &g = B.G[idx];
        if (!(g.qmask & blocked) && !(need_local(g, B.diag_free) & ~local))
            ++cnt;
        else
            blocked |= g.qmask;
    }
    return cnt;
}

// Greedy on the section's actual gate count: starting from the first remaining
// gate's qubits, repeatedly add the need-set of a remaining gate that raises
// the number of admitted gates the most (per added qubit if `per_qubit`).
uint64_t choose_gain(const Blocker &B, const std::vector<int> &rem, uint64_t start, int cap,
                     bool per_qubit, size_t window) {
    uint64_t chosen = start | need_local(B.G[rem[0]], B.diag_free);
    int cur = scan_count(B, rem, chosen);
    std::vector<uint64_t> seen;
    while (popc(chosen) < cap) {
        uint64_t best_add = 0;
        double best_score = 0.0;
        seen.clear();
        const size_t lim = std::min(window, rem.size());
        for (size_t t = 0; t < lim; ++t) {
            uint64_t nm = need_local(B.G[rem[t]], B.diag_free) & ~chosen;
            if (!nm || popc(chosen | nm) > cap) continue;
            if (std::find(seen.begin(), seen.end(), nm) != seen.end()) continue;
            seen.push_back(nm);
            int cnt = scan_count(B, rem, chosen | nm);
            double score = per_qubit ? double(cnt - cur) / popc(nm) : double(cnt - cur);
            if (score > best_score) {
                best_score = score;
                best_add = nm;
            }
        }
        if (!best_add) break;
        chosen |= best_add;
        cur = scan_count(B, rem, chosen);
    }
    return chosen;
}

uint64_t fill_low(uint64_t chosen, int cap, int n) {
    for (int q = 0; q < n && popc(chosen) < cap; ++q) chosen |= bit(q);
    return chosen;
}

// the candidate chunk sets for one section (remap semantics: logical == physical)
void chunk_candidates(const Blocker &B, const std::vector<int> &rem, uint64_t start, int c,
                      int n, std::vector<uint64_t> &out) {
    out.clear();
    out.push_back(choose_inorder(B, rem, start, c, 1));
    uint64_t multi = choose_inorder(B, rem, start, c, 2);
    out.push_back(multi);
    // paper order: multi-qubit gates choose first, then 1-qubit gates fill
    out.push_back(choose_inorder(B, rem, multi, c, 1));
    out.push_back(choose_gain(B, rem, start, c, false, 96));
    out.push_back(choose_gain(B, rem, start, c, true, 96));
    (void)n;
}

std::vector<int> scan_rest(const Blocker &B, const std::vector<int> &rem, uint64_t local) {
    std::vector<int> next;
    uint64_t blocked = 0;
    for (int idx : rem) {
        const GateRec &g = B.G[idx];
        if (!(g.qmask & blocked) && !(need_local(g, B.diag_free) & ~local)) continue;
        blocked |= g.qmask;
        next.push_back(idx);
    }
    return next;
}

// Sections a greedy plan (best-count candidate per section, no lookahead)
// needs for the gates in `rem` (remap semantics).
int rollout_sections(const Blocker &B, std::vector<int> rem, uint64_t start, int c, int n) {
    int sections = 0;
    std::vector<uint64_t> cands;
    while (!rem.empty()) {
        chunk_candidates(B, rem, start, c, n, cands);
        uint64_t best = 0;
        int best_cnt = -1;
        for (uint64_t cand : cands) {
            const uint64_t full = fill_low(cand, c, n);
            const int cnt = scan_count(B, rem, full);
            if (cnt > best_cnt) {
                best_cnt = cnt;
                best = full;
            }
        }
        rem = scan_rest(B, rem, best);
        ++sections;
    }
    return sections;
}

// Beam search over section sequences (remap semantics): every state is the
// list of gates still to run; each state is expanded with the candidate chunk
// sets of the greedy planner and the `width` states with the fewest remaining
// gates survive each level.  The first level on which a state has no gate left
// gives the plan.
std::vector<uint64_t> beam_chunks(const Blocker &B, const std::vector<int> &rem0, uint64_t start,
                                  int c, int n, int width, bool rollout) {
    struct St {
        std::vector<int> rem;
        std::vector<uint64_t> chunks;
        int est;                 // sections a greedy plan of the rest needs (rollout scoring)
    };
    std::vector<St> beam{St{rem0, {}, 0}};
    std::vector<uint64_t> cands;
    while (true) {
        std::vector<St> next;
        for (const St &s : beam) {
            chunk_candidates(B, s.rem, start, c, n, cands);
            for (uint64_t cand : cands) {
                const uint64_t full = fill_low(cand, c, n);
                St t;
                t.rem = scan_rest(B, s.rem, full);
                t.chunks = s.chunks;
                t.chunks.push_back(full);
                if (t.rem.empty()) return t.chunks;
                bool dup = false;
                for (const St &u : next) dup = dup || u.rem == t.rem;
                if (dup) continue;
                t.est = rollout ? rollout_sections(B, t.rem, start, c, n) : 0;
                next.push_back(std::move(t));
            }
        }
        std::stable_sort(next.begin(), next.end(), [](const St &a, const St &b) {
            return a.est != b.est ? a.est < b.est : a.rem.size() < b.rem.size();
        });
        if ((int)next.size() > width) next.resize(width);
        beam.swap(next);
    }
}

// Exact minimum number of sections (remap semantics) by breadth-first search
// over the sets of gates already run (at most 64 gates).  A section with chunk
// set C runs every remaining gate whose needed qubits lie in C and none of
// whose qubits is blocked by an earlier deferred gate (the scan of the
// listing); running more gates never hurts, so each (state, C) pair has one
// successor.  Returns false when the search would exceed `max_states`.
bool exact_chunks(const Blocker &B, int ng, uint64_t pinned, int c, int n, size_t max_states,
                  std::vector<uint64_t> &out) {
    const uint64_t all = ng == 64 ? ~0ull : ((1ull << ng) - 1);
    std::vector<uint64_t> needm(ng), qm(ng);
    for (int i = 0; i < ng; ++i) {
        needm[i] = need_local(B.G[i], B.diag_free);
        qm[i] = B.G[i].qmask;
    }
    auto closure = [&](uint64_t done, uint64_t C) {
        uint64_t blocked = 0;
        for (int i = 0; i < ng; ++i) {
            if ((done >> i) & 1) continue;
            if (!(qm[i] & blocked) && !(needm[i] & ~C))
                done |= 1ull << i;
            else
                blocked |= qm[i];
        }
        return done;
    };
    // chunk sets: every c-subset of the n qubits that holds the pinned ones
    std::vector<uint64_t> chunks;
    const int free_bits = n - popc(pinned);
    const int want = c - popc(pinned);
    if (want < 0 || free_bits > 24) return false;
    std::vector<int> freeq;
    for (int q = 0; q < n; ++q)
        if (!((pinned >> q) & 1)) freeq.push_back(q);
    for (uint64_t sub = 0; sub < (1ull << free_bits); ++sub) {
        if (popc(sub) != std::min(want, free_bits)) continue;
        uint64_t C = pinned;
        for (int j = 0; j < free_bits; ++j)
            if ((sub >> j) & 1) C |= bit(freeq[j]);
        chunks.push_back(C);
        if (chunks.size() > 4096) return false;
    }
    std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> parent;  // state -> (prev, chunk)
    std::vector<uint64_t> frontier{0};
    parent[0] = {0, 0};
    if (ng == 0) return true;
    while (!frontier.empty()) {
        std::vector<uint64_t> next;
        for (uint64_t s : frontier) {
            for (uint64_t C : chunks) {
                const uint64_t t = closure(s, C);
                if (t == s || parent.count(t)) continue;
                parent[t] = {s, C};
                if (t == all) {
                    for (uint64_t x = t; x != 0; x = parent[x].first) out.push_back(parent[x].second);
                    std::reverse(out.begin(), out.end());
                    return true;
                }
                next.push_back(t);
                if (parent.size() > max_states) return false;
            }
        }
        // keep only states no other state of the level contains (a superset of the
        // gates run is never worse)
        std::sort(next.begin(), next.end(), [](uint64_t a, uint64_t b) { return popc(a) > popc(b); });
        std::vector<uint64_t> kept;
        for (uint64_t t : next) {
            bool dom = false;
            for (uint64_t u : kept)
                if ((t & u) == t) {
                    dom = true;
                    break;
                }
            if (!dom) kept.push_back(t);
        }
        frontier.swap(kept);
    }
    return false;
}

}  // namespace

// ---------------------------------------------------------------------------

static qsv_status validate_and_build(int n, const qsv_gate *g, size_t ng, std::vector<GateRec> &out,
                               int64_t &n_params, std::string &err) {
    out.clear();
    out.reserve(ng);
    n_params = 0;
    for (size_t i = 0; i < ng; ++i) {
        const qsv_gate &s = g[i];
        GateRec r;
        r.kind = s.kind;
        int nq = 0;
        if (s.kind == QSV_AMP_DAMP || s.kind == QSV_PHASE_DAMP || s.kind == QSV_DEPOLARIZE ||
            s.kind == QSV_KRAUS) {
            err = "gate " + std::to_string(i) + ": noise channels need a density-matrix plan "
                  "(qsv_plan_density)";
            return QSV_E_UNSUPPORTED;
        }
        if (!gate_arity(s.kind, nq)) {
            err = "gate " + std::to_string(i) + ": unknown kind " + std::to_string(s.kind);
            return QSV_E_INVALID;
        }
        if (nq < 0) {
            if (s.nq < 1 || s.nq > QSV_MAX_GATE_QUBITS) {
                err = "gate " + std::to_string(i) + ": unitary arity must be 1..5";
                return QSV_E_INVALID;
            }
            nq = s.nq;
        }
        if (s.nq != nq) {
            err = "gate " + std::to_string(i) + ": nq does not match its kind";
            return QSV_E_INVALID;
        }
        r.nq = nq;
        for (int j = 0; j < nq; ++j) {
            if (s.q[j] < 0 || s.q[j] >= n) {
                err = "gate " + std::to_string(i) + ": qubit out of range";
                return QSV_E_INVALID;
            }
            if (r.qmask & bit(s.q[j])) {
                err = "gate " + std::to_string(i) + ": repeated qubit";
                return QSV_E_INVALID;
            }
            r.q[j] = s.q[j];
            r.qmask |= bit(s.q[j]);
        }
        for (int j = 0; j < 3; ++j) r.p[j] = s.p[j];
        if (!std::isfinite(r.p[0]) || !std::isfinite(r.p[1]) || !std::isfinite(r.p[2])) {
            err = "gate " + std::to_string(i) + ": non-finite angle";
            return QSV_E_NUMERIC;
        }
        r.param = s.param;
        if (s.param >= 0) {
            if (s.kind != QSV_RX && s.kind != QSV_RY && s.kind != QSV_RZ && s.kind != QSV_P) {
                err = "gate " + std::to_string(i) + ": only rx/ry/rz/p take a bound parameter";
                return QSV_E_INVALID;
            }
            n_params = std::max<int64_t>(n_params, (int64_t)s.param + 1);
        }
        r.diagonal = kind_is_diagonal(s.kind);
        r.is_swap = s.kind == QSV_SWAP;
        if (s.kind == QSV_UNITARY) {
            if (!s.m) {
                err = "gate " + std::to_string(i) + ": unitary without matrix";
                return QSV_E_INVALID;
            }
            size_t d = size_t(1) << nq;
            r.m.resize(d * d);
            for (size_t e = 0; e < d * d; ++e) {
                r.m[e] = cd(s.m[2 * e], s.m[2 * e + 1]);
                if (!std::isfinite(s.m[2 * e]) || !std::isfinite(s.m[2 * e + 1])) {
                    err = "gate " + std::to_string(i) + ": non-finite matrix entry";
                    return QSV_E_NUMERIC;
                }
            }
            bool diag = true;
            for (size_t a = 0; a < d && diag; ++a)
                for (size_t b = 0; b < d; ++b)
                    if (a != b && r.m[a * d + b] != cd(0.0, 0.0)) {
                        diag = false;
                        break;
                    }
            r.diagonal = diag;
        } else {
            named_matrix(s.kind, r.p, r.m);
        }
        out.push_back(std::move(r));
    }
    return QSV_OK;
}

// Permute a k-qubit matrix from gate order (local bit j = gate qubit j) into the
// order in which local bit j is the j-th smallest of `keys` (keys[j] = sort key
// of gate qubit j).  Returns the sorted keys' permutation in `order`.
static std::vector<cd> sorted_matrix(const std::vector<cd> &m, int k, const int *keys,
                                     std::vector<int> &order) {
    order.resize(k);
    for (int j = 0; j < k; ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return keys[a] < keys[b]; });
    // new local bit t holds gate bit order[t]
    size_t d = size_t(1) << k;
    auto remap = [&](size_t x) {
        size_t y = 0;
        for (int t = 0; t < k; ++t) y |= ((x >> order[t]) & 1) << t;
        return y;
    };
    std::vector<cd> out(d * d);
    for (size_t a = 0; a < d; ++a)
        for (size_t b = 0; b < d; ++b) out[remap(a) * d + remap(b)] = m[a * d + b];
    return out;
}

// ---------------------------------------------------------------------------
// blocking

static bool block_circuit(Plan &P) {
    const int n = P.n;
    const int c = P.c;
    const bool diag_free = P.opt.diag_free != 0;
    const bool materialise = P.opt.swap_mode == QSV_SWAP_MATERIALIZE;
    const int L = materialise ? 0 : P.opt.pinned_low_bits;
    Blocker B{P.gates, diag_free};

    std::vector<int> rem(P.gates.size());
    for (size_t i = 0; i < rem.size(); ++i) rem[i] = (int)i;

    std::vector<int> layout(n), inv(n);  // logical -> physical, physical -> logical
    for (int q = 0; q < n; ++q) layout[q] = inv[q] = q;
    const uint64_t pinned = (L > 0) ? ((1ull << L) - 1) : 0;

    // Candidate scoring: for circuits of up to 1024 gates (remap mode) each
    // candidate is scored by the sections a greedy plan of the rest needs
    // (about a second of host time at 600 gates); larger circuits use one
    // section of lookahead.
    const int strategy = P.opt.planner;
    const bool rollout = !materialise && P.gates.size() <= 1024 && strategy == QSV_PLANNER_DEFAULT;
    P.sections.clear();
    P.chunk_swaps = 0;
    uint64_t prev_local_logical = 0;
    bool first = true;
    // beam and exact strategies fix the whole sequence of chunk sets up front
    // (remap semantics); the default and greedy planners choose section by section
    std::vector<uint64_t> fixed;
    if (strategy == QSV_PLANNER_BEAM || strategy == QSV_PLANNER_EXACT) {
        if (strategy == QSV_PLANNER_EXACT) {
            if (!exact_chunks(B, (int)P.gates.size(), pinned, c, n, 4000000, fixed)) return false;
        } else {
            // a beam ranked by remaining gates (width 16) and, for circuits the
            // default planner also rolls out, one ranked by the greedy rollout of
            // the rest (width 8); the shorter plan wins
            fixed = beam_chunks(B, rem, pinned, c, n, 16, false);
            if (P.gates.size() <= 1024) {
                std::vector<uint64_t> r = beam_chunks(B, rem, pinned, c, n, 8, true);
                if (r.size() < fixed.size()) fixed.swap(r);
            }
            // never worse than the default planner: its section count is the bound
            Plan D;
            D.n = n;
            D.c = c;
            D.gates = P.gates;
            D.opt = P.opt;
            D.opt.planner = QSV_PLANNER_DEFAULT;
            (void)block_circuit(D);
            if (D.sections.size() < fixed.size()) {
                fixed.clear();
                for (const HostSection &S : D.sections) {
                    uint64_t m = 0;
                    for (int ph : S.phys_local) m |= bit(ph);
                    fixed.push_back(m);
                }
            }
        }
    }
    size_t fixed_at = 0;
    while (!rem.empty()) {
        // candidate chunk sets; the first remaining gate is never blocked, so
        // each candidate admits it
        uint64_t start = 0;
        if (!materialise) start = pinned;  // remap: logical == physical, low bits pinned
        std::vector<uint64_t> cands, cands2;
        chunk_candidates(B, rem, start, c, n, cands);
        uint64_t best = 0;
        int best_score = INT32_MIN, best_cnt = -1;
        for (uint64_t cand : cands) {
            uint64_t full = cand;
            if (materialise) {
                // fill with qubits already in the chunk (no swap needed)
                for (int p = 0; p < c && popc(full) < c; ++p) full |= bit(inv[p]);
            }
            full = fill_low(full, c, n);
            int cnt = scan_count(B, rem, full);
            std::vector<int> nxt = scan_rest(B, rem, full);
            int score;
            if (rollout) {
                // fewest sections for the rest of the circuit under the greedy rule
                score = -rollout_sections(B, nxt, start, c, n);
            } else {
                // one section of lookahead: gates this section plus the best next one
                score = cnt;
                if (!nxt.empty()) {
                    chunk_candidates(B, nxt, start, c, n, cands2);
                    int b2 = 0;
                    for (uint64_t c2 : cands2)
                        b2 = std::max(b2, scan_count(B, nxt, fill_low(c2, c, n)));
                    score += b2;
                }
            }
            if (score > best_score || (score == best_score && cnt > best_cnt)) {
                best_score = score;
                best_cnt = cnt;
                best = full;
            }
        }
        if (fixed_at < fixed.size()) best = fixed[fixed_at++];
        uint64_t local = best;  // logical qubits in the chunk

        HostSection S;
        if (materialise) {
            // chunk_swaps: every chosen qubit outside physical [0, c) trades places with
            // an unchosen qubit inside, the one used farthest in the future (ties: highest slot)
            std::vector<int> next_use(n, INT32_MAX);
            for (size_t t = rem.size(); t-- > 0;) {
                const GateRec &g = P.gates[rem[t]];
                for (int j = 0; j < g.nq; ++j) next_use[g.q[j]] = (int)t;
            }
            for (int q = 0; q < n; ++q) {
                if (!((local >> q) & 1) || layout[q] < c) continue;
                int victim_slot = -1;
                for (int p = 0; p < c; ++p) {
                    int lq = inv[p];
                    if ((local >> lq) & 1) continue;
                    if (victim_slot < 0 || next_use[lq] > next_use[inv[victim_slot]] ||
                        (next_use[lq] == next_use[inv[victim_slot]] && p > victim_slot))
                        victim_slot = p;
                }
                int a = victim_slot, b = layout[q];
                int qa = inv[a];
                S.swaps_before.push_back({a, b});
                layout[q] = a;
                layout[qa] = b;
                inv[a] = q;
                inv[b] = qa;
                ++P.chunk_swaps;
            }
        } else if (!first) {
            P.chunk_swaps += popc(local & ~prev_local_logical);
        }
        uint64_t phys_mask = 0;
        for (int q = 0; q < n; ++q)
            if ((local >> q) & 1) phys_mask |= bit(layout[q]);
        for (int p = 0; p < n; ++p)
            if ((phys_mask >> p) & 1) S.phys_local.push_back(p);
        S.layout_at = layout;

        std::vector<int> next;
        uint64_t blocked = 0;
        for (int idx : rem) {
            const GateRec &g = P.gates[idx];
            if (!(g.qmask & blocked) && !(need_local(g, diag_free) & ~local))
                S.gates.push_back(idx);
            else {
                blocked |= g.qmask;
                next.push_back(idx);
            }
        }
        P.sections.push_back(std::move(S));
        rem.swap(next);
        prev_local_logical = local;
        first = false;
    }
    if (P.sections.empty()) {
        // an empty circuit still has one (identity) section so that the apply is well defined
        HostSection S;
        for (int p = 0; p < std::min(c, n); ++p) S.phys_local.push_back(p);
        S.layout_at = layout;
        P.sections.push_back(S);
    }
    P.final_perm = layout;
    // restore swaps (materialise): bring every logical qubit home with transpositions
    P.restore_swaps.clear();
    if (materialise) {
        std::vector<int> lay = layout, iv = inv;
        for (int q = 0; q < n; ++q) {
            if (lay[q] == q) continue;
            int a = q, b = lay[q];  // physical a holds iv[a]; move q from b to a
            int qa = iv[a];
            P.restore_swaps.push_back({std::min(a, b), std::max(a, b)});
            lay[q] = a;
            lay[qa] = b;
            iv[a] = q;
            iv[b] = qa;
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// register phases + fusion for one section

namespace {

struct POp {                      // op before encoding, on data positions
    DevOp op;
    std::vector<cd> m;            // dense matrix / diagonal table (FP64)
    bool fusable = false;         // dense-able on register positions only
    uint32_t regmask = 0;         // register positions it reads/writes (fusable ops)
};

// Embed op `o` (fusable) as a dense matrix over the positions in `pos` (ascending).
std::vector<cd> embed(const POp &o, const std::vector<int> &pos) {
    int k = (int)pos.size();
    size_t d = size_t(1) << k;
    auto idx_of = [&](int p) {
        for (int t = 0; t < k; ++t)
            if (pos[t] == p) return t;
        return -1;
    };
    std::vector<cd> E(d * d, cd(0, 0));
    const DevOp &op = o.op;
    for (size_t x = 0; x < d; ++x) {
        // column x: the image of basis state x
        if (op.type == OP_DENSE) {
            int kk = op.k;
            int t[5];
            for (int j = 0; j < kk; ++j) t[j] = idx_of(op.a[j]);
            size_t sub = 0;
            for (int j = 0; j < kk; ++j) sub |= ((x >> t[j]) & 1) << j;
            size_t rest = x;
            for (int j = 0; j < kk; ++j) rest &= ~(size_t(1) << t[j]);
            size_t dk = size_t(1) << kk;
            for (size_t row = 0; row < dk; ++row) {
                size_t y = rest;
                for (int j = 0; j < kk; ++j) y |= ((row >> j) & 1) << t[j];
                E[y * d + x] += o.m[row * dk + sub];
            }
        } else if (op.type == OP_XREG) {
            int t = idx_of(op.a[0]);
            E[(x ^ (size_t(1) << t)) * d + x] = 1.0;
        } else if (op.type == OP_CX) {
            int t = idx_of(op.a[0]), cc = idx_of(op.a[1]);
            size_t y = ((x >> cc) & 1) ? (x ^ (size_t(1) << t)) : x;
            E[y * d + x] = 1.0;
        } else if (op.type == OP_DIAG) {
            size_t sub = 0;
            for (int j = 0; j < op.k; ++j) sub |= ((x >> idx_of(op.a[j])) & 1) << j;
            E[x * d + x] = o.m[sub];
        }
    }
    return E;
}

std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, size_t d) {
    std::vector<cd> C(d * d, cd(0, 0));
    for (size_t i = 0; i < d; ++i)
        for (size_t k = 0; k < d; ++k) {
            cd a = A[i * d + k];
            if (a == cd(0, 0)) continue;
            for (size_t j = 0; j < d; ++j) C[i * d + j] += a * B[k * d + j];
        }
    return C;
}

std::vector<POp> fuse(const std::vector<POp> &in, int f) {
    if (f < 2) return in;
    std::vector<POp> out;
    size_t i = 0;
    while (i < in.size()) {
        if (!in[i].fusable) {
            out.push_back(in[i++]);
            continue;
        }
        uint32_t mask = in[i].regmask;
        size_t j = i + 1;
        while (j < in.size() && in[j].fusable && popc(mask | in[j].regmask) <= f) {
            mask |= in[j].regmask;
            ++j;
        }
        if (j == i + 1) {
            out.push_back(in[i++]);
            continue;
        }
        std::vector<int> pos;
        for (int p = 0; p < 32; ++p)
            if ((mask >> p) & 1) pos.push_back(p);
        size_t d = size_t(1) << pos.size();
        std::vector<cd> M(d * d, cd(0, 0));
        for (size_t t = 0; t < d; ++t) M[t * d + t] = 1.0;
        for (size_t t = i; t < j; ++t) M = matmul(embed(in[t], pos), M, d);
        POp F;
        std::memset(&F.op, 0, sizeof(F.op));
        F.op.type = OP_DENSE;
        F.op.k = (uint8_t)pos.size();
        for (size_t t = 0; t < pos.size(); ++t) F.op.a[t] = (uint8_t)pos[t];
        F.op.slot = -1;
        F.m = std::move(M);
        F.fusable = true;
        F.regmask = mask;
        out.push_back(std::move(F));
        i = j;
    }
    return out;
}

// positions an op reads or writes (sources outside the chunk excluded)
uint32_t touched(const POp &o) {
    if (o.fusable) return o.regmask;
    uint32_t m = 0;
    for (int j = 0; j < o.op.k && j < 5; ++j)
        if (o.op.a[j] < SRC_GLOBAL) m |= 1u << o.op.a[j];
    if (o.op.type == OP_CX || o.op.type == OP_XREG || o.op.type == OP_PROT) m |= 1u << o.op.a[0];
    if (o.op.type == OP_CX && o.op.a[1] < SRC_GLOBAL) m |= 1u << o.op.a[1];
    if (o.op.type == OP_PDIAG && o.op.a[0] < SRC_GLOBAL) m |= 1u << o.op.a[0];
    return m;
}

// Block fusion (for the matrix-core path, where a fused op's cost grows with
// its width, not with the gates in it): starting from the first unplaced op,
// take every later dense-able op whose positions keep the block within f
// qubits and that commutes past all ops left behind so far (disjoint
// positions), multiply them in circuit order, and place the block where its
// first op was.  Ops left behind keep their order.
std::vector<POp> fuse_blocks(const std::vector<POp> &in, int f) {
    if (f < 2) return in;
    std::vector<POp> out;
    std::vector<char> used(in.size(), 0);
    for (size_t i = 0; i < in.size(); ++i) {
        if (used[i]) continue;
        used[i] = 1;
        if (!in[i].fusable) {
            out.push_back(in[i]);
            continue;
        }
        uint32_t mask = in[i].regmask, blocked = 0;
        std::vector<size_t> members = {i};
        for (size_t j = i + 1; j < in.size(); ++j) {
            if (used[j]) continue;
            const uint32_t tj = touched(in[j]);
            if (in[j].fusable && !(tj & blocked) && popc(mask | tj) <= f) {
                mask |= tj;
                members.push_back(j);
                used[j] = 1;
            } else {
                blocked |= tj;
            }
            if ((mask & ~blocked) == 0) break;  // nothing more can join
        }
        if (members.size() == 1) {
            out.push_back(in[i]);
            continue;
        }
        std::vector<int> pos;
        for (int p = 0; p < 32; ++p)
            if ((mask >> p) & 1) pos.push_back(p);
        size_t d = size_t(1) << pos.size();
        std::vector<cd> M(d * d, cd(0, 0));
        for (size_t t = 0; t < d; ++t) M[t * d + t] = 1.0;
        for (size_t t : members) M = matmul(embed(in[t], pos), M, d);
        POp F;
        std::memset(&F.op, 0, sizeof(F.op));
        F.op.type = OP_DENSE;
        F.op.k = (uint8_t)pos.size();
        for (size_t t = 0; t < pos.size(); ++t) F.op.a[t] = (uint8_t)pos[t];
        F.op.slot = -1;
        F.m = std::move(M);
        F.fusable = true;
        F.regmask = mask;
        out.push_back(std::move(F));
    }
    return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// LDS swizzle of each transposition
//
// A transposition writes every amplitude component to LDS element index
// x = sum of 2^slot over its set data positions and reads it back under the
// next phase's map.  The element actually used is x ^ M(x), M linear with
// M(2^s) = swz[s] holding only bits below min(s, T): a unitriangular map, so a
// permutation of the buffer.  Lanes of one wave are thread bits 0..5 (data
// positions R..R+5); the LDS serves a group of consecutive lanes per cycle, and
// the group is conflict-free when the low bits of its addresses (the bank) are
// distinct, i.e. when the low-T projections of the lanes' address vectors
// 2^s ^ swz[s] are linearly independent.  The masks are searched so that this
// holds for both the write map and the read map, for 128-byte and 256-byte
// bank rows (T = log2 of the row's elements), with a fixed-seed search.  The
// phase stores the per-position vectors (xw, xr), so the kernel indexes no
// table at run time.

static int gf2_rank(uint32_t *v, int m) {
    int rank = 0;
    for (int bit = 31; bit >= 0 && rank < m; --bit) {
        int piv = -1;
        for (int i = rank; i < m; ++i)
            if ((v[i] >> bit) & 1u) { piv = i; break; }
        if (piv < 0) continue;
        std::swap(v[rank], v[piv]);
        for (int i = 0; i < m; ++i)
            if (i != rank && ((v[i] >> bit) & 1u)) v[i] ^= v[rank];
        ++rank;
    }
    return rank;
}

static void assign_swizzles(Plan &P, const DevSection &ds, int R) {
    const int C = (int)ds.c;
    const int EB = P.dtype == QSV_C128 ? 8 : 4;        // component bytes
    const int TB = C - R;                               // thread bits
    const int L = std::min(6, TB);                      // lane bits of one wave
    const int T1 = std::min(C, EB == 8 ? 4 : 5);        // 128-byte bank row
    const int T2 = std::min(C, T1 + 1);                 // 256-byte bank row
    auto score = [&](const uint8_t *map, const uint8_t *col) {
        int sc = 0;
        for (int T : {T1, T2}) {
            const int m = std::min(T, L);
            uint32_t v[8];
            for (int b = 0; b < m; ++b) {
                const int s = map[R + b];
                v[b] = ((1u << s) ^ col[s]) & ((1u << T) - 1u);
            }
            sc += gf2_rank(v, m);
        }
        return sc;
    };
    int best_possible = 0;
    for (int T : {T1, T2}) best_possible += 2 * std::min(T, L);
    uint64_t rng = 0x9E3779B97F4A7C15ull;
    auto next = [&]() {
        rng ^= rng << 13;
        rng ^= rng >> 7;
        rng ^= rng << 17;
        return rng;
    };
    for (uint32_t p = ds.phase_begin; p + 1 < ds.phase_end; ++p) {
        DevPhase &a = P.dphase[p];
        const uint8_t *wr = a.wr, *rd = P.dphase[p + 1].rd;
        uint8_t best[16] = {0}, col[16] = {0};
        int best_sc = score(wr, best) + score(rd, best);
        // only the lane slots of either map need a mask
        bool lane_slot[16] = {false};
        for (int b = 0; b < L; ++b) lane_slot[wr[R + b]] = lane_slot[rd[R + b]] = true;
        for (int it = 0; it < 4096 && best_sc < best_possible; ++it) {
            for (int s = 0; s < C; ++s) {
                const int lim = std::min(s, T2);
                col[s] = (lane_slot[s] && lim > 0) ? (uint8_t)(next() & ((1u << lim) - 1u)) : 0;
            }
            const int sc = score(wr, col) + score(rd, col);
            if (sc > best_sc) {
                best_sc = sc;
                std::memcpy(best, col, sizeof(best));
            }
        }
        for (int q = 0; q < C; ++q) {
            a.xw[q] = (uint16_t)((1u << wr[q]) ^ best[wr[q]]);
            a.xr[q] = (uint16_t)((1u << rd[q]) ^ best[rd[q]]);
        }
    }
}

static void lower_section(Plan &P, int si) {
    HostSection &S = P.sections[si];
    const int C = (int)S.phys_local.size();
    const int R = std::min(P.r, C);
    const std::vector<int> &layout = S.layout_at;
    const int n = P.n;

    // slot of a logical qubit (rank of its physical bit among the chunk's), -1 if non-local
    std::vector<int> slot(n, -1);
    for (int q = 0; q < n; ++q) {
        auto it = std::find(S.phys_local.begin(), S.phys_local.end(), layout[q]);
        if (it != S.phys_local.end()) slot[q] = (int)(it - S.phys_local.begin());
    }
    std::vector<int> slot_q(C);  // slot -> logical qubit
    for (int q = 0; q < n; ++q)
        if (slot[q] >= 0) slot_q[slot[q]] = q;

    DevSection ds;
    std::memset(&ds, 0, sizeof(ds));
    for (int s = 0; s < C; ++s) ds.slot_phys[s] = (uint8_t)S.phys_local[s];
    {
        int t = 0;
        for (int p = 0; p < n; ++p)
            if (std::find(S.phys_local.begin(), S.phys_local.end(), p) == S.phys_local.end())
                ds.nl_phys[t++] = (uint8_t)p;
        ds.n_nl = (uint32_t)t;
    }
    ds.c = (uint32_t)C;
    ds.phase_begin = (uint32_t)P.dphase.size();
    ds.param_slot = (uint32_t)P.n_param_ops;

    // position labels: pos2q[pos] = logical qubit held by data position pos
    std::vector<int> pos2q(C), q2pos(n, -1);
    auto set_map = [&](const std::vector<int> &regq) {
        std::vector<int> rest;
        for (int s = 0; s < C; ++s) {
            int q = slot_q[s];
            if (std::find(regq.begin(), regq.end(), q) == regq.end()) rest.push_back(q);
        }
        // registers: chosen qubits by slot ascending; threads: remaining qubits by slot ascending
        std::vector<int> rq = regq;
        std::sort(rq.begin(), rq.end(), [&](int a, int b) { return slot[a] < slot[b]; });
        for (int i = 0; i < R; ++i) pos2q[i] = rq[i];
        for (int i = 0; i < C - R; ++i) pos2q[R + i] = rest[i];
        std::fill(q2pos.begin(), q2pos.end(), -1);
        for (int i = 0; i < C; ++i) q2pos[pos2q[i]] = i;
    };
    auto src_of = [&](int q) -> uint8_t {
        if (q2pos[q] >= 0) return (uint8_t)q2pos[q];
        return (uint8_t)(SRC_GLOBAL + layout[q]);
    };

    std::vector<int> rem = S.gates;
    bool first = true;
    DevPhase cur;
    std::memset(&cur, 0, sizeof(cur));
    auto snapshot = [&](uint8_t *dst) {
        for (int p = 0; p < C; ++p) dst[p] = (uint8_t)slot[pos2q[p]];
    };

    if (rem.empty()) {
        // identity section: one phase, registers on the highest slots
        std::vector<int> regq;
        for (int s = C - 1; s >= 0 && (int)regq.size() < R; --s) regq.push_back(slot_q[s]);
        set_map(regq);
        snapshot(cur.rd);
        snapshot(cur.wr);
        cur.op_begin = cur.op_end = (uint32_t)P.dops.size();
        P.dphase.push_back(cur);
    }
    while (!rem.empty()) {
        // choose the register qubits: in-order greedy with blocking
        uint64_t chosen = 0, blocked = 0;
        for (int idx : rem) {
            const GateRec &g = P.gates[idx];
            uint64_t rn = need_reg(g);
            if (g.qmask & blocked) {
                blocked |= g.qmask;
                continue;
            }
            if (popc(chosen | rn) <= R)
                chosen |= rn;
            else
                blocked |= g.qmask;
        }
        std::vector<int> regq;
        for (int q = 0; q < n; ++q)
            if ((chosen >> q) & 1) regq.push_back(q);
        if (!first) {
            // keep qubits already in registers when there is room (no preference otherwise)
            for (int p = 0; p < R && (int)regq.size() < R; ++p)
                if (std::find(regq.begin(), regq.end(), pos2q[p]) == regq.end())
                    regq.push_back(pos2q[p]);
        }
        // fill from the highest slots so the lowest slots stay on threads (coalescing)
        for (int s = C - 1; s >= 0 && (int)regq.size() < R; --s)
            if (std::find(regq.begin(), regq.end(), slot_q[s]) == regq.end())
                regq.push_back(slot_q[s]);

        if (!first) {
            snapshot(cur.wr);
            P.dphase.push_back(cur);
        }
        set_map(regq);
        std::memset(&cur, 0, sizeof(cur));
        snapshot(cur.rd);
        cur.op_begin = (uint32_t)P.dops.size();

        // scan
        std::vector<POp> pops;
        std::vector<int> next;
        blocked = 0;
        for (int idx : rem) {
            const GateRec &g = P.gates[idx];
            bool ok = !(g.qmask & blocked);
            if (ok) {
                uint64_t rn = need_reg(g);
                for (int q = 0; q < n; ++q)
                    if (((rn >> q) & 1) && !(q2pos[q] >= 0 && q2pos[q] < R)) ok = false;
            }
            if (!ok) {
                blocked |= g.qmask;
                next.push_back(idx);
                continue;
            }
            POp o;
            std::memset(&o.op, 0, sizeof(o.op));
            o.op.slot = -1;
            if (g.is_swap) {
                // relabel: the two positions exchange the qubits they stand for
                int pa = q2pos[g.q[0]], pb = q2pos[g.q[1]];
                std::swap(pos2q[pa], pos2q[pb]);
                q2pos[g.q[0]] = pb;
                q2pos[g.q[1]] = pa;
                continue;
            }
            if (is_param_rot(g)) {
                RotKind rk = g.kind == QSV_RX ? ROT_RX : g.kind == QSV_RY ? ROT_RY
                           : g.kind == QSV_RZ ? ROT_RZ : ROT_P;
                o.op.rot = rk;
                o.op.k = 1;
                o.op.arg = g.param;
                o.op.slot = (int32_t)P.n_param_ops;
                P.pslots.push_back(PSlot{g.param, (int32_t)rk});
                if (rk == ROT_RX || rk == ROT_RY) {
                    o.op.type = OP_PROT;
                    o.op.a[0] = (uint8_t)q2pos[g.q[0]];
                    P.flops += 16.0 * std::ldexp(1.0, n);
                } else {
                    o.op.type = OP_PDIAG;
                    o.op.a[0] = src_of(g.q[0]);
                    P.flops += 6.0 * std::ldexp(1.0, n);
                }
                ++P.n_param_ops;
                ++ds.n_params_used;
                pops.push_back(std::move(o));
                continue;
            }
            if (g.kind == QSV_X) {
                o.op.type = OP_XREG;
                o.op.k = 1;
                o.op.a[0] = (uint8_t)q2pos[g.q[0]];
                o.fusable = true;
                o.regmask = 1u << o.op.a[0];
            } else if (g.kind == QSV_CX) {
                o.op.type = OP_CX;
                o.op.k = 2;
                o.op.a[0] = (uint8_t)q2pos[g.q[1]];
                o.op.a[1] = src_of(g.q[0]);
                o.fusable = o.op.a[1] < R;
                o.regmask = (1u << o.op.a[0]) | (o.fusable ? (1u << o.op.a[1]) : 0u);
            } else if (g.diagonal) {
                o.op.type = OP_DIAG;
                o.op.k = (uint8_t)g.nq;
                size_t d = size_t(1) << g.nq;
                o.m.resize(d);
                for (size_t t = 0; t < d; ++t) o.m[t] = g.m[t * d + t];
                bool allreg = true;
                for (int j = 0; j < g.nq; ++j) {
                    o.op.a[j] = src_of(g.q[j]);
                    if (o.op.a[j] >= R) allreg = false;
                    else o.regmask |= 1u << o.op.a[j];
                }
                o.fusable = allreg;
            } else {
                o.op.type = OP_DENSE;
                o.op.k = (uint8_t)g.nq;
                int keys[5];
                for (int j = 0; j < g.nq; ++j) keys[j] = q2pos[g.q[j]];
                std::vector<int> order;
                o.m = sorted_matrix(g.m, g.nq, keys, order);
                for (int t = 0; t < g.nq; ++t) {
                    o.op.a[t] = (uint8_t)keys[order[t]];
                    o.regmask |= 1u << o.op.a[t];
                }
                o.fusable = true;
            }
            pops.push_back(std::move(o));
        }
        int f = std::min(P.fusion_eff, R);
        std::vector<POp> fused = P.opt.section_kernel == QSV_KERNEL_MFMA ? fuse_blocks(pops, f)
                                                                         : fuse(pops, f);
        for (POp &o : fused) {
            if (o.op.type == OP_DENSE || o.op.type == OP_DIAG) {
                o.op.arg = (int32_t)P.dmats.size();
                P.dmats.insert(P.dmats.end(), o.m.begin(), o.m.end());
            }
            if (o.op.type == OP_DENSE) {
                P.flops += 8.0 * std::ldexp(1.0, o.op.k) * std::ldexp(1.0, n);
                P.kmax = std::max(P.kmax, (int)o.op.k);
            }
            if (o.op.type == OP_DIAG) P.flops += 6.0 * std::ldexp(1.0, n);
            P.dops.push_back(o.op);
        }
        cur.op_end = (uint32_t)P.dops.size();
        rem.swap(next);
        first = false;
    }
    if (!S.gates.empty()) {
        snapshot(cur.wr);
        P.dphase.push_back(cur);
    }
    ds.phase_end = (uint32_t)P.dphase.size();
    // HBM access through the coalesced map: lanes on the lowest local bits, then
    // the registers, then the remaining thread bits.  When the first (last)
    // phase puts a low bit in registers, an op-free phase in that map goes in
    // front (behind): one more LDS transposition instead of scattered 16-byte
    // accesses.  Only for states of many chunks (small ones stay in cache).
    if (P.opt.io_phases && C > R && n - C >= 8) {
        const int nlane = std::min(6, C - R);
        DevPhase io;
        std::memset(&io, 0, sizeof(io));
        for (int p = 0; p < C; ++p) {
            int sl;
            if (p < R) sl = nlane + p;
            else if (p - R < nlane) sl = p - R;
            else sl = p;
            io.rd[p] = io.wr[p] = (uint8_t)sl;
        }
        auto coalesced = [&](const uint8_t *m) {
            for (int b = 0; b < nlane; ++b)
                if (m[R + b] != b) return false;
            return true;
        };
        if (!coalesced(P.dphase[ds.phase_begin].rd)) {
            io.op_begin = io.op_end = P.dphase[ds.phase_begin].op_begin;
            P.dphase.insert(P.dphase.begin() + ds.phase_begin, io);
        }
        if (!coalesced(P.dphase.back().wr)) {
            io.op_begin = io.op_end = P.dphase.back().op_end;
            P.dphase.push_back(io);
        }
        ds.phase_end = (uint32_t)P.dphase.size();
    }
    bool dense_only = true;
    for (uint32_t ph = ds.phase_begin; ph < ds.phase_end; ++ph)
        for (uint32_t o = P.dphase[ph].op_begin; o < P.dphase[ph].op_end; ++o)
            if (P.dops[o].type != OP_DENSE) dense_only = false;
    ds.flags = dense_only ? SEC_DENSE_ONLY : 0u;
    // physical bit of every data position where the chunk is gathered / scattered
    {
        const DevPhase &f = P.dphase[ds.phase_begin], &l = P.dphase[ds.phase_end - 1];
        bool moves = false;
        for (int p = 0; p < C; ++p) {
            ds.gather_phys[p] = ds.slot_phys[f.rd[p]];
            ds.scatter_phys[p] = ds.slot_phys[l.wr[p]];
            if (p >= R && ds.gather_phys[p] != ds.scatter_phys[p]) moves = true;
        }
        if (moves && ds.phase_end - ds.phase_begin == 1) ds.flags |= SEC_SYNC_SCATTER;
    }
    assign_swizzles(P, ds, R);
    P.dsec.push_back(ds);
}

// ---------------------------------------------------------------------------
// paired phases: a section whose gates are all dense 2-qubit gates on local
// qubits runs phases of exactly two ops at fixed register positions, ops[2p] on
// positions (0, 1) and ops[2p + 1] on (2, 3) (the identity when a phase has only
// one gate pair).  Gates on the same pair fuse into one 4 x 4 matrix.  Fixed
// positions let the kernel update the amplitudes in place with no run-time
// choice of registers; all relabelling happens in the LDS transpositions.

// 4 x 4 matrix of a 2-qubit gate in the order (x0, x1) of the pair it acts on
static std::vector<cd> pair_matrix(const GateRec &g, int x0) {
    if (g.q[0] == x0) return g.m;
    std::vector<cd> m(16);
    auto sw = [](int i) { return ((i & 1) << 1) | ((i >> 1) & 1); };
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) m[r * 4 + c] = g.m[sw(r) * 4 + sw(c)];
    return m;
}

static bool paired_eligible(const Plan &P, const HostSection &S) {
    if (S.gates.empty()) return false;
    for (int gi : S.gates) {
        const GateRec &g = P.gates[gi];
        if (g.nq != 2 || g.is_swap || g.param >= 0) return false;
        if (need_local(g, P.opt.diag_free != 0) != g.qmask) return false;
    }
    return true;
}

static void lower_section_paired(Plan &P, int si) {
    HostSection &S = P.sections[si];
    const int C = (int)S.phys_local.size();
    const int n = P.n;
    const std::vector<int> &layout = S.layout_at;
    std::vector<int> slot(n, -1);
    for (int q = 0; q < n; ++q) {
        auto it = std::find(S.phys_local.begin(), S.phys_local.end(), layout[q]);
        if (it != S.phys_local.end()) slot[q] = (int)(it - S.phys_local.begin());
    }
    std::vector<int> slot_q(C);
    for (int q = 0; q < n; ++q)
        if (slot[q] >= 0) slot_q[slot[q]] = q;

    DevSection ds;
    std::memset(&ds, 0, sizeof(ds));
    for (int s2 = 0; s2 < C; ++s2) ds.slot_phys[s2] = (uint8_t)S.phys_local[s2];
    {
        int t = 0;
        for (int p = 0; p < n; ++p)
            if (std::find(S.phys_local.begin(), S.phys_local.end(), p) == S.phys_local.end())
                ds.nl_phys[t++] = (uint8_t)p;
        ds.n_nl = (uint32_t)t;
    }
    ds.c = (uint32_t)C;
    ds.phase_begin = (uint32_t)P.dphase.size();
    ds.param_slot = (uint32_t)P.n_param_ops;

    std::vector<cd> ident(16, cd(0, 0));
    for (int i = 0; i < 4; ++i) ident[i * 5] = 1.0;
    auto push_op = [&](int p0, const std::vector<cd> &m, bool real_op) {
        DevOp op;
        std::memset(&op, 0, sizeof(op));
        op.type = OP_DENSE;
        op.k = 2;
        op.a[0] = (uint8_t)p0;
        op.a[1] = (uint8_t)(p0 + 1);
        op.slot = -1;
        op.arg = (int32_t)P.dmats.size();
        P.dmats.insert(P.dmats.end(), m.begin(), m.end());
        P.dops.push_back(op);
        if (real_op) P.flops += 32.0 * std::ldexp(1.0, n);
    };

    // Tasks: chains of gates on one qubit pair with nothing in between on either
    // qubit, fused into one 4 x 4 matrix; a task depends on the last earlier task
    // on each of its qubits.
    struct Task {
        uint64_t mask;
        int q0, q1;
        std::vector<cd> m;
        std::vector<int> succ;
        int npred = 0, label = 0;
    };
    std::vector<Task> tasks;
    {
        std::vector<int> last(n, -1);
        for (int gi : S.gates) {
            const GateRec &g = P.gates[gi];
            const int x = g.q[0], y = g.q[1];
            const int tx = last[x], ty = last[y];
            if (tx >= 0 && tx == ty && tasks[tx].mask == g.qmask) {
                tasks[tx].m = matmul(pair_matrix(g, tasks[tx].q0), tasks[tx].m, 4);
                continue;
            }
            Task t;
            t.mask = g.qmask;
            t.q0 = x;
            t.q1 = y;
            t.m = g.m;
            const int id = (int)tasks.size();
            if (tx >= 0) {
                tasks[tx].succ.push_back(id);
                ++t.npred;
            }
            if (ty >= 0 && ty != tx) {
                tasks[ty].succ.push_back(id);
                ++t.npred;
            }
            tasks.push_back(std::move(t));
            last[x] = last[y] = id;
        }
    }
    // Two tasks per phase (two register pairs) with unit-time tasks and precedence:
    // the Coffman-Graham order (labels from the sinks up, smallest decreasing list
    // of successor labels first) scheduled two at a time by highest label needs the
    // fewest phases.
    {
        const int T = (int)tasks.size();
        for (int k = 1; k <= T; ++k) {
            int pick = -1;
            std::vector<int> best;
            for (int t = T - 1; t >= 0; --t) {
                if (tasks[t].label) continue;
                bool ok = true;
                std::vector<int> key;
                for (int u : tasks[t].succ) {
                    if (!tasks[u].label) ok = false;
                    key.push_back(tasks[u].label);
                }
                if (!ok) continue;
                std::sort(key.begin(), key.end(), std::greater<int>());
                if (pick < 0 || key < best) {
                    pick = t;
                    best.swap(key);
                }
            }
            tasks[pick].label = k;
        }
    }
    std::vector<int> ready;
    for (int t = 0; t < (int)tasks.size(); ++t)
        if (tasks[t].npred == 0) ready.push_back(t);
    while (!ready.empty()) {
        std::sort(ready.begin(), ready.end(),
                  [&](int a, int b) { return tasks[a].label > tasks[b].label; });
        const Task &TA = tasks[ready[0]];
        const int a0 = TA.q0, a1 = TA.q1;
        const std::vector<cd> mA = TA.m;
        std::vector<cd> mB = ident;
        int b0 = -1, b1 = -1;
        uint64_t maskB = 0;
        std::vector<int> done = {ready[0]};
        if (ready.size() > 1) {
            const Task &TB = tasks[ready[1]];
            b0 = TB.q0;
            b1 = TB.q1;
            maskB = TB.mask;
            mB = TB.m;
            done.push_back(ready[1]);
        }
        ready.erase(ready.begin(), ready.begin() + (long)done.size());
        for (int t : done)
            for (int u : tasks[t].succ)
                if (--tasks[u].npred == 0) ready.push_back(u);
        // register positions: (a0, a1, b0, b1), filled from the highest slots when
        // the phase has one pair; then the other local qubits by ascending slot
        std::vector<int> regq = {a0, a1};
        if (maskB) {
            regq.push_back(b0);
            regq.push_back(b1);
        } else {
            for (int s2 = C - 1; s2 >= 0 && (int)regq.size() < 4; --s2)
                if (slot_q[s2] != a0 && slot_q[s2] != a1) regq.push_back(slot_q[s2]);
        }
        DevPhase ph;
        std::memset(&ph, 0, sizeof(ph));
        int p = 0;
        for (int q : regq) ph.rd[p++] = (uint8_t)slot[q];
        for (int s2 = 0; s2 < C; ++s2)
            if (std::find(regq.begin(), regq.end(), slot_q[s2]) == regq.end()) ph.rd[p++] = (uint8_t)s2;
        std::memcpy(ph.wr, ph.rd, sizeof(ph.rd));
        ph.op_begin = (uint32_t)P.dops.size();
        push_op(0, mA, true);
        push_op(2, mB, maskB != 0);
        ph.op_end = (uint32_t)P.dops.size();
        P.dphase.push_back(ph);
    }
    P.kmax = std::max(P.kmax, 2);
    ds.phase_end = (uint32_t)P.dphase.size();
    ds.flags = SEC_DENSE_ONLY | SEC_PAIRED;
    const DevPhase &f = P.dphase[ds.phase_begin], &l = P.dphase[ds.phase_end - 1];
    for (int q = 0; q < C; ++q) {
        ds.gather_phys[q] = ds.slot_phys[f.rd[q]];
        ds.scatter_phys[q] = ds.slot_phys[l.wr[q]];
    }
    assign_swizzles(P, ds, 4);
    P.dsec.push_back(ds);
}

// ---------------------------------------------------------------------------
// per-gate op list

static void lower_per_gate(Plan &P) {
    P.pg.clear();
    for (size_t i = 0; i < P.gates.size(); ++i) {
        const GateRec &g = P.gates[i];
        PgOp o;
        std::memset(&o, 0, sizeof(o));
        o.gate = (int32_t)i;
        o.k = (uint8_t)g.nq;
        for (int j = 0; j < g.nq; ++j) o.q[j] = (uint8_t)g.q[j];
        if (g.param >= 0) {
            o.kind = 0;  // resolved at run time (not supported in per-gate mode)
        } else if (g.kind == QSV_X) {
            o.kind = PG_X;
        } else if (g.kind == QSV_CX) {
            o.kind = PG_CX;
        } else if (g.kind == QSV_SWAP) {
            o.kind = PG_SWAP;
        } else if (g.kind == QSV_CZ || g.kind == QSV_CP) {
            o.kind = PG_CPHASE;
            o.arg = (int32_t)P.dmats.size();
            P.dmats.push_back(g.m[15]);
        } else if (g.nq == 1 && g.diagonal && g.m[0] == cd(1.0, 0.0)) {
            o.kind = PG_PHASE1;
            o.arg = (int32_t)P.dmats.size();
            P.dmats.push_back(g.m[3]);
        } else if (g.nq == 1 && g.diagonal) {
            o.kind = PG_DIAG1;
            o.arg = (int32_t)P.dmats.size();
            P.dmats.push_back(g.m[0]);
            P.dmats.push_back(g.m[3]);
        } else {
            o.kind = PG_DENSE;
            int keys[5];
            for (int j = 0; j < g.nq; ++j) keys[j] = g.q[j];
            std::vector<int> order;
            std::vector<cd> m = sorted_matrix(g.m, g.nq, keys, order);
            for (int t = 0; t < g.nq; ++t) o.q[t] = (uint8_t)g.q[order[t]];
            o.arg = (int32_t)P.dmats.size();
            P.dmats.insert(P.dmats.end(), m.begin(), m.end());
        }
        P.pg.push_back(o);
    }
}

// ---------------------------------------------------------------------------

static std::atomic<uint64_t> g_plan_uid{1};

qsv_status build_plan(const qsv_options &opt_in, qsv_dtype dt, int n, const qsv_gate *g,
                      size_t ng, Plan &P, std::string &err) {
    if (dt != QSV_C64 && dt != QSV_C128) {
        err = "dtype must be QSV_C64 or QSV_C128";
        return QSV_E_INVALID;
    }
    if (n < 1 || n > QSV_MAX_QUBITS) {
        err = "n must be in [1, " + std::to_string(QSV_MAX_QUBITS) + "]";
        return QSV_E_INVALID;
    }
    if (ng > 0 && !g) {
        err = "gates pointer is NULL";
        return QSV_E_INVALID;
    }
    qsv_options def;
    default_options(dt, def);
    qsv_options o = opt_in;
    if (o.chunk_bits == 0) o.chunk_bits = def.chunk_bits;
    if (o.pinned_low_bits < 0) o.pinned_low_bits = def.pinned_low_bits;
    if (o.register_bits == 0) o.register_bits = def.register_bits;
    if (o.chunk_bits < 1 || o.chunk_bits > 14) {
        err = "chunk_bits must be in [1, 14] (the chunk lives in on-chip memory)";
        return QSV_E_INVALID;
    }
    if (o.register_bits < 1 || o.register_bits > 5) {
        err = "register_bits must be in [1, 5]";
        return QSV_E_INVALID;
    }
    if (o.io_phases != 0 && o.io_phases != 1) {
        err = "io_phases must be 0 or 1";
        return QSV_E_INVALID;
    }
    if (o.section_kernel != QSV_KERNEL_REGISTERS && o.section_kernel != QSV_KERNEL_LDS &&
        o.section_kernel != QSV_KERNEL_PAIRED && o.section_kernel != QSV_KERNEL_MFMA) {
        err = "section_kernel must be QSV_KERNEL_REGISTERS, _LDS, _PAIRED or _MFMA";
        return QSV_E_INVALID;
    }
    if (o.planner < QSV_PLANNER_DEFAULT || o.planner > QSV_PLANNER_EXACT) {
        err = "planner must be one of QSV_PLANNER_DEFAULT, _GREEDY, _BEAM, _EXACT";
        return QSV_E_INVALID;
    }
    if ((o.planner == QSV_PLANNER_BEAM || o.planner == QSV_PLANNER_EXACT) &&
        o.swap_mode != QSV_SWAP_REMAP) {
        err = "beam and exact planners need swap_mode QSV_SWAP_REMAP";
        return QSV_E_UNSUPPORTED;
    }
    if (o.planner == QSV_PLANNER_EXACT && (ng > 64 || n > 24)) {
        err = "the exact planner takes at most 64 gates and 24 qubits";
        return QSV_E_UNSUPPORTED;
    }
    if (o.swap_mode != QSV_SWAP_REMAP && o.swap_mode != QSV_SWAP_MATERIALIZE) {
        err = "swap_mode must be QSV_SWAP_REMAP or QSV_SWAP_MATERIALIZE";
        return QSV_E_INVALID;
    }
    if (o.fusion_max_qubits < 0 || o.fusion_max_qubits > 5) {
        err = "fusion_max_qubits must be in [0, 5]";
        return QSV_E_INVALID;
    }
    size_t bytes_per_amp = dt == QSV_C64 ? 8 : 16;
    if ((size_t(1) << std::min(o.chunk_bits, n)) * bytes_per_amp > 128 * 1024) {
        err = "chunk of 2^chunk_bits amplitudes exceeds 128 KiB of LDS";
        return QSV_E_INVALID;
    }
    P = Plan();
    P.n = n;
    P.dtype = dt;
    {
        const qsv_status vs = validate_and_build(n, g, ng, P.gates, P.n_params, err);
        if (vs != QSV_OK) return vs;
    }
    int maxk = 1;
    for (const GateRec &r : P.gates)
        if (!r.diagonal && !r.is_swap && r.kind != QSV_CX) maxk = std::max(maxk, r.nq);
    P.c = std::min(o.chunk_bits, n);
    // a dense gate must fit in one thread's registers
    P.r = std::min(std::max(o.register_bits, maxk), P.c);
    if (maxk > P.c) {
        err = "a gate acts on more qubits than the chunk holds";
        return QSV_E_INVALID;
    }
    if (lds_resident(o)) {
        // the whole chunk is one register phase: op positions are LDS index bits
        const bool mfma = o.section_kernel == QSV_KERNEL_MFMA;
        if (P.n_params > 0) {
            err = "the LDS-resident section kernel takes no bound parameters";
            return QSV_E_UNSUPPORTED;
        }
        if (maxk > (mfma ? 5 : 4)) {
            err = mfma ? "the MFMA section kernel applies dense gates of at most 5 qubits"
                       : "the LDS-resident section kernel applies dense gates of at most 4 qubits";
            return QSV_E_UNSUPPORTED;
        }
        if (mfma && P.c < 9) {
            // a 5-qubit op needs at least one tile of 16 amplitude groups
            err = "the MFMA section kernel needs chunk_bits >= 9";
            return QSV_E_UNSUPPORTED;
        }
        if (n - P.c + std::min(P.c, 9) > 31) {
            err = "n - chunk_bits too large for the LDS-resident kernel's launch grid";
            return QSV_E_UNSUPPORTED;
        }
        P.r = P.c;
    }
    if (o.section_kernel == QSV_KERNEL_PAIRED) {
        // paired phases hold two gate pairs in registers: 4 register bits
        if (P.c < 4 || maxk > 4) {
            err = "paired phases need chunk_bits >= 4 and gates of at most 4 qubits";
            return QSV_E_UNSUPPORTED;
        }
        P.r = 4;
    }
    if (!lds_resident(o) && P.c - P.r > (P.r <= 4 ? 9 : 8)) {
        err = "chunk_bits - register_bits must be <= 9 for register_bits <= 4 and <= 8 for "
              "register_bits = 5 (512 / 256 threads per workgroup)";
        return QSV_E_INVALID;
    }
    if (n - P.r > 31 || n - P.c > 30) {
        // a section launch has 2^(n - c) workgroups of 2^(c - r) work-items: at
        // most 2^31 - 1 workgroups and 2^32 - 1 work-items per grid dimension
        err = "n - register_bits must be <= 31 and n - chunk_bits <= 30 (launch grid limits)";
        return QSV_E_UNSUPPORTED;
    }
    int maxlocal = 1;
    for (const GateRec &r : P.gates) maxlocal = std::max(maxlocal, r.nq);
    if (o.pinned_low_bits > P.c - maxlocal) o.pinned_low_bits = std::max(0, P.c - maxlocal);
    if (o.pinned_low_bits > n) o.pinned_low_bits = n;
    o.register_bits = P.r;
    o.chunk_bits = P.c;
    P.opt = o;
    // fused ops run in one thread's registers: at most r qubits, and at most 4
    // (the widest fused-op kernel instance); on the matrix cores up to 5
    const int fmax = o.section_kernel == QSV_KERNEL_MFMA ? 5 : 4;
    P.fusion_eff = o.fusion_max_qubits < 2 ? o.fusion_max_qubits : std::min(o.fusion_max_qubits, std::min(P.r, fmax));
    if (lds_resident(o)) o.io_phases = 0, P.opt.io_phases = 0;

    if (!block_circuit(P)) {
        err = "the exact planner's search exceeded its state budget (use a smaller circuit or "
              "another planner)";
        return QSV_E_UNSUPPORTED;
    }
    for (size_t s = 0; s < P.sections.size(); ++s) {
        if (o.section_kernel == QSV_KERNEL_PAIRED && paired_eligible(P, P.sections[s]))
            lower_section_paired(P, (int)s);
        else
            lower_section(P, (int)s);
    }
    lower_per_gate(P);
    P.poff.assign(P.n_params + 1, 0);
    for (const PSlot &ps : P.pslots) P.poff[ps.param + 1]++;
    for (int64_t q = 0; q < P.n_params; ++q) P.poff[q + 1] += P.poff[q];
    P.plist.assign(P.pslots.size(), 0);
    {
        std::vector<int32_t> fill(P.poff.begin(), P.poff.end() - 1);
        for (size_t k = 0; k < P.pslots.size(); ++k) P.plist[fill[P.pslots[k].param]++] = (int32_t)k;
    }
    P.uid = g_plan_uid.fetch_add(1);
    return QSV_OK;
}

}  // namespace qsv
