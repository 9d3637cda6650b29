// Section kernel with the chunk resident in LDS for the whole section.
//
// One workgroup owns one chunk of 2^c amplitudes (Sec. II-B; the chunk of a
// blocked section, Sec. IV-C).  It gathers the chunk from HBM into LDS once,
// applies every op of the section there, and scatters it back once: the
// paper's "one read and one write of the state per section", with the
// workgroup's LDS as the cache.  Unlike the register-phase kernel, an op's
// qubits are plain bit positions of the LDS index (runtime values), so no
// kernel code depends on which qubits an op touches: each thread takes whole
// amplitude groups of the op (the pair-wise update of Sec. II-A generalised to
// 2^k members), reads them from LDS, applies the matrix in registers and
// writes them back; a barrier separates consecutive ops.  Fused blocks of 4
// and 5 qubits can instead run on the matrix cores (lds_mfma).
//
// LDS index bits are the section's data positions (ascending chunk slots at the
// start, relabelled by in-section SWAP gates); the LDS address is the index
// under a GF(2)-linear swizzle (XOR of index bits into the bank-selecting low
// bits), so every address is a per-lane part XOR a uniform part.
#include <algorithm>

#include "section_core.hpp"

namespace qsv {

using namespace sec;

namespace {

constexpr int LDS_THREADS = 512;

// element swizzle of a 16- or 8-byte LDS element index (GF(2)-linear)
template <typename V> __device__ __forceinline__ uint32_t swz(uint32_t i) {
    return lds_swizzle<(int)sizeof(V)>(i);
}

// bits of x deposited at the positions of `pos` (pos[j] = destination bit of bit j)
__device__ __forceinline__ uint32_t deposit(uint32_t x, const Bytes16 &pos, uint32_t nbits) {
    uint32_t out = 0;
    for (uint32_t j = 0; j < nbits; ++j) out |= ((x >> j) & 1u) << pos[j];
    return out;
}

// x with a zero bit inserted at each position of mask (ascending, uniform)
__device__ __forceinline__ uint32_t insert_zeros(uint32_t x, uint32_t mask) {
    while (mask) {
        const uint32_t low = mask & (0u - mask);   // lowest set bit
        x = ((x & ~(low - 1u)) << 1) | (x & (low - 1u));
        mask &= mask - 1u;
    }
    return x;
}

// dense 2^K x 2^K matrix on LDS index bits a[0] < ... < a[K-1]
template <typename V, int K>
__device__ __forceinline__ void lds_dense(V *lds, const uint32_t (&a)[5], cptr<V> m, uint32_t c,
                                          unsigned tid, unsigned nthr) {
    constexpr int D = 1 << K;
    uint32_t amask = 0;
    for (int j = 0; j < K; ++j) amask |= 1u << a[j];
    const uint32_t groups = 1u << (c - K);
    // member offsets (uniform): bit j of L at position a[j]
    uint32_t moff[D];
    for (int L = 0; L < D; ++L) {
        uint32_t o = 0;
        for (int j = 0; j < K; ++j) o |= ((uint32_t)(L >> j) & 1u) << a[j];
        moff[L] = swz<V>(o);
    }
    for (uint32_t g = tid; g < groups; g += nthr) {
        const uint32_t b = swz<V>(insert_zeros(g, amask));
        V in[D];
        static_for<D>([&](auto L) __attribute__((always_inline)) { in[L.value] = lds[b ^ moff[L.value]]; });
        static_for<D>([&](auto ROW) __attribute__((always_inline)) {
            V acc;
            acc.x = 0;
            acc.y = 0;
            static_for<D>([&](auto L) __attribute__((always_inline)) {
                acc = cfma(ldc(m + (ROW.value * D + L.value)), in[L.value], acc);
            });
            lds[b ^ moff[ROW.value]] = acc;
        });
    }
}

// MFMA 16x16x4 blocks (one instruction per element type).  A and B take one
// element per lane, C and D four: A[i][k] sits in lane i + 16 k and B[k][j] in
// lane j + 16 k; lane l holds, as its element v, D[4 (l / 16) + v][l % 16] for
// float and D[l / 16 + 4 v][l % 16] for double (both measured on gfx950).
typedef double D4 __attribute__((ext_vector_type(4)));
typedef float F4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ D4 mfma16(double a, double b, D4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ F4 mfma16(float a, float b, F4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Dense 2^K x 2^K op (K = 4, 5: a fused block of gates) on LDS index bits
// a[0] < ... < a[K-1], as a matrix product on the matrix cores: with the
// chunk's 2^(c-K) amplitude groups as the columns of X (row = the group
// member, bits at a[]), Y = U X.  The complex product is four real ones,
// Yr = Ur Xr - Ui Xi and Yi = Ui Xr + Ur Xi, each built from 16x16x4 blocks:
// 16 rows of U by 4 members by 16 groups.  A wave owns tiles of 16 groups;
// it loads all 2^K members of its 16 groups from LDS (B operands: lane j + 16 k
// takes member 4 s + k of group j at step s), runs the (2^K / 16) x (2^K / 4)
// x 4 blocks, and writes the results in place (D of row tile t: member
// 16 t + 4 (l / 16) + v, or 16 t + l / 16 + 4 v for double, of group l % 16).
// Every group belongs to one wave, so the op needs no barrier
// inside; the caller's barrier separates it from the next op.  Needs c >= K + 4.
template <typename V, int K>
__device__ __forceinline__ void lds_mfma(V *lds, const uint32_t (&a)[5], cptr<V> m, uint32_t c,
                                         unsigned tid, unsigned nthr) {
    using E = decltype(V{}.x);
    typedef E E4 __attribute__((ext_vector_type(4)));
    constexpr int D = 1 << K, RT = D / 16, KS = D / 4;
    constexpr bool F64 = sizeof(E) == 8;  // output row order of the double instruction
    const uint32_t lane = tid & 63u, li = lane & 15u, lk = lane >> 4;
    const uint32_t wave = tid >> 6, nwaves = nthr >> 6;
    uint32_t amask = 0;
    for (int j = 0; j < K; ++j) amask |= 1u << a[j];
    auto dep = [&](uint32_t r) {  // member index -> LDS index bits
        uint32_t o = 0;
        for (int j = 0; j < K; ++j) o |= ((r >> j) & 1u) << a[j];
        return o;
    };
    // lane bits 4-5 give member bits 0-1 of a B element, and bits 2-3 (float) or
    // 0-1 (double) of a D element
    const uint32_t in_lane = swz<V>(dep(lk)), out_lane = swz<V>(dep(F64 ? lk : 4u * lk));
    const uint32_t ntiles = 1u << (c - K - 4);
    for (uint32_t t = wave; t < ntiles; t += nwaves) {
        const uint32_t gb = swz<V>(insert_zeros(t * 16u + li, amask));
        V x[KS];
        static_for<KS>([&](auto S) __attribute__((always_inline)) {
            x[S.value] = lds[gb ^ in_lane ^ swz<V>(dep(4u * S.value))];
        });
        static_for<RT>([&](auto T) __attribute__((always_inline)) {
            E4 yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
            static_for<KS>([&](auto S) __attribute__((always_inline)) {
                const V u = ldc(m + ((T.value * 16 + li) * D + 4 * S.value + lk));
                yr = mfma16(u.x, x[S.value].x, yr);
                yr = mfma16(-u.y, x[S.value].y, yr);
                yi = mfma16(u.y, x[S.value].x, yi);
                yi = mfma16(u.x, x[S.value].y, yi);
            });
            static_for<4>([&](auto W) __attribute__((always_inline)) {
                V y;
                y.x = yr[W.value];
                y.y = yi[W.value];
                lds[gb ^ out_lane ^ swz<V>(dep(16u * T.value + (F64 ? 4u * W.value : W.value)))] = y;
            });
        });
    }
}

// KMAX: widest dense op applied on the vector units.  MFMA: dense ops of 4
// and 5 qubits go to the matrix cores.  At most 128 registers per lane, so
// that two 512-thread workgroups (two 64 KiB chunks) share a compute unit.
template <typename T, int KMAX, bool MFMA>
__global__ void __launch_bounds__(LDS_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
k_section_lds(typename Amp<T>::V *__restrict__ state, int n, const DevSection *__restrict__ secs_g,
              int sec, const DevPhase *__restrict__ phases_g, const DevOp *__restrict__ ops_g,
              const typename Amp<T>::V *__restrict__ mats_g) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *lds = reinterpret_cast<V *>(lds_raw);
    const cptr<DevSection> S = (cptr<DevSection>)secs_g + sec;
    const cptr<DevPhase> PH = (cptr<DevPhase>)phases_g + S->phase_begin;
    const cptr<DevOp> ops = (cptr<DevOp>)ops_g;
    const cptr<V> mats = (cptr<V>)mats_g;
    const uint32_t c = S->c;
    const uint32_t N = 1u << c;
    const unsigned tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t tbits = 31 - __builtin_clz(nthr);     // nthr is a power of two
    const uint64_t base = chunk_base(S, blockIdx.x);
    V *st = state + ((uint64_t)blockIdx.y << n);

    // gather: LDS index i = tid + j * nthr; its physical offset is the deposit of
    // the thread bits (per lane) OR that of the j bits (uniform)
    {
        const Bytes16 g = ld16(S->gather_phys);
        uint64_t toff = 0;
        for (uint32_t b = 0; b < tbits && b < c; ++b) toff |= (uint64_t)((tid >> b) & 1u) << g[b];
        const uint32_t tsw = swz<V>(tid);
        const uint32_t per = N > nthr ? (N >> tbits) : 1u;
        if (tid < N)
            for (uint32_t j = 0; j < per; ++j) {
                uint64_t joff = 0;
                for (uint32_t b = tbits; b < c; ++b) joff |= (uint64_t)((j >> (b - tbits)) & 1u) << g[b];
                lds[tsw ^ swz<V>(j << tbits)] = st[base | toff | joff];
            }
    }
    __syncthreads();

    const uint32_t o_end = PH->op_end;
    for (uint32_t o = PH->op_begin; o < o_end; ++o) {
        const OpH op = load_op(ops + o);
        uint32_t a[5] = {op.a[0], op.a[1], op.a[2], op.a[3], op.a[4]};
        if (op.type == OP_DENSE) {
            const cptr<V> mm = mats + op.arg;
            switch (op.k) {
                case 1: lds_dense<V, 1>(lds, a, mm, c, tid, nthr); break;
                case 2: lds_dense<V, 2>(lds, a, mm, c, tid, nthr); break;
                case 3: if constexpr (KMAX >= 3) lds_dense<V, 3>(lds, a, mm, c, tid, nthr); break;
                case 4:
                    if constexpr (MFMA) lds_mfma<V, 4>(lds, a, mm, c, tid, nthr);
                    else if constexpr (KMAX >= 4) lds_dense<V, 4>(lds, a, mm, c, tid, nthr);
                    break;
                case 5: if constexpr (MFMA) lds_mfma<V, 5>(lds, a, mm, c, tid, nthr); break;
                default: break;
            }
        } else if (op.type == OP_DIAG) {
            // diagonal over its k bit sources (LDS index bits or the chunk's global bits)
            const cptr<V> tab = mats + op.arg;
            // (fixed-length loops keep the tables in registers)
            uint32_t gsel = 0, lmask[5];
            static_for<5>([&](auto J) __attribute__((always_inline)) {
                const uint32_t s = a[J.value];
                const bool on = J.value < (int)op.k;
                lmask[J.value] = (!on || s >= SRC_GLOBAL) ? 0u : (1u << s);
                if (on && s >= SRC_GLOBAL) gsel |= (uint32_t)((base >> (s - SRC_GLOBAL)) & 1ull) << J.value;
            });
            for (uint32_t i = tid; i < N; i += nthr) {
                uint32_t sel = gsel;
                static_for<5>([&](auto J) __attribute__((always_inline)) {
                    sel |= ((i & lmask[J.value]) != 0 ? 1u : 0u) << J.value;
                });
                const uint32_t ad = swz<V>(i);
                lds[ad] = cmul(ldc(tab + sel), lds[ad]);
            }
        } else if (op.type == OP_XREG || op.type == OP_CX) {
            // X on bit a[0], controlled (OP_CX) by source a[1]: swap the pairs whose control is set
            const uint32_t t = 1u << a[0];
            const uint32_t cs = op.type == OP_CX ? a[1] : 0u;
            const bool gctl = op.type == OP_CX && cs >= SRC_GLOBAL;
            const bool gon = gctl ? ((base >> (cs - SRC_GLOBAL)) & 1ull) != 0 : true;
            const uint32_t cm = (op.type == OP_CX && !gctl) ? (1u << cs) : 0u;
            if (gon) {
                for (uint32_t g = tid; g < (N >> 1); g += nthr) {
                    const uint32_t i0 = insert_zeros(g, t);
                    if (cm && !(i0 & cm)) continue;
                    const uint32_t p0 = swz<V>(i0), p1 = swz<V>(i0 | t);
                    const V x0 = lds[p0], x1 = lds[p1];
                    lds[p0] = x1;
                    lds[p1] = x0;
                }
            }
        }
        __syncthreads();
    }

    // scatter through the section's final position -> physical map
    {
        const Bytes16 g = ld16(S->scatter_phys);
        uint64_t toff = 0;
        for (uint32_t b = 0; b < tbits && b < c; ++b) toff |= (uint64_t)((tid >> b) & 1u) << g[b];
        const uint32_t tsw = swz<V>(tid);
        const uint32_t per = N > nthr ? (N >> tbits) : 1u;
        if (tid < N)
            for (uint32_t j = 0; j < per; ++j) {
                uint64_t joff = 0;
                for (uint32_t b = tbits; b < c; ++b) joff |= (uint64_t)((j >> (b - tbits)) & 1u) << g[b];
                st[base | toff | joff] = lds[tsw ^ swz<V>(j << tbits)];
            }
    }
}

template <typename T, int KMAX, bool MFMA>
hipError_t launch_lds_t(void *state, int n, int batch, DevPlanView pv, int sec, int c, hipStream_t s) {
    using V = typename Amp<T>::V;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_section_lds<T, KMAX, MFMA>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t lds = (size_t(1) << c) * sizeof(V);
    if (lds > 160 * 1024 || (MFMA && c < 9)) return hipErrorInvalidConfiguration;
    const unsigned threads = (unsigned)std::min<uint64_t>(LDS_THREADS, std::max<uint64_t>(64, 1ull << c));
    dim3 grid((unsigned)(1ull << (n - c)), (unsigned)batch);
    hipLaunchKernelGGL((k_section_lds<T, KMAX, MFMA>), grid, dim3(threads), lds, s, (V *)state, n, pv.secs,
                       sec, pv.phases, pv.ops, (const V *)pv.mats);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_section_lds(qsv_dtype dt, int kmax, bool mfma, void *state, int n, int batch,
                              DevPlanView pv, int sec, int c, hipStream_t s) {
    if (dt == QSV_C128) {
        if (mfma) return launch_lds_t<double, 3, true>(state, n, batch, pv, sec, c, s);
        if (kmax <= 2) return launch_lds_t<double, 2, false>(state, n, batch, pv, sec, c, s);
        return launch_lds_t<double, 4, false>(state, n, batch, pv, sec, c, s);
    }
    if (mfma) return launch_lds_t<float, 3, true>(state, n, batch, pv, sec, c, s);
    if (kmax <= 2) return launch_lds_t<float, 2, false>(state, n, batch, pv, sec, c, s);
    return launch_lds_t<float, 4, false>(state, n, batch, pv, sec, c, s);
}

}  // namespace qsv
