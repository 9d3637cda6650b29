// Device building blocks of the section kernel, shared by the blocked apply,
// the batched-trajectory kernel and the adjoint sweep.
//
// One workgroup owns one chunk of 2^c amplitudes (Sec. II-B: a chunk is the
// set of amplitudes sharing the values of the n - c non-local bits; here the
// non-local bits are arbitrary, so the chunk is gathered from HBM instead of
// being a contiguous block).  Each of the 2^(c-r) threads holds 2^r amplitudes
// in registers.  The section's gates run in "phases": during a phase r chunk
// qubits are register qubits (a gate on them touches only the thread's own
// registers: the pair-wise update of Sec. II-A, Fig. "u3_gate", done in
// registers) and the other c - r are spread over the threads.  Between phases
// the chunk is transposed through LDS.  HBM sees one read at the first phase
// and one write at the last.
//
// Data position p of an amplitude: bits 0..r-1 = register index, bits
// r..c-1 = thread index.  A phase maps positions to chunk slots (rd at its
// start, wr at its end; SWAP gates relabel positions mid-phase); a slot maps
// to a physical bit of the amplitude index.
#pragma once

#include <type_traits>
#include <utility>

#include "device.hpp"

namespace qsv {
namespace sec {


template <typename V> __device__ __forceinline__ V cmul(V m, V x) {
    V r;
    r.x = m.x * x.x - m.y * x.y;
    r.y = m.x * x.y + m.y * x.x;
    return r;
}
// Plan tables are read through the constant address space: every workgroup
// reads the same entries, so the loads become scalar (SGPR) loads even inside
// loops that contain barriers.
template <typename X> using cptr = const X __attribute__((address_space(4))) *;

template <typename V> __device__ __forceinline__ V ldc(cptr<V> p) {
    V r;
    r.x = p->x;
    r.y = p->y;
    return r;
}

// Byte tables in constant memory are read a dword at a time: scalar loads have
// no byte form, and a byte load would go through the vector memory pipeline
// (with a wait on every outstanding vector load before the byte is usable).
struct Bytes16 {
    uint32_t w[4];
    __device__ __forceinline__ uint32_t operator[](int i) const {
        return (w[i >> 2] >> ((i & 3) * 8)) & 0xffu;
    }
};
__device__ __forceinline__ Bytes16 ld16(cptr<uint8_t> p) {  // p 4-byte aligned
    const cptr<uint32_t> q = (cptr<uint32_t>)p;
    Bytes16 b;
    b.w[0] = q[0];
    b.w[1] = q[1];
    b.w[2] = q[2];
    b.w[3] = q[3];
    return b;
}

// 16-bit tables, likewise a dword at a time.
struct Half16 {
    uint32_t w[8];
    __device__ __forceinline__ uint32_t operator[](int i) const {
        return (w[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
    }
};
__device__ __forceinline__ Half16 ld16h(cptr<uint16_t> p) {  // p 4-byte aligned
    const cptr<uint32_t> q = (cptr<uint32_t>)p;
    Half16 h;
#pragma unroll
    for (int i = 0; i < 8; ++i) h.w[i] = q[i];
    return h;
}

// One in-section op, decoded from its four dwords (scalar registers).
struct OpH {
    uint32_t type, k, a[5], rot;
    int32_t arg, slot;
};
struct OpRaw {
    uint32_t w[4];
};
__device__ __forceinline__ OpRaw load_op_raw(cptr<DevOp> op) {
    const cptr<uint32_t> q = (cptr<uint32_t>)op;
    OpRaw r;
    r.w[0] = q[0];
    r.w[1] = q[1];
    r.w[2] = q[2];
    r.w[3] = q[3];
    return r;
}
__device__ __forceinline__ OpH decode_op(const OpRaw &r) {
    const uint32_t w0 = r.w[0], w1 = r.w[1];
    OpH h;
    h.type = w0 & 0xffu;
    h.k = (w0 >> 8) & 0xffu;
    h.a[0] = (w0 >> 16) & 0xffu;
    h.a[1] = w0 >> 24;
    h.a[2] = w1 & 0xffu;
    h.a[3] = (w1 >> 8) & 0xffu;
    h.a[4] = (w1 >> 16) & 0xffu;
    h.rot = w1 >> 24;
    h.arg = (int32_t)r.w[2];
    h.slot = (int32_t)r.w[3];
    return h;
}
__device__ __forceinline__ OpH load_op(cptr<DevOp> op) {
    const cptr<uint32_t> q = (cptr<uint32_t>)op;
    const uint32_t w0 = q[0], w1 = q[1];
    OpH h;
    h.type = w0 & 0xffu;
    h.k = (w0 >> 8) & 0xffu;
    h.a[0] = (w0 >> 16) & 0xffu;
    h.a[1] = w0 >> 24;
    h.a[2] = w1 & 0xffu;
    h.a[3] = (w1 >> 8) & 0xffu;
    h.a[4] = (w1 >> 16) & 0xffu;
    h.rot = w1 >> 24;
    h.arg = (int32_t)q[2];
    h.slot = (int32_t)q[3];
    return h;
}

// component-wise select (a select of whole structs becomes a select of their
// addresses, which would keep the register array in scratch memory)
template <typename V> __device__ __forceinline__ V sel(bool c, V a, V b) {
    V r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    return r;
}
template <typename V> __device__ __forceinline__ V cfma(V m, V x, V acc) {
    acc.x = fma(m.x, x.x, acc.x);
    acc.x = fma(-m.y, x.y, acc.x);
    acc.y = fma(m.x, x.y, acc.y);
    acc.y = fma(m.y, x.x, acc.y);
    return acc;
}

// compile-time loops and index helpers ---------------------------------------
// Every register index below is a constant expression, so the per-thread
// amplitude array stays in VGPRs (a runtime index would move it to scratch).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F> __device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// scatter the bits of g into the R - K register bits not among P (ascending)
template <int R, int... P> __host__ __device__ constexpr int dep_rest(int g) {
    constexpr int pos[] = {P...};
    int out = 0, t = 0;
    for (int b = 0; b < R; ++b) {
        bool in = false;
        for (int j = 0; j < (int)sizeof...(P); ++j) in = in || (pos[j] == b);
        if (!in) {
            out |= ((g >> t) & 1) << b;
            ++t;
        }
    }
    return out;
}
// scatter the bits of l into the positions P (bit j of l -> bit P_j)
template <int... P> __host__ __device__ constexpr int dep_pos(int l) {
    constexpr int pos[] = {P...};
    int out = 0;
    for (int j = 0; j < (int)sizeof...(P); ++j) out |= ((l >> j) & 1) << pos[j];
    return out;
}

// Copies a uniform complex value into VGPRs.  The empty asm hides the value's
// uniformity from the compiler, which would otherwise keep it in SGPRs.
template <typename V> __device__ __forceinline__ V to_vgpr(V u) {
    asm volatile("" : "+v"(u.x), "+v"(u.y));
    return u;
}

// dense 2^K x 2^K matrix (row-major, uniform memory) on register positions P...
// STAGE reads the matrix into VGPRs once, before the amplitude groups.  On gfx950
// an FP32 FMA with an SGPR operand issues at half the rate of one with VGPR
// operands (FP64 issue does not depend on it).  The paired kernel and the batch
// kernel stage their FP32 1- and 2-qubit matrices (up to 32 floats).  The
// section register kernels do not: measured, staging made them slower or no
// faster (at r = 5 it costs a wave per SIMD).
template <bool STAGE, typename V, int R, int... P>
__device__ __forceinline__ void dense_apply_m(V (&a)[1 << R], cptr<V> m) {
    constexpr int K = sizeof...(P);
    constexpr int D = 1 << K;
    V u[STAGE ? D * D : 1];
    if constexpr (STAGE)
        static_for<D * D>([&](auto I) __attribute__((always_inline)) { u[I.value] = to_vgpr(ldc(m + I.value)); });
    static_for<(1 << (R - K))>([&](auto G) __attribute__((always_inline)) {
        constexpr int b = dep_rest<R, P...>(G.value);
        V in[D];
        static_for<D>([&](auto L) __attribute__((always_inline)) { in[L.value] = a[b | dep_pos<P...>(L.value)]; });
        static_for<D>([&](auto ROW) __attribute__((always_inline)) {
            V acc;
            acc.x = 0;
            acc.y = 0;
            static_for<D>([&](auto L) __attribute__((always_inline)) {
                constexpr int e = ROW.value * D + L.value;
                if constexpr (STAGE) acc = cfma(u[e], in[L.value], acc);
                else acc = cfma(ldc(m + e), in[L.value], acc);
            });
            a[b | dep_pos<P...>(ROW.value)] = acc;
        });
        // one amplitude group at a time: keeps the live temporaries to one group
        __builtin_amdgcn_sched_barrier(0);
    });
}
template <typename V, int R, int... P>
__device__ __forceinline__ void dense_apply(V (&a)[1 << R], cptr<V> m) {
    dense_apply_m<false, V, R, P...>(a, m);
}

// dispatch of runtime positions (ascending) to the compile-time instances;
// STAGE as in dense_apply_m
template <typename V, int R, bool STAGE = false, int P0 = 0>
__device__ __forceinline__ void dispatch1(V (&a)[1 << R], int a0, cptr<V> m) {
    if constexpr (P0 < R) {
        if (a0 == P0) dense_apply_m<STAGE, V, R, P0>(a, m);
        else dispatch1<V, R, STAGE, P0 + 1>(a, a0, m);
    }
}
template <typename V, int R, bool STAGE = false, int P0 = 0, int P1 = 1>
__device__ __forceinline__ void dispatch2(V (&a)[1 << R], int a0, int a1, cptr<V> m) {
    if constexpr (P0 < R - 1) {
        if constexpr (P1 < R) {
            if (a0 == P0 && a1 == P1) dense_apply_m<STAGE, V, R, P0, P1>(a, m);
            else dispatch2<V, R, STAGE, P0, P1 + 1>(a, a0, a1, m);
        } else {
            dispatch2<V, R, STAGE, P0 + 1, P0 + 2>(a, a0, a1, m);
        }
    }
}
template <typename V, int R, int P0 = 0, int P1 = 1, int P2 = 2>
__device__ __forceinline__ void dispatch3(V (&a)[1 << R], int a0, int a1, int a2, cptr<V> m) {
    if constexpr (R >= 3 && P0 < R - 2) {
        if constexpr (P1 < R - 1) {
            if constexpr (P2 < R) {
                if (a0 == P0 && a1 == P1 && a2 == P2) dense_apply<V, R, P0, P1, P2>(a, m);
                else dispatch3<V, R, P0, P1, P2 + 1>(a, a0, a1, a2, m);
            } else {
                dispatch3<V, R, P0, P1 + 1, P1 + 2>(a, a0, a1, a2, m);
            }
        } else {
            dispatch3<V, R, P0 + 1, P0 + 2, P0 + 3>(a, a0, a1, a2, m);
        }
    }
}
template <typename V, int R, int P0 = 0, int P1 = 1, int P2 = 2, int P3 = 3>
__device__ __forceinline__ void dispatch4(V (&a)[1 << R], int a0, int a1, int a2, int a3,
                                          cptr<V> m) {
    if constexpr (R >= 4 && P0 < R - 3) {
        if constexpr (P1 < R - 2) {
            if constexpr (P2 < R - 1) {
                if constexpr (P3 < R) {
                    if (a0 == P0 && a1 == P1 && a2 == P2 && a3 == P3)
                        dense_apply<V, R, P0, P1, P2, P3>(a, m);
                    else
                        dispatch4<V, R, P0, P1, P2, P3 + 1>(a, a0, a1, a2, a3, m);
                } else {
                    dispatch4<V, R, P0, P1, P2 + 1, P2 + 2>(a, a0, a1, a2, a3, m);
                }
            } else {
                dispatch4<V, R, P0, P1 + 1, P1 + 2, P1 + 3>(a, a0, a1, a2, a3, m);
            }
        } else {
            dispatch4<V, R, P0 + 1, P0 + 2, P0 + 3, P0 + 4>(a, a0, a1, a2, a3, m);
        }
    }
}
// 1-qubit matrix given by value (parameterised rotations)
template <typename V, int R, int P>
__device__ __forceinline__ void apply1_val(V (&a)[1 << R], V m00, V m01, V m10, V m11) {
    static_for<(1 << (R - 1))>([&](auto G) __attribute__((always_inline)) {
        constexpr int i0 = dep_rest<R, P>(G.value), i1 = i0 | (1 << P);
        V x0 = a[i0], x1 = a[i1];
        V y0 = cmul(m00, x0), y1 = cmul(m10, x0);
        a[i0] = cfma(m01, x1, y0);
        a[i1] = cfma(m11, x1, y1);
    });
}
template <typename V, int R, int P = 0>
__device__ __forceinline__ void dispatch1_val(V (&a)[1 << R], int a0, V m00, V m01, V m10,
                                              V m11) {
    if constexpr (P < R) {
        if (a0 == P) apply1_val<V, R, P>(a, m00, m01, m10, m11);
        else dispatch1_val<V, R, P + 1>(a, a0, m00, m01, m10, m11);
    }
}

// X on register position T, optionally controlled by a bit source
template <typename V, int R, int T>
__device__ __forceinline__ void cx_apply(V (&a)[1 << R], bool has_ctl, unsigned src,
                                         uint32_t pbase, unsigned gbit) {
    static_for<(1 << (R - 1))>([&](auto G) __attribute__((always_inline)) {
        constexpr int i0 = dep_rest<R, T>(G.value), i1 = i0 | (1 << T);
        bool c = true;
        if (has_ctl) c = src >= SRC_GLOBAL ? (gbit != 0) : (((pbase | i0) >> src) & 1u) != 0;
        V x0 = a[i0], x1 = a[i1];
        a[i0] = sel(c, x1, x0);
        a[i1] = sel(c, x0, x1);
    });
}
template <typename V, int R, int T = 0>
__device__ __forceinline__ void dispatch_cx(V (&a)[1 << R], int t, bool has_ctl, unsigned src,
                                            uint32_t pbase, unsigned gbit) {
    if constexpr (T < R) {
        if (t == T) cx_apply<V, R, T>(a, has_ctl, src, pbase, gbit);
        else dispatch_cx<V, R, T + 1>(a, t, has_ctl, src, pbase, gbit);
    }
}

__device__ __forceinline__ unsigned src_bit(unsigned s, uint32_t pidx, uint64_t base) {
    return s >= SRC_GLOBAL ? (unsigned)((base >> (s - SRC_GLOBAL)) & 1ull) : ((pidx >> s) & 1u);
}

// LDS byte address (t ^ u) + base as one VALU op (v_xad_u32): t per lane, u
// uniform, base the LDS buffer's address.  Written as inline asm so that the
// byte scaling folded into t and u is not factored back out of the XOR.
__device__ __forceinline__ uint32_t lds_xad(uint32_t t, uint32_t u, uint32_t base) {
    uint32_t r;
    asm("v_xad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(t), "s"(u), "v"(base));
    return r;
}
// one LDS element (a real component or a whole amplitude) to / from an LDS
// byte address: a single access
template <typename L> __device__ __forceinline__ void lds_put(uint32_t addr, L v) {
    *(__attribute__((address_space(3))) L *)(uintptr_t)addr = v;
}
template <typename L> __device__ __forceinline__ L lds_get(uint32_t addr) {
    return *(__attribute__((address_space(3))) L *)(uintptr_t)addr;
}

// LDS bank swizzle of the index of an EB-byte element: XOR-fold the higher
// index bits into the bank-selecting low bits (128 B rows: 8 elements of 16
// bytes, 16 of 8 or 32 of 4).  The map is linear over GF(2), swz(x ^ y) =
// swz(x) ^ swz(y), so the address of every element is the thread's swizzled
// part XOR a uniform (scalar) swizzled register part.
template <int EB> __device__ __forceinline__ uint32_t lds_swizzle(uint32_t j) {
    if constexpr (EB == 16) return j ^ (((j >> 3) ^ (j >> 6) ^ (j >> 9) ^ (j >> 12)) & 7u);
    else if constexpr (EB == 8) return j ^ (((j >> 4) ^ (j >> 8) ^ (j >> 12)) & 15u);
    else return j ^ (((j >> 5) ^ (j >> 10)) & 31u);
}


// ---- chunk-level steps --------------------------------------------------------

// Gather / scatter of one chunk.  phys[p] = physical bit of data position p:
// positions [0, R) select the register, [R, R + TB) the thread.
template <typename V, int R>
__device__ __forceinline__ uint64_t thread_offset(const Bytes16 &phys, unsigned tid, int TB) {
    uint64_t toff = 0;
    static_for<9>([&](auto B) __attribute__((always_inline)) {
        if (B.value < TB) toff |= (uint64_t)((tid >> B.value) & 1u) << phys[R + B.value];
    });
    return toff;
}

template <typename V, int R>
__device__ __forceinline__ void chunk_gather(V (&a)[1 << R], const V *__restrict__ st,
                                             cptr<uint8_t> phys_tab, uint64_t base,
                                             unsigned tid, int TB) {
    const Bytes16 phys = ld16(phys_tab);
    const V *tp = st + (base | thread_offset<V, R>(phys, tid, TB));
    static_for<(1 << R)>([&](auto I) __attribute__((always_inline)) {
        uint64_t ro = 0;  // uniform
        static_for<R>([&](auto B) __attribute__((always_inline)) {
            if constexpr (((I.value >> B.value) & 1) != 0) ro |= 1ull << phys[B.value];
        });
        a[I.value] = tp[ro];
    });
}

template <typename V, int R>
__device__ __forceinline__ void chunk_scatter(const V (&a)[1 << R], V *__restrict__ st,
                                              cptr<uint8_t> phys_tab, uint64_t base,
                                              unsigned tid, int TB) {
    const Bytes16 phys = ld16(phys_tab);
    // A fresh copy of tid: otherwise the compiler computes the thread offset's
    // per-bit terms before the phase loop (or shares the gather's) and holds
    // them in VGPRs through every phase.
    unsigned t = tid;
    asm volatile("" : "+v"(t));
    V *tp = st + (base | thread_offset<V, R>(phys, t, TB));
    static_for<(1 << R)>([&](auto I) __attribute__((always_inline)) {
        uint64_t ro = 0;  // uniform
        static_for<R>([&](auto B) __attribute__((always_inline)) {
            if constexpr (((I.value >> B.value) & 1) != 0) ro |= 1ull << phys[B.value];
        });
        tp[ro] = a[I.value];
    });
}

// Between the gather and the scatter of a section flagged SEC_SYNC_SCATTER:
// every wave's loads of the chunk complete before any wave stores into it.  A
// workgroup-scope fence does not wait for outstanding vector loads, so the
// wait is explicit: s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their
// maxima, gfx9 encoding).
__device__ __forceinline__ void gather_scatter_barrier() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_s_barrier();
}

// Workgroup barrier that orders LDS accesses only: outstanding global stores
// and loads are not waited for.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS transposition from position->slot map `from` to map `to`.  SPLIT: one
// real component at a time, real parts then imaginary parts, through a buffer
// of 2^c components (half the chunk's bytes).  Compared with moving whole
// amplitudes (SPLIT = false, a buffer of the chunk's size) this adds two
// barriers per transposition and halves the LDS a workgroup holds, which lets
// three section workgroups share a CU (c = 12 complex128, c = 13 complex64)
// instead of two: for HBM-resident states the extra one hides more latency
// than the barriers cost.  Threads with active == false take part in the
// barriers only.
//
// With SPLIT the layout is the plan's: xw_tab / xr_tab give per data position
// the element-index vector of the write and the read map, the swizzle chosen
// per transposition already applied (lanes served together hit distinct
// banks for both maps).  Otherwise (from_tab / to_tab) the fixed lds_swizzle.
// Both layouts are GF(2)-linear, so every address is the thread's part XOR a
// uniform register part.
template <typename V, int R, bool SPLIT = true>
__device__ __forceinline__ void chunk_transpose(V (&a)[1 << R], V *lds, cptr<uint8_t> from_tab,
                                                cptr<uint8_t> to_tab, cptr<uint16_t> xw_tab,
                                                cptr<uint16_t> xr_tab, unsigned tid, int TB,
                                                bool active) {
    using E = decltype(V{}.x);
    typedef E __attribute__((ext_vector_type(2))) E2;
    using L = typename std::conditional<SPLIT, E, E2>::type;  // LDS element
    constexpr int EB = sizeof(L);
    static_assert(EB == 4 || EB == 8 || EB == 16, "float or double components");
    // byte offsets: thread part (per lane) ^ register part (uniform, one scalar
    // value per register bit, combined per element)
    const uint32_t lbase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)lds;
    uint32_t tws = 0, trs = 0;
    uint32_t sw[R], sr[R];
    if constexpr (SPLIT) {
        // Entries past the chunk's positions are zero and every thread of a
        // SPLIT caller has tid < 2^TB, so no bit needs a TB test.  Bits 0..5 are
        // the lane's (vector ops); bits 6..8 are the wave's (scalar ops).
        const Half16 xw = ld16h(xw_tab), xr = ld16h(xr_tab);
        static_for<6>([&](auto B) __attribute__((always_inline)) {
            if constexpr (R + B.value < 16) {
                const uint32_t on = (uint32_t)((int32_t)(tid << (31 - B.value)) >> 31);  // 0 or ~0
                tws ^= on & xw[R + B.value];
                trs ^= on & xr[R + B.value];
            }
        });
        const uint32_t wid = __builtin_amdgcn_readfirstlane(tid >> 6);
        uint32_t uw = 0, ur = 0;
        static_for<3>([&](auto B) __attribute__((always_inline)) {
            if constexpr (R + 6 + B.value < 16) {
                if ((wid >> B.value) & 1u) {
                    uw ^= xw[R + 6 + B.value];
                    ur ^= xr[R + 6 + B.value];
                }
            }
        });
        tws = (tws ^ uw) * EB;
        trs = (trs ^ ur) * EB;
        static_for<R>([&](auto B) __attribute__((always_inline)) {
            sw[B.value] = xw[B.value] * EB;
            sr[B.value] = xr[B.value] * EB;
        });
    } else {
        const Bytes16 from = ld16(from_tab), to = ld16(to_tab);
        uint32_t tw = 0, tr = 0;
        static_for<9>([&](auto B) __attribute__((always_inline)) {
            if (B.value < TB) {
                tw |= ((tid >> B.value) & 1u) << from[R + B.value];
                tr |= ((tid >> B.value) & 1u) << to[R + B.value];
            }
        });
        tws = lds_swizzle<EB>(tw) * EB;
        trs = lds_swizzle<EB>(tr) * EB;
        static_for<R>([&](auto B) __attribute__((always_inline)) {
            sw[B.value] = lds_swizzle<EB>(1u << from[B.value]) * EB;
            sr[B.value] = lds_swizzle<EB>(1u << to[B.value]) * EB;
        });
    }
    static_for<SPLIT ? 2 : 1>([&](auto H) __attribute__((always_inline)) {
        lds_barrier();  // the previous pass's reads are done before this pass writes
        if (active) {
            static_for<(1 << R)>([&](auto I) __attribute__((always_inline)) {
                uint32_t u = 0;
                static_for<R>([&](auto B) __attribute__((always_inline)) {
                    if constexpr (((I.value >> B.value) & 1) != 0) u ^= sw[B.value];
                });
                L w;
                if constexpr (SPLIT) {
                    w = H.value == 0 ? a[I.value].x : a[I.value].y;
                } else {
                    w.x = a[I.value].x;
                    w.y = a[I.value].y;
                }
                lds_put<L>(lds_xad(tws, u, lbase), w);
            });
        }
        lds_barrier();
        if (active) {
            static_for<(1 << R)>([&](auto I) __attribute__((always_inline)) {
                uint32_t u = 0;
                static_for<R>([&](auto B) __attribute__((always_inline)) {
                    if constexpr (((I.value >> B.value) & 1) != 0) u ^= sr[B.value];
                });
                const L v = lds_get<L>(lds_xad(trs, u, lbase));
                if constexpr (!SPLIT) {
                    a[I.value].x = v.x;
                    a[I.value].y = v.y;
                } else if constexpr (H.value == 0) {
                    a[I.value].x = v;
                } else {
                    a[I.value].y = v;
                }
            });
        }
    });
}

// Forward application of the ops [o_begin, o_end) of one phase to the
// registers.  pbase = thread index << R; base = the chunk's physical base index.
template <typename T, int R, int KMAX, bool DENSE_ONLY = false, bool STAGE = false>
__device__ __forceinline__ void chunk_ops(typename Amp<T>::V (&a)[1 << R], cptr<DevOp> ops,
                                          uint32_t o_begin, uint32_t o_end,
                                          cptr<typename Amp<T>::V> mats,
                                          cptr<typename Amp<T>::V> ptab, uint32_t pbase,
                                          uint64_t base) {
    using V = typename Amp<T>::V;
    constexpr int RA = 1 << R;
    if (o_begin >= o_end) return;
    // the next op's record is loaded while the current op computes (decoded
    // only when its op starts), so every op's matrix loads issue at once
    OpRaw nxt = load_op_raw(ops + o_begin);
    for (uint32_t o = o_begin; o < o_end; ++o) {
        const OpH op = decode_op(nxt);
        if (o + 1 < o_end) nxt = load_op_raw(ops + o + 1);
        const uint32_t type = op.type;
        const uint32_t k = op.k;
        if (type == OP_DENSE) {
            const cptr<V> mm = mats + op.arg;
            if (k == 1) dispatch1<V, R, STAGE>(a, op.a[0], mm);
            else if (k == 2) dispatch2<V, R, STAGE>(a, op.a[0], op.a[1], mm);
            else if constexpr (KMAX >= 3) {
                if (k == 3) dispatch3<V, R>(a, op.a[0], op.a[1], op.a[2], mm);
                else if constexpr (KMAX >= 4) {
                    if (k == 4) dispatch4<V, R>(a, op.a[0], op.a[1], op.a[2], op.a[3], mm);
                    else if constexpr (KMAX >= 5) {
                        if (op.a[0] == 0 && op.a[4] == 4) dense_apply<V, R, 0, 1, 2, 3, 4>(a, mm);
                    }
                }
            }
        } else if constexpr (DENSE_ONLY) {
            // sections flagged dense-only carry no other op
        } else if (type == OP_XREG) {
            dispatch_cx<V, R>(a, op.a[0], false, 0, pbase, 0);
        } else if (type == OP_CX) {
            const unsigned s = op.a[1];
            const unsigned gbit =
                s >= SRC_GLOBAL ? (unsigned)((base >> (s - SRC_GLOBAL)) & 1ull) : 0u;
            dispatch_cx<V, R>(a, op.a[0], true, s, pbase, gbit);
        } else if (type == OP_DIAG) {
            const cptr<V> tab = mats + op.arg;
            if (k == 1) {
                const V d0 = ldc(tab), d1 = ldc(tab + 1);
                const unsigned s0 = op.a[0];
                static_for<RA>([&](auto I) __attribute__((always_inline)) {
                    const unsigned b0 = src_bit(s0, pbase | I.value, base);
                    a[I.value] = cmul(sel(b0 != 0, d1, d0), a[I.value]);
                });
            } else if (k == 2) {
                const V d0 = ldc(tab), d1 = ldc(tab + 1), d2 = ldc(tab + 2), d3 = ldc(tab + 3);
                const unsigned s0 = op.a[0], s1 = op.a[1];
                static_for<RA>([&](auto I) __attribute__((always_inline)) {
                    const unsigned b0 = src_bit(s0, pbase | I.value, base);
                    const unsigned b1 = src_bit(s1, pbase | I.value, base);
                    const V lo = sel(b0 != 0, d1, d0), hi = sel(b0 != 0, d3, d2);
                    a[I.value] = cmul(sel(b1 != 0, hi, lo), a[I.value]);
                });
            } else {
                static_for<RA>([&](auto I) __attribute__((always_inline)) {
                    unsigned idx = 0;
                    static_for<5>([&](auto J) __attribute__((always_inline)) {
                        if (J.value < k) idx |= src_bit(op.a[J.value], pbase | I.value, base) << J.value;
                    });
                    a[I.value] = cmul(ldc(tab + idx), a[I.value]);
                });
            }
        } else if (type == OP_PROT) {
            const V cs = ldc(ptab + 2 * op.slot), sn = ldc(ptab + 2 * op.slot + 1);
            V ms;
            if (op.rot == ROT_RY) {
                ms.x = -sn.x;
                ms.y = 0;
                dispatch1_val<V, R>(a, op.a[0], cs, ms, sn, cs);
            } else {  // RX: [[c, -i s], [-i s, c]]
                ms.x = 0;
                ms.y = -sn.x;
                dispatch1_val<V, R>(a, op.a[0], cs, ms, ms, cs);
            }
        } else if (type == OP_PDIAG) {
            const V d0 = ldc(ptab + 2 * op.slot), d1 = ldc(ptab + 2 * op.slot + 1);
            const unsigned s0 = op.a[0];
            static_for<RA>([&](auto I) __attribute__((always_inline)) {
                a[I.value] = cmul(sel(src_bit(s0, pbase | I.value, base) != 0, d1, d0), a[I.value]);
            });
        }
    }
}

// Physical index of the chunk's first amplitude: the bits of the chunk id
// deposited into the non-local bits, i.e. a zero inserted at every local bit
// (slot_phys is ascending).
__device__ __forceinline__ uint64_t chunk_base(cptr<DevSection> S, uint64_t chunk) {
    const Bytes16 loc = ld16(S->slot_phys);
    const uint32_t c = S->c;
    uint64_t x = chunk;
    static_for<16>([&](auto I) __attribute__((always_inline)) {
        if (I.value < c) {
            const uint32_t l = loc[I.value];
            const uint64_t low = x & ((1ull << l) - 1ull);
            x = ((x >> l) << (l + 1)) | low;
        }
    });
    return x;
}

// All phases of one section on the registers of one chunk (no HBM traffic).
template <typename T, int R, int KMAX, bool DENSE_ONLY = false, bool SPLIT = true, bool STAGE = false>
__device__ __forceinline__ void chunk_phases(typename Amp<T>::V (&a)[1 << R], cptr<DevPhase> ph,
                                             int nph, cptr<DevOp> ops,
                                             cptr<typename Amp<T>::V> mats,
                                             cptr<typename Amp<T>::V> ptab, uint64_t base,
                                             typename Amp<T>::V *lds, int TB, bool active) {
    using V = typename Amp<T>::V;
    const unsigned tid = threadIdx.x;
    const uint32_t pbase = tid << R;
    for (int p = 0; p < nph; ++p) {
        const cptr<DevPhase> P = ph + p;
        chunk_ops<T, R, KMAX, DENSE_ONLY, STAGE>(a, ops, P->op_begin, P->op_end, mats, ptab, pbase, base);
        if (p + 1 < nph)
            chunk_transpose<V, R, SPLIT>(a, lds, P->wr, ph[p + 1].rd, P->xw, P->xr, tid, TB, active);
    }
}

// One chunk of one section, forward: gather, phases, scatter.
template <typename T, int R, int KMAX, bool DENSE_ONLY = false, bool SPLIT = true, bool STAGE = false>
__device__ __forceinline__ void run_chunk(typename Amp<T>::V *__restrict__ st,
                                          cptr<DevSection> S, cptr<DevPhase> phases,
                                          cptr<DevOp> ops, cptr<typename Amp<T>::V> mats,
                                          cptr<typename Amp<T>::V> ptab, uint64_t chunk,
                                          typename Amp<T>::V *lds, bool active) {
    using V = typename Amp<T>::V;
    const int TB = (int)S->c - R;
    const unsigned tid = threadIdx.x;
    const uint64_t base = chunk_base(S, chunk);
    const cptr<DevPhase> ph = phases + S->phase_begin;
    const int nph = (int)(S->phase_end - S->phase_begin);
    V a[1 << R];
    if (active) chunk_gather<V, R>(a, st, S->gather_phys, base, tid, TB);
    chunk_phases<T, R, KMAX, DENSE_ONLY, SPLIT, STAGE>(a, ph, nph, ops, mats, ptab, base, lds, TB, active);
    if (S->flags & SEC_SYNC_SCATTER) gather_scatter_barrier();
    if (active) chunk_scatter<V, R>(a, st, S->scatter_phys, base, tid, TB);
}

// One chunk of a paired section: every phase applies ops[2p] on register
// positions (0, 1) and ops[2p + 1] on (2, 3).  The positions are fixed, so the
// code has no run-time choice of registers and every update is in place.
template <typename T, int R>
__device__ __forceinline__ void run_chunk_paired(typename Amp<T>::V *__restrict__ st,
                                                 cptr<DevSection> S, cptr<DevPhase> phases,
                                                 cptr<DevOp> ops, cptr<typename Amp<T>::V> mats,
                                                 uint64_t chunk, typename Amp<T>::V *lds) {
    using V = typename Amp<T>::V;
    const int TB = (int)S->c - R;
    const unsigned tid = threadIdx.x;
    const uint64_t base = chunk_base(S, chunk);
    const cptr<DevPhase> ph = phases + S->phase_begin;
    const int nph = (int)(S->phase_end - S->phase_begin);
    V a[1 << R];
    chunk_gather<V, R>(a, st, S->gather_phys, base, tid, TB);
    for (int p = 0; p < nph; ++p) {
        const cptr<DevPhase> P = ph + p;
        const uint32_t o = P->op_begin;
        constexpr bool STAGE = sizeof(V) == 8;  // FP32 entries to VGPRs
        dense_apply_m<STAGE, V, R, 0, 1>(a, mats + ops[o].arg);
        dense_apply_m<STAGE, V, R, 2, 3>(a, mats + ops[o + 1].arg);
        if (p + 1 < nph)
            chunk_transpose<V, R, true>(a, lds, P->wr, ph[p + 1].rd, P->xw, P->xr, tid, TB, true);
    }
    chunk_scatter<V, R>(a, st, S->scatter_phys, base, tid, TB);
}

// sum over the thread's registers of |a|^2 in FP64
template <typename V, int R> __device__ __forceinline__ double reg_norm2(const V (&a)[1 << R]) {
    double s = 0.0;
    static_for<(1 << R)>([&](auto I) __attribute__((always_inline)) {
        s += (double)a[I.value].x * (double)a[I.value].x + (double)a[I.value].y * (double)a[I.value].y;
    });
    return s;
}

// Same as run_chunk, and also returns (in thread 0) the chunk's FP64 sum of
// |a|^2 after the section, reduced in a fixed order through `red` (blockDim.x
// doubles of LDS).
template <typename T, int R, int KMAX, bool SPLIT = true, bool STAGE = false>
__device__ __forceinline__ double run_chunk_norm(typename Amp<T>::V *__restrict__ st,
                                                 cptr<DevSection> S, cptr<DevPhase> phases,
                                                 cptr<DevOp> ops, cptr<typename Amp<T>::V> mats,
                                                 cptr<typename Amp<T>::V> ptab, uint64_t chunk,
                                                 typename Amp<T>::V *lds, double *red, bool active) {
    using V = typename Amp<T>::V;
    const int TB = (int)S->c - R;
    const unsigned tid = threadIdx.x;
    const uint64_t base = chunk_base(S, chunk);
    const cptr<DevPhase> ph = phases + S->phase_begin;
    const int nph = (int)(S->phase_end - S->phase_begin);
    V a[1 << R];
    if (active) chunk_gather<V, R>(a, st, S->gather_phys, base, tid, TB);
    chunk_phases<T, R, KMAX, false, SPLIT, STAGE>(a, ph, nph, ops, mats, ptab, base, lds, TB, active);
    if (S->flags & SEC_SYNC_SCATTER) gather_scatter_barrier();
    if (active) chunk_scatter<V, R>(a, st, S->scatter_phys, base, tid, TB);
    red[tid] = active ? reg_norm2<V, R>(a) : 0.0;
    __syncthreads();
    for (unsigned s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

}  // namespace sec
}  // namespace qsv
