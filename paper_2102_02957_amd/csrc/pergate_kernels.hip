// Per-gate kernels: the unblocked path, one launch and one pass over the state
// per gate (the baseline of Sec. V-A).  Amplitude pairs are formed as in
// Sec. II-A (Fig. "u3_gate"): the group index g is widened by inserting a zero
// bit at every target qubit, then the 2^k members of the group differ only in
// those bits.  64-bit indices throughout (a 33-qubit state has 2^33 entries).
#include "device.hpp"

namespace qsv {

namespace {

template <typename V> __device__ __forceinline__ V cmul(V m, V x) {
    V r;
    r.x = m.x * x.x - m.y * x.y;
    r.y = m.x * x.y + m.y * x.x;
    return r;
}

__device__ __forceinline__ uint64_t insert_zero(uint64_t g, int q) {
    uint64_t low = g & ((1ull << q) - 1);
    return ((g - low) << 1) | low;
}

struct QList { uint8_t q[5]; uint8_t k; };

template <typename V, int K>
__global__ void __launch_bounds__(256)
k_pg_dense(V *__restrict__ st, uint64_t ngroups, QList ql, const V *__restrict__ m) {
    constexpr int D = 1 << K;
    // K <= 2: the matrix lives in registers; larger ones are read through the
    // scalar cache (uniform addresses)
    V mm[K <= 2 ? D * D : 1];
    if constexpr (K <= 2) {
#pragma unroll
        for (int e = 0; e < D * D; ++e) mm[e] = m[e];
    }
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ngroups; g += stride) {
        uint64_t b = g;
#pragma unroll
        for (int j = 0; j < K; ++j) b = insert_zero(b, ql.q[j]);  // q ascending
        uint64_t idx[D];
        V in[D];
#pragma unroll
        for (int l = 0; l < D; ++l) {
            uint64_t o = 0;
#pragma unroll
            for (int j = 0; j < K; ++j) o |= (uint64_t)((l >> j) & 1) << ql.q[j];
            idx[l] = b | o;
            in[l] = st[idx[l]];
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int l = 0; l < D; ++l) {
                const V e = (K <= 2) ? mm[(K <= 2) ? r * D + l : 0] : m[r * D + l];
                acc.x = fma(e.x, in[l].x, acc.x);
                acc.x = fma(-e.y, in[l].y, acc.x);
                acc.y = fma(e.x, in[l].y, acc.y);
                acc.y = fma(e.y, in[l].x, acc.y);
            }
            st[idx[r]] = acc;
        }
    }
}

// 1q diagonal on every amplitude (rz): full pass
template <typename V>
__global__ void __launch_bounds__(256)
k_pg_diag1(V *__restrict__ st, uint64_t total, int q, V d0, V d1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
        st[i] = cmul(((i >> q) & 1) ? d1 : d0, st[i]);
}

// phase on the amplitudes with all bits in `mask` set (z/s/t/p: 1 bit; cz/cp: 2 bits)
template <typename V>
__global__ void __launch_bounds__(256)
k_pg_phase(V *__restrict__ st, uint64_t count, int qa, int qb, uint64_t mask, V d) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        uint64_t i = insert_zero(g, qa);
        if (qb >= 0) i = insert_zero(i, qb);
        i |= mask;
        st[i] = cmul(d, st[i]);
    }
}

// exchange amplitude i (bits of `set0` clear except those in `fix`) with i ^ flip:
//   X:    groups insert qa,           i,       i ^ (1<<qa)
//   CX:   groups insert c, t; i |= c, i,       i ^ (1<<t)
//   SWAP: groups insert a, b; i |= a, i,       i ^ a ^ b
template <typename V>
__global__ void __launch_bounds__(256)
k_pg_exchange(V *__restrict__ st, uint64_t count, int qa, int qb, uint64_t set, uint64_t flip) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        uint64_t i = insert_zero(g, qa);
        if (qb >= 0) i = insert_zero(i, qb);
        i |= set;
        uint64_t j = i ^ flip;
        V x = st[i], y = st[j];
        st[i] = y;
        st[j] = x;
    }
}

unsigned grid_for(uint64_t work) {
    uint64_t b = (work + 255) / 256;
    const uint64_t cap = 256ull * 2048;  // grid-stride beyond this
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

template <typename T>
static hipError_t pergate_t(void *state, int n, const PgOp &op, const void *mats, hipStream_t s) {
    using V = typename Amp<T>::V;
    V *st = (V *)state;
    const V *M = (const V *)mats;
    const uint64_t N = 1ull << n;
    switch (op.kind) {
        case PG_DENSE: {
            QList ql;
            for (int j = 0; j < 5; ++j) ql.q[j] = op.q[j];
            ql.k = op.k;
            uint64_t ng = N >> op.k;
            unsigned grid = grid_for(ng);
            const V *m = M + op.arg;
            switch (op.k) {
                case 1: hipLaunchKernelGGL((k_pg_dense<V, 1>), dim3(grid), dim3(256), 0, s, st, ng, ql, m); break;
                case 2: hipLaunchKernelGGL((k_pg_dense<V, 2>), dim3(grid), dim3(256), 0, s, st, ng, ql, m); break;
                case 3: hipLaunchKernelGGL((k_pg_dense<V, 3>), dim3(grid), dim3(256), 0, s, st, ng, ql, m); break;
                case 4: hipLaunchKernelGGL((k_pg_dense<V, 4>), dim3(grid), dim3(256), 0, s, st, ng, ql, m); break;
                case 5: hipLaunchKernelGGL((k_pg_dense<V, 5>), dim3(grid), dim3(256), 0, s, st, ng, ql, m); break;
                default: return hipErrorInvalidValue;
            }
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Host-side values for the diagonal / phase kernels are passed as arguments,
// so the launcher takes them from the plan's host copy.
template <typename T>
static hipError_t pergate_host_t(void *state, int n, const PgOp &op, const cd *hmats,
                                 const void *dmats, hipStream_t s) {
    using V = typename Amp<T>::V;
    V *st = (V *)state;
    const uint64_t N = 1ull << n;
    auto cv = [](cd z) {
        V v;
        v.x = (T)z.real();
        v.y = (T)z.imag();
        return v;
    };
    switch (op.kind) {
        case PG_DENSE:
            return pergate_t<T>(state, n, op, dmats, s);
        case PG_DIAG1: {
            uint64_t total = N;
            hipLaunchKernelGGL((k_pg_diag1<V>), dim3(grid_for(total)), dim3(256), 0, s, st, total,
                               (int)op.q[0], cv(hmats[op.arg]), cv(hmats[op.arg + 1]));
            break;
        }
        case PG_PHASE1: {
            uint64_t cnt = N >> 1;
            hipLaunchKernelGGL((k_pg_phase<V>), dim3(grid_for(cnt)), dim3(256), 0, s, st, cnt,
                               (int)op.q[0], -1, 1ull << op.q[0], cv(hmats[op.arg]));
            break;
        }
        case PG_CPHASE: {
            int a = op.q[0] < op.q[1] ? op.q[0] : op.q[1];
            int b = op.q[0] < op.q[1] ? op.q[1] : op.q[0];
            uint64_t cnt = N >> 2;
            hipLaunchKernelGGL((k_pg_phase<V>), dim3(grid_for(cnt)), dim3(256), 0, s, st, cnt, a, b,
                               (1ull << a) | (1ull << b), cv(hmats[op.arg]));
            break;
        }
        case PG_X: {
            uint64_t cnt = N >> 1;
            hipLaunchKernelGGL((k_pg_exchange<V>), dim3(grid_for(cnt)), dim3(256), 0, s, st, cnt,
                               (int)op.q[0], -1, 0ull, 1ull << op.q[0]);
            break;
        }
        case PG_CX: {
            int c = op.q[0], t = op.q[1];
            int a = c < t ? c : t, b = c < t ? t : c;
            uint64_t cnt = N >> 2;
            hipLaunchKernelGGL((k_pg_exchange<V>), dim3(grid_for(cnt)), dim3(256), 0, s, st, cnt, a, b,
                               1ull << c, 1ull << t);
            break;
        }
        case PG_SWAP: {
            int a = op.q[0] < op.q[1] ? op.q[0] : op.q[1];
            int b = op.q[0] < op.q[1] ? op.q[1] : op.q[0];
            uint64_t cnt = N >> 2;
            hipLaunchKernelGGL((k_pg_exchange<V>), dim3(grid_for(cnt)), dim3(256), 0, s, st, cnt, a, b,
                               1ull << a, (1ull << a) | (1ull << b));
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pergate_host(qsv_dtype dt, void *state, int n, const PgOp &op, const cd *hmats,
                               const void *dmats, hipStream_t s) {
    if (dt == QSV_C128) return pergate_host_t<double>(state, n, op, hmats, dmats, s);
    return pergate_host_t<float>(state, n, op, hmats, dmats, s);
}

}  // namespace qsv
