// Adjoint gradient of E(theta) = <psi|H|psi>, psi = U_G(theta) ... U_1(theta)|0>,
// H a sum of Z-strings, for a batch of parameter vectors.
//
// forward : psi = blocked apply of the parameterised plan (qsv_apply_params path)
// energy  : E = sum_x |psi_x|^2 h(x)                       (FP64 reduction)
// lambda  : lambda = H psi                                  (diagonal, one pass)
// reverse : the blocked plan walked backwards, one kernel per section holding
//           the psi and lambda chunks; per op j in reverse order
//               psi    <- U_j^dag psi       (psi is now psi_{j-1})
//               grad_j += 2 Re <lambda| dU_j/dtheta |psi_{j-1}>   (parameterised ops)
//               lambda <- U_j^dag lambda
//           per-chunk partials are written per (state, parameterised op, chunk)
// reduce  : partials -> per-op sums -> grad[b][p] (sum over the ops driven by p),
//           all in fixed order (deterministic).
#include <algorithm>
#include <vector>

#include "section_core.hpp"

namespace qsv {

using namespace sec;

namespace {

// dense 2^K x 2^K conjugate transpose (row-major m) on register positions P...
template <typename V, int R, int... P>
__device__ __forceinline__ void dense_apply_adj(V (&a)[1 << R], cptr<V> m) {
    constexpr int D = 1 << sizeof...(P);
    static_for<(1 << (R - (int)sizeof...(P)))>([&](auto G) __attribute__((always_inline)) {
        constexpr int b = dep_rest<R, P...>(G.value);
        V in[D];
        static_for<D>([&](auto L) __attribute__((always_inline)) { in[L.value] = a[b | dep_pos<P...>(L.value)]; });
        static_for<D>([&](auto ROW) __attribute__((always_inline)) {
            V acc;
            acc.x = 0;
            acc.y = 0;
            static_for<D>([&](auto L) __attribute__((always_inline)) {
                V e = ldc(m + (L.value * D + ROW.value));
                e.y = -e.y;
                acc = cfma(e, in[L.value], acc);
            });
            a[b | dep_pos<P...>(ROW.value)] = acc;
        });
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <typename V, int R, int P0 = 0>
__device__ __forceinline__ void adj1(V (&a)[1 << R], int a0, cptr<V> m) {
    if constexpr (P0 < R) {
        if (a0 == P0) dense_apply_adj<V, R, P0>(a, m);
        else adj1<V, R, P0 + 1>(a, a0, m);
    }
}
template <typename V, int R, int P0 = 0, int P1 = 1>
__device__ __forceinline__ void adj2(V (&a)[1 << R], int a0, int a1, cptr<V> m) {
    if constexpr (P0 < R - 1) {
        if constexpr (P1 < R) {
            if (a0 == P0 && a1 == P1) dense_apply_adj<V, R, P0, P1>(a, m);
            else adj2<V, R, P0, P1 + 1>(a, a0, a1, m);
        } else {
            adj2<V, R, P0 + 1, P0 + 2>(a, a0, a1, m);
        }
    }
}

// 2 Re sum conj(lam) (dU psi) for a 1-qubit matrix dU on register position P
template <typename V, int R, int P>
__device__ __forceinline__ double dgrad1(const V (&psi)[1 << R], const V (&lam)[1 << R], V d00,
                                         V d01, V d10, V d11) {
    double acc = 0.0;
    static_for<(1 << (R - 1))>([&](auto G) __attribute__((always_inline)) {
        constexpr int i0 = dep_rest<R, P>(G.value), i1 = i0 | (1 << P);
        const V v0 = cfma(d01, psi[i1], cmul(d00, psi[i0]));
        const V v1 = cfma(d11, psi[i1], cmul(d10, psi[i0]));
        acc += (double)lam[i0].x * v0.x + (double)lam[i0].y * v0.y;
        acc += (double)lam[i1].x * v1.x + (double)lam[i1].y * v1.y;
    });
    return 2.0 * acc;
}
template <typename V, int R, int P = 0>
__device__ __forceinline__ double dgrad1_dispatch(const V (&psi)[1 << R], const V (&lam)[1 << R],
                                                  int a0, V d00, V d01, V d10, V d11) {
    if constexpr (P < R) {
        if (a0 == P) return dgrad1<V, R, P>(psi, lam, d00, d01, d10, d11);
        return dgrad1_dispatch<V, R, P + 1>(psi, lam, a0, d00, d01, d10, d11);
    }
    return 0.0;
}

// inverse of one forward op, applied to the registers
template <typename T, int R, int KMAX>
__device__ __forceinline__ void op_inverse(typename Amp<T>::V (&a)[1 << R], const OpH &op,
                                           cptr<typename Amp<T>::V> mats,
                                           cptr<typename Amp<T>::V> ptab, uint32_t pbase,
                                           uint64_t base) {
    using V = typename Amp<T>::V;
    constexpr int RA = 1 << R;
    const uint32_t type = op.type, k = op.k;
    if (type == OP_DENSE) {
        const cptr<V> m = mats + op.arg;
        if (k == 1) adj1<V, R>(a, op.a[0], m);
        else adj2<V, R>(a, op.a[0], op.a[1], m);
    } else if (type == OP_XREG) {
        dispatch_cx<V, R>(a, op.a[0], false, 0, pbase, 0);
    } else if (type == OP_CX) {
        const unsigned s = op.a[1];
        const unsigned gbit = s >= SRC_GLOBAL ? (unsigned)((base >> (s - SRC_GLOBAL)) & 1ull) : 0u;
        dispatch_cx<V, R>(a, op.a[0], true, s, pbase, gbit);
    } else if (type == OP_DIAG) {
        const cptr<V> tab = mats + op.arg;
        static_for<RA>([&](auto I) __attribute__((always_inline)) {
            unsigned idx = 0;
            static_for<5>([&](auto J) __attribute__((always_inline)) {
                if (J.value < k) idx |= src_bit(op.a[J.value], pbase | I.value, base) << J.value;
            });
            V d = ldc(tab + idx);
            d.y = -d.y;
            a[I.value] = cmul(d, a[I.value]);
        });
    } else if (type == OP_PROT) {
        const V cs = ldc(ptab + 2 * op.slot), sn = ldc(ptab + 2 * op.slot + 1);
        V ms;
        if (op.rot == ROT_RY) {  // RY(-t) = [[c, s], [-s, c]]
            ms.x = -sn.x;
            ms.y = 0;
            dispatch1_val<V, R>(a, op.a[0], cs, sn, ms, cs);
        } else {  // RX(-t) = [[c, i s], [i s, c]]
            V is;
            is.x = 0;
            is.y = sn.x;
            dispatch1_val<V, R>(a, op.a[0], cs, is, is, cs);
        }
    } else if (type == OP_PDIAG) {
        V d0 = ldc(ptab + 2 * op.slot), d1 = ldc(ptab + 2 * op.slot + 1);
        d0.y = -d0.y;
        d1.y = -d1.y;
        const unsigned s0 = op.a[0];
        static_for<RA>([&](auto I) __attribute__((always_inline)) {
            a[I.value] = cmul(sel(src_bit(s0, pbase | I.value, base) != 0, d1, d0), a[I.value]);
        });
    }
    (void)KMAX;
}

// 2 Re <lam| dU |psi> over the thread's registers for a parameterised op
template <typename T, int R>
__device__ __forceinline__ double op_dgrad(const typename Amp<T>::V (&psi)[1 << R],
                                           const typename Amp<T>::V (&lam)[1 << R], const OpH &op,
                                           cptr<typename Amp<T>::V> ptab, uint32_t pbase,
                                           uint64_t base) {
    using V = typename Amp<T>::V;
    constexpr int RA = 1 << R;
    const V t0 = ldc(ptab + 2 * op.slot), t1 = ldc(ptab + 2 * op.slot + 1);
    if (op.type == OP_PROT) {
        // RY: dU = 1/2 [[-s, -c], [c, -s]];  RX: dU = 1/2 [[-s, -i c], [-i c, -s]]
        const T c = t0.x * (T)0.5, s = t1.x * (T)0.5;
        V ms, d01, d10;
        ms.x = -s;
        ms.y = 0;
        if (op.rot == ROT_RY) {
            d01.x = -c; d01.y = 0;
            d10.x = c;  d10.y = 0;
        } else {
            d01.x = 0; d01.y = -c;
            d10 = d01;
        }
        return dgrad1_dispatch<V, R>(psi, lam, op.a[0], ms, d01, d10, ms);
    }
    // RZ: dU = diag(-i/2 d0, i/2 d1);  P: dU = diag(0, i d1)
    V e0, e1;
    if (op.rot == ROT_RZ) {
        e0.x = (T)0.5 * t0.y;  e0.y = (T)-0.5 * t0.x;
        e1.x = (T)-0.5 * t1.y; e1.y = (T)0.5 * t1.x;
    } else {
        e0.x = 0; e0.y = 0;
        e1.x = -t1.y; e1.y = t1.x;
    }
    const unsigned s0 = op.a[0];
    double acc = 0.0;
    static_for<RA>([&](auto I) __attribute__((always_inline)) {
        const V v = cmul(sel(src_bit(s0, pbase | I.value, base) != 0, e1, e0), psi[I.value]);
        acc += (double)lam[I.value].x * v.x + (double)lam[I.value].y * v.y;
    });
    return 2.0 * acc;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

// One section of the reverse sweep: grid = (chunks, batch).  `part` receives
// per-(state, param op, chunk) partials: part[(b * nslots + slot) * nchunks + chunk].
template <typename T, int R, int KMAX>
__global__ void __launch_bounds__(256)
k_adjoint_section(typename Amp<T>::V *__restrict__ psi_g, typename Amp<T>::V *__restrict__ lam_g,
                  int n, const DevSection *__restrict__ secs_g, int sec,
                  const DevPhase *__restrict__ phases_g, const DevOp *__restrict__ ops_g,
                  const typename Amp<T>::V *__restrict__ mats_g,
                  const typename Amp<T>::V *__restrict__ ptab_g, int nslots,
                  double *__restrict__ part) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *lds = reinterpret_cast<V *>(lds_raw);
    __shared__ double red[64];
    const unsigned tid = threadIdx.x;
    const uint64_t chunk = blockIdx.x, nchunks = gridDim.x;
    const int b = blockIdx.y;
    V *psi_st = psi_g + ((uint64_t)b << n);
    V *lam_st = lam_g + ((uint64_t)b << n);
    const cptr<V> ptab = (cptr<V>)ptab_g + (size_t)b * 2 * nslots;
    const cptr<DevSection> S = (cptr<DevSection>)secs_g + sec;
    const cptr<DevPhase> ph = (cptr<DevPhase>)phases_g + S->phase_begin;
    const cptr<DevOp> ops = (cptr<DevOp>)ops_g;
    const cptr<V> mats = (cptr<V>)mats_g;
    const int nph = (int)(S->phase_end - S->phase_begin);
    const int TB = (int)S->c - R;
    const uint64_t base = chunk_base(S, chunk);
    const uint32_t pbase = tid << R;
    const int nwaves = (int)(blockDim.x + 63) / 64;
    // per-wave gradient partials of this section's parameterised ops, after the
    // chunk's transposition area: wpart[(slot - param_slot) * nwaves + wave]
    const size_t chunk_bytes = nph > 1 ? ((sizeof(V) / 2) << S->c) : 0;
    double *wpart = reinterpret_cast<double *>(lds_raw + chunk_bytes);
    const bool whole_waves = blockDim.x >= 64;

    V psi[1 << R], lam[1 << R];
    chunk_gather<V, R>(psi, psi_st, S->scatter_phys, base, tid, TB);
    chunk_gather<V, R>(lam, lam_st, S->scatter_phys, base, tid, TB);
    for (int p = nph - 1; p >= 0; --p) {
        const cptr<DevPhase> P = ph + p;
        for (int o = (int)P->op_end - 1; o >= (int)P->op_begin; --o) {
            const OpH op = load_op(ops + o);
            op_inverse<T, R, KMAX>(psi, op, mats, ptab, pbase, base);
            if (op.type == OP_PROT || op.type == OP_PDIAG) {
                const double g = op_dgrad<T, R>(psi, lam, op, ptab, pbase, base);
                if (whole_waves) {
                    // wave sum now, cross-wave sum once per section (no barrier here)
                    const double w = wave_sum(g);
                    if ((tid & 63) == 0)
                        wpart[(size_t)(op.slot - (int32_t)S->param_slot) * nwaves + (tid >> 6)] = w;
                } else {
                    // partial wave: fixed-order sum through LDS
                    red[tid] = g;
                    __syncthreads();
                    double total = 0.0;
                    for (unsigned t = 0; t < blockDim.x; ++t) total += red[t];
                    if (tid == 0) part[((size_t)b * nslots + op.slot) * nchunks + chunk] = total;
                    __syncthreads();
                }
            }
            op_inverse<T, R, KMAX>(lam, op, mats, ptab, pbase, base);
        }
        if (p > 0) {
            // the reverse of the transposition after phase p - 1: write in its
            // read layout, read in its write layout
            const cptr<DevPhase> Q = ph + (p - 1);
            chunk_transpose<V, R>(psi, lds, P->rd, Q->wr, Q->xr, Q->xw, tid, TB, true);
            chunk_transpose<V, R>(lam, lds, P->rd, Q->wr, Q->xr, Q->xw, tid, TB, true);
        }
    }
    if (whole_waves && S->n_params_used > 0) {
        __syncthreads();
        for (uint32_t i = tid; i < S->n_params_used; i += blockDim.x) {
            double total = 0.0;
            for (int w = 0; w < nwaves; ++w) total += wpart[(size_t)i * nwaves + w];
            part[((size_t)b * nslots + S->param_slot + i) * nchunks + chunk] = total;
        }
    }
    if (S->flags & SEC_SYNC_SCATTER) gather_scatter_barrier();
    chunk_scatter<V, R>(psi, psi_st, S->gather_phys, base, tid, TB);
    chunk_scatter<V, R>(lam, lam_st, S->gather_phys, base, tid, TB);
}

// lambda = h(x) psi for a Z-string observable (batch over blockIdx.y)
template <typename V>
__global__ void __launch_bounds__(256)
k_apply_zsum(const V *__restrict__ psi, V *__restrict__ lam, int n,
             const qsv_zterm *__restrict__ terms, int nt) {
    const uint64_t N = 1ull << n;
    const V *p = psi + ((uint64_t)blockIdx.y << n);
    V *l = lam + ((uint64_t)blockIdx.y << n);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        double h = 0.0;
        for (int j = 0; j < nt; ++j) h += (__popcll(i & terms[j].zmask) & 1) ? -terms[j].coeff : terms[j].coeff;
        V v = p[i];
        v.x = (decltype(v.x))((double)v.x * h);
        v.y = (decltype(v.y))((double)v.y * h);
        l[i] = v;
    }
}

// slot sums: ssum[b * nslots + slot] = sum over chunks (chunk order)
__global__ void __launch_bounds__(256)
k_slot_sums(const double *__restrict__ part, int nslots, int batch, uint64_t nchunks,
            double *__restrict__ ssum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslots * batch) return;
    const double *p = part + (size_t)i * nchunks;
    double s = 0.0;
    for (uint64_t g = 0; g < nchunks; ++g) s += p[g];
    ssum[i] = s;
}

// grad[b * P + p] = sum of ssum over the slots driven by parameter p (slot order)
__global__ void __launch_bounds__(256)
k_param_grads(const double *__restrict__ ssum, const int32_t *__restrict__ off,
              const int32_t *__restrict__ slots, int nparams, int nslots, int batch,
              double *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nparams * batch) return;
    const int b = i / nparams, p = i % nparams;
    double s = 0.0;
    for (int k = off[p]; k < off[p + 1]; ++k) s += ssum[(size_t)b * nslots + slots[k]];
    grad[i] = s;
}

// dynamic LDS limit of the reverse-section kernel (160 KiB less its static part)
constexpr size_t ADJ_MAX_DYN_LDS = 159 * 1024;

template <typename T, int R, int KMAX>
static hipError_t adj_launch_t(void *psi, void *lam, int n, int batch, DevPlanView pv, int sec,
                               int c, size_t lds, const void *ptab, int nslots, double *part,
                               hipStream_t s) {
    using V = typename Amp<T>::V;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_adjoint_section<T, R, KMAX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           ADJ_MAX_DYN_LDS);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (c - R > 8 || c < R || lds > ADJ_MAX_DYN_LDS) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)(1ull << (n - c)), (unsigned)batch);
    hipLaunchKernelGGL((k_adjoint_section<T, R, KMAX>), grid, dim3(1u << (c - R)), lds, s,
                       (V *)psi, (V *)lam, n, pv.secs, sec, pv.phases, pv.ops, (const V *)pv.mats,
                       (const V *)ptab, nslots, part);
    return hipGetLastError();
}

hipError_t launch_adjoint_section(qsv_dtype dt, int r, void *psi, void *lam, int n, int batch,
                                  DevPlanView pv, int sec, int c, size_t lds, const void *ptab,
                                  int nslots, double *part, hipStream_t s) {
#define QSV_ADJ(T_, R_) return adj_launch_t<T_, R_, 2>(psi, lam, n, batch, pv, sec, c, lds, ptab, nslots, part, s)
    if (dt == QSV_C128) {
        switch (r) {
            case 1: QSV_ADJ(double, 1);
            case 2: QSV_ADJ(double, 2);
            case 3: QSV_ADJ(double, 3);
            case 4: QSV_ADJ(double, 4);
        }
    } else {
        switch (r) {
            case 1: QSV_ADJ(float, 1);
            case 2: QSV_ADJ(float, 2);
            case 3: QSV_ADJ(float, 3);
            case 4: QSV_ADJ(float, 4);
            case 5: QSV_ADJ(float, 5);
        }
    }
#undef QSV_ADJ
    return hipErrorInvalidValue;
}

hipError_t launch_apply_zsum(qsv_dtype dt, const void *psi, void *lam, int n, int batch,
                             const qsv_zterm *terms, int nt, hipStream_t s) {
    const uint64_t N = 1ull << n;
    dim3 grid((unsigned)std::min<uint64_t>((N + 255) / 256, 4096), batch);
    if (dt == QSV_C128)
        hipLaunchKernelGGL((k_apply_zsum<Cplx<double>>), grid, dim3(256), 0, s,
                           (const Cplx<double> *)psi, (Cplx<double> *)lam, n, terms, nt);
    else
        hipLaunchKernelGGL((k_apply_zsum<Cplx<float>>), grid, dim3(256), 0, s,
                           (const Cplx<float> *)psi, (Cplx<float> *)lam, n, terms, nt);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double *part, int nslots, int batch, uint64_t nchunks,
                              double *ssum, const int32_t *off, const int32_t *slots, int nparams,
                              double *grad, hipStream_t s) {
    const int a = nslots * batch, b = nparams * batch;
    if (a > 0)
        hipLaunchKernelGGL(k_slot_sums, dim3((a + 255) / 256), dim3(256), 0, s, part, nslots, batch,
                           nchunks, ssum);
    if (b > 0)
        hipLaunchKernelGGL(k_param_grads, dim3((b + 255) / 256), dim3(256), 0, s, ssum, off, slots,
                           nparams, nslots, batch, grad);
    return hipGetLastError();
}

}  // namespace qsv
