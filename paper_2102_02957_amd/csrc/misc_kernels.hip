// State initialisation, copies, bit-swap permutation passes and the FP64
// reductions (norm, overlap, diagonal Z-string expectation, renormalisation).
#include <algorithm>
#include <mutex>

#include "device.hpp"

namespace qsv {

namespace {

constexpr int RED_THREADS = 256;

unsigned grid_for(uint64_t work, uint64_t cap = 256ull * 2048) {
    uint64_t b = (work + 255) / 256;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// |basis> in every one of `batch` states (Sec. IV-C: only one amplitude is 1).
// A fill kernel, not a memset, so that the call may sit in a captured graph.
template <typename V>
__global__ void __launch_bounds__(256)
k_fill_basis(V *__restrict__ st, uint64_t total, int n, uint64_t basis) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t mask = (1ull << n) - 1;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        V v;
        v.x = ((i & mask) == basis) ? 1 : 0;
        v.y = 0;
        st[i] = v;
    }
}

__global__ void __launch_bounds__(256)
k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

struct BitPairs { uint8_t a[32]; uint8_t b[32]; int n; };

// In-place permutation that swaps physical bits a_j <-> b_j (disjoint pairs):
// the paper's chunk_swap materialised (Fig. "chunk_swap").  It is an
// involution, so amplitude x trades places with y = x with the bit pairs
// exchanged whenever y > x.
template <typename V>
__global__ void __launch_bounds__(256)
k_swap_bits(V *__restrict__ st, uint64_t total, BitPairs bp) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        uint64_t y = x;
        for (int j = 0; j < bp.n; ++j) {
            uint64_t ba = (x >> bp.a[j]) & 1, bb = (x >> bp.b[j]) & 1;
            if (ba != bb) y ^= (1ull << bp.a[j]) | (1ull << bp.b[j]);
        }
        if (y > x) {
            V u = st[x], w = st[y];
            st[x] = w;
            st[y] = u;
        }
    }
}

template <typename V>
__device__ __forceinline__ double abs2(V v) {
    return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

__device__ __forceinline__ double zsum(uint64_t x, const qsv_zterm *__restrict__ t, int nt) {
    double h = 0.0;
    for (int j = 0; j < nt; ++j)
        h += (__popcll(x & t[j].zmask) & 1) ? -t[j].coeff : t[j].coeff;
    return h;
}

// block-level FP64 sum of W values per thread, fixed order (deterministic)
template <int W>
__device__ __forceinline__ void block_sum(double (&v)[W], double *out) {
    __shared__ double sh[W][RED_THREADS];
    for (int w = 0; w < W; ++w) sh[w][threadIdx.x] = v[w];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int w = 0; w < W; ++w) sh[w][threadIdx.x] += sh[w][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int w = 0; w < W; ++w) out[w] = sh[w][0];
}

// kind 0: norm, 1: overlap (re, im, |a|^2, |b|^2), 2: Z-string expectation
template <typename V, int KIND>
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_partial(const V *__restrict__ a, const V *__restrict__ b, int n,
                 const qsv_zterm *__restrict__ terms, int nt, double *__restrict__ partials) {
    constexpr int W = KIND == 1 ? 4 : 1;
    const uint64_t N = 1ull << n;
    const V *pa = a + ((uint64_t)blockIdx.y << n);
    const V *pb = b ? b + ((uint64_t)blockIdx.y << n) : nullptr;
    double acc[W];
    for (int w = 0; w < W; ++w) acc[w] = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * RED_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < N; i += stride) {
        V x = pa[i];
        if constexpr (KIND == 0) {
            acc[0] += abs2(x);
        } else if constexpr (KIND == 1) {
            V y = pb[i];
            acc[0] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
            acc[1] += (double)x.x * (double)y.y - (double)x.y * (double)y.x;
            acc[2] += abs2(x);
            acc[3] += abs2(y);
        } else {
            acc[0] += abs2(x) * zsum(i, terms, nt);
        }
    }
    block_sum<W>(acc, partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * W);
}

template <int W>
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_final(const double *__restrict__ partials, int nblk, double *__restrict__ out) {
    const double *p = partials + (size_t)blockIdx.x * nblk * W;
    double acc[W];
    for (int w = 0; w < W; ++w) acc[w] = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RED_THREADS)
        for (int w = 0; w < W; ++w) acc[w] += p[(size_t)i * W + w];
    block_sum<W>(acc, out + (size_t)blockIdx.x * W);
}

// Diagonal of a density matrix held as a 2n-qubit state (rho[i][i] at index
// i | (i << n)): per-block FP64 sums of Re rho[i][i] (KIND 0, the trace) or of
// Re rho[i][i] h(i) for Z-strings h (KIND 1), in a fixed order.
template <typename V, int KIND>
__global__ void __launch_bounds__(RED_THREADS)
k_dm_diag_partial(const V *__restrict__ rho, int n, const qsv_zterm *__restrict__ terms, int nt,
                  double *__restrict__ partials) {
    const uint64_t N = 1ull << n;
    double acc[1] = {0.0};
    const uint64_t stride = (uint64_t)gridDim.x * RED_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < N; i += stride) {
        const double d = (double)rho[i | (i << n)].x;
        if constexpr (KIND == 0) acc[0] += d;
        else acc[0] += d * zsum(i, terms, nt);
    }
    block_sum<1>(acc, partials + blockIdx.x);
}

template <typename V>
__global__ void __launch_bounds__(256)
k_scale(V *__restrict__ st, int n, const double *__restrict__ norm2) {
    const double nn = norm2[blockIdx.y];
    if (!(nn > 0.0) || !isfinite(nn)) return;
    const double f = 1.0 / sqrt(nn);
    V *p = st + ((uint64_t)blockIdx.y << n);
    const uint64_t N = 1ull << n;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        V v = p[i];
        v.x = (decltype(v.x))((double)v.x * f);
        v.y = (decltype(v.y))((double)v.y * f);
        p[i] = v;
    }
}

// Per-state parameter tables of the parameterised ops (see OP_PROT / OP_PDIAG):
//   RX, RY: (cos(t/2), 0), (sin(t/2), 0);  RZ: e^{-i t/2}, e^{i t/2};  P: 1, e^{i t}
template <typename V>
__global__ void __launch_bounds__(256)
k_param_table(const double *__restrict__ params, int n_params, const PSlot *__restrict__ slots,
              int nslots, int batch, V *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslots * batch) return;
    const int b = i / nslots, k = i % nslots;
    const PSlot ps = slots[k];
    const double t = params[(size_t)b * n_params + ps.param];
    double s, c;
    V v0, v1;
    if (ps.rot == ROT_RX || ps.rot == ROT_RY) {
        sincos(0.5 * t, &s, &c);
        v0.x = c; v0.y = 0;
        v1.x = s; v1.y = 0;
    } else if (ps.rot == ROT_RZ) {
        sincos(0.5 * t, &s, &c);
        v0.x = c; v0.y = -s;
        v1.x = c; v1.y = s;
    } else {
        sincos(t, &s, &c);
        v0.x = 1; v0.y = 0;
        v1.x = c; v1.y = s;
    }
    out[(size_t)b * 2 * nslots + 2 * k] = v0;
    out[(size_t)b * 2 * nslots + 2 * k + 1] = v1;
}

}  // namespace

hipError_t launch_param_table(qsv_dtype dt, const double *params, int n_params,
                              const PSlot *slots, int nslots, int batch, void *ptab, hipStream_t s) {
    const int total = nslots * batch;
    if (total == 0) return hipSuccess;
    const int blocks = (total + 255) / 256;
    if (dt == QSV_C128)
        hipLaunchKernelGGL((k_param_table<Cplx<double>>), dim3(blocks), dim3(256), 0, s, params,
                           n_params, slots, nslots, batch, (Cplx<double> *)ptab);
    else
        hipLaunchKernelGGL((k_param_table<Cplx<float>>), dim3(blocks), dim3(256), 0, s, params,
                           n_params, slots, nslots, batch, (Cplx<float> *)ptab);
    return hipGetLastError();
}

int reduce_blocks(int n) {
    uint64_t N = 1ull << n;
    uint64_t b = (N + RED_THREADS * 8 - 1) / (RED_THREADS * 8);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_fill_basis(qsv_dtype dt, void *state, int n, int batch, uint64_t basis,
                             hipStream_t s) {
    uint64_t total = (uint64_t)batch << n;
    if (dt == QSV_C128)
        hipLaunchKernelGGL((k_fill_basis<Cplx<double>>), dim3(grid_for(total)), dim3(256), 0, s,
                           (Cplx<double> *)state, total, n, basis);
    else
        hipLaunchKernelGGL((k_fill_basis<Cplx<float>>), dim3(grid_for(total)), dim3(256), 0, s,
                           (Cplx<float> *)state, total, n, basis);
    return hipGetLastError();
}

hipError_t launch_copy(qsv_dtype dt, void *dst, const void *src, int n, hipStream_t s) {
    uint64_t bytes = (1ull << n) * (dt == QSV_C128 ? 16 : 8);
    if (bytes % 16 == 0) {
        uint64_t n16 = bytes / 16;
        hipLaunchKernelGGL(k_copy16, dim3(grid_for(n16, 256ull * 64)), dim3(256), 0, s, (uint4 *)dst,
                           (const uint4 *)src, n16);
        return hipGetLastError();
    }
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_swap_bits(qsv_dtype dt, void *state, int n, const uint8_t *pa, const uint8_t *pb,
                            int npairs, hipStream_t s) {
    BitPairs bp;
    bp.n = npairs;
    for (int j = 0; j < npairs && j < 32; ++j) {
        bp.a[j] = pa[j];
        bp.b[j] = pb[j];
    }
    uint64_t total = 1ull << n;
    if (dt == QSV_C128)
        hipLaunchKernelGGL((k_swap_bits<Cplx<double>>), dim3(grid_for(total)), dim3(256), 0, s,
                           (Cplx<double> *)state, total, bp);
    else
        hipLaunchKernelGGL((k_swap_bits<Cplx<float>>), dim3(grid_for(total)), dim3(256), 0, s,
                           (Cplx<float> *)state, total, bp);
    return hipGetLastError();
}

template <typename V>
static hipError_t reduce_t(int kind, const void *a, const void *b, int n, int batch,
                           const qsv_zterm *terms, int nt, double *partials, int nblk, double *out,
                           hipStream_t s) {
    dim3 grid(nblk, batch);
    if (kind == 0) {
        hipLaunchKernelGGL((k_reduce_partial<V, 0>), grid, dim3(RED_THREADS), 0, s, (const V *)a,
                           nullptr, n, nullptr, 0, partials);
        hipLaunchKernelGGL((k_reduce_final<1>), dim3(batch), dim3(RED_THREADS), 0, s, partials,
                           nblk, out);
    } else if (kind == 1) {
        hipLaunchKernelGGL((k_reduce_partial<V, 1>), grid, dim3(RED_THREADS), 0, s, (const V *)a,
                           (const V *)b, n, nullptr, 0, partials);
        hipLaunchKernelGGL((k_reduce_final<4>), dim3(batch), dim3(RED_THREADS), 0, s, partials,
                           nblk, out);
    } else {
        hipLaunchKernelGGL((k_reduce_partial<V, 2>), grid, dim3(RED_THREADS), 0, s, (const V *)a,
                           nullptr, n, terms, nt, partials);
        hipLaunchKernelGGL((k_reduce_final<1>), dim3(batch), dim3(RED_THREADS), 0, s, partials,
                           nblk, out);
    }
    return hipGetLastError();
}

hipError_t launch_reduce(qsv_dtype dt, int kind, const void *a, const void *b, int n, int batch,
                         const qsv_zterm *terms_dev, int n_terms, double *partials, int nblk,
                         double *out, hipStream_t s) {
    if (dt == QSV_C128)
        return reduce_t<Cplx<double>>(kind, a, b, n, batch, terms_dev, n_terms, partials, nblk, out, s);
    return reduce_t<Cplx<float>>(kind, a, b, n, batch, terms_dev, n_terms, partials, nblk, out, s);
}

// Reduction partials for callers that cannot allocate (qsv_overlap_noalloc):
// one fixed array per GPU, held by the library until the process ends.  Every
// partial is written before it is read, so nothing has to be cleared between
// calls.  On the host, `scratch` names a host-side stand-in, not device memory:
// kernels get the address that hipGetSymbolAddress returns for the current
// device.
constexpr size_t NOALLOC_PARTIALS = QSV_NOALLOC_PARTIALS;
static_assert(NOALLOC_PARTIALS >= 2048 * 4, "reduce_blocks() <= 2048 blocks, 4 sums each");
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

hipError_t noalloc_scratch(int device, double **ptr, size_t *cap) {
    static std::mutex mu;
    static double *addr[64];
    static bool known[64];
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!known[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
        known[device] = true;
    }
    *ptr = addr[device];
    *cap = NOALLOC_PARTIALS;
    return hipSuccess;
}

// Observable upload without a host staging buffer: up to TERMS_PER_LAUNCH
// terms travel by value in the kernel's argument block, so the host array may
// be released as soon as the call returns and the copy needs no
// synchronisation (and may sit in a captured graph).
constexpr int TERMS_PER_LAUNCH = 128;
struct TermBlock {
    qsv_zterm t[TERMS_PER_LAUNCH];
    int count;
};
static_assert(sizeof(TermBlock) <= 4096, "kernel argument block");

__global__ void __launch_bounds__(TERMS_PER_LAUNCH)
k_store_terms(TermBlock blk, qsv_zterm *__restrict__ dst) {
    const int i = threadIdx.x;
    if (i < blk.count) dst[i] = blk.t[i];
}

hipError_t launch_store_terms(const qsv_zterm *host, size_t nt, qsv_zterm *dev, hipStream_t s) {
    for (size_t off = 0; off < nt; off += TERMS_PER_LAUNCH) {
        TermBlock blk;
        blk.count = (int)std::min<size_t>(TERMS_PER_LAUNCH, nt - off);
        for (int i = 0; i < blk.count; ++i) blk.t[i] = host[off + i];
        hipLaunchKernelGGL(k_store_terms, dim3(1), dim3(TERMS_PER_LAUNCH), 0, s, blk, dev + off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_dm_reduce(qsv_dtype dt, int kind, const void *rho, int n,
                            const qsv_zterm *terms_dev, int n_terms, double *partials, int nblk,
                            double *out, hipStream_t s) {
#define QSV_DM(V)                                                                              \
    if (kind == 0)                                                                             \
        hipLaunchKernelGGL((k_dm_diag_partial<V, 0>), dim3(nblk), dim3(RED_THREADS), 0, s,      \
                           (const V *)rho, n, nullptr, 0, partials);                           \
    else                                                                                       \
        hipLaunchKernelGGL((k_dm_diag_partial<V, 1>), dim3(nblk), dim3(RED_THREADS), 0, s,      \
                           (const V *)rho, n, terms_dev, n_terms, partials);
    if (dt == QSV_C128) {
        QSV_DM(Cplx<double>)
    } else {
        QSV_DM(Cplx<float>)
    }
#undef QSV_DM
    hipLaunchKernelGGL((k_reduce_final<1>), dim3(1), dim3(RED_THREADS), 0, s, partials, nblk, out);
    return hipGetLastError();
}

hipError_t launch_scale_by_norm(qsv_dtype dt, void *state, int n, int batch, const double *norm2,
                                hipStream_t s) {
    dim3 grid(grid_for(1ull << n, 4096), batch);
    if (dt == QSV_C128)
        hipLaunchKernelGGL((k_scale<Cplx<double>>), grid, dim3(256), 0, s, (Cplx<double> *)state, n, norm2);
    else
        hipLaunchKernelGGL((k_scale<Cplx<float>>), grid, dim3(256), 0, s, (Cplx<float> *)state, n, norm2);
    return hipGetLastError();
}

}  // namespace qsv
