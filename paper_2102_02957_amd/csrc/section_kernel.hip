// The section kernel: one blocked section (begin_blocking .. end_blocking,
// Sec. IV-A / IV-C) applied to every chunk of the state.
//
// One workgroup owns one chunk of 2^c amplitudes (Sec. III-B: a chunk is the
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
#include "section_core.hpp"

namespace qsv {

using namespace sec;

// KMAX: widest dense op the kernel instance carries code for (register pressure
// of the whole kernel follows the widest case, so narrow plans use KMAX = 2).
template <typename T, int R, int KMAX>
__global__ void __launch_bounds__(256)
k_section(typename Amp<T>::V *__restrict__ state, int n, const DevSection *__restrict__ secs_g,
          int sec, const DevPhase *__restrict__ phases_g, const DevOp *__restrict__ ops_g,
          const typename Amp<T>::V *__restrict__ mats_g, const double *__restrict__ params,
          int n_params) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *st = state + ((uint64_t)blockIdx.y << n);
    const double *prm = params ? params + (size_t)blockIdx.y * n_params : nullptr;
    run_chunk<T, R, KMAX>(st, (cptr<DevSection>)secs_g + sec, (cptr<DevPhase>)phases_g,
                          (cptr<DevOp>)ops_g, (cptr<V>)mats_g, prm, blockIdx.x,
                          reinterpret_cast<V *>(lds_raw), true);
}

template <typename T, int R, int KMAX>
static hipError_t launch_section_t(void *state, int n, int batch, DevPlanView pv, int sec, int c,
                                   size_t lds_bytes, const double *params, int n_params,
                                   hipStream_t s) {
    using V = typename Amp<T>::V;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_section<T, R, KMAX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (c - R > 8 || c < R) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)(1ull << (n - c)), (unsigned)batch);
    dim3 block(1u << (c - R));
    hipLaunchKernelGGL((k_section<T, R, KMAX>), grid, block, lds_bytes, s, (V *)state, n, pv.secs,
                       sec, pv.phases, pv.ops, (const V *)pv.mats, params, n_params);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_section_dt(int r, int kmax, void *state, int n, int batch, DevPlanView pv,
                                    int sec, int c, size_t lds_bytes, const double *params,
                                    int n_params, hipStream_t s) {
#define QSV_SEC(R_, K_) \
    return launch_section_t<T, R_, K_>(state, n, batch, pv, sec, c, lds_bytes, params, n_params, s)
    const bool wide = kmax > 2;
    switch (r) {
        case 1: QSV_SEC(1, 1);
        case 2: QSV_SEC(2, 2);
        case 3: if (wide) QSV_SEC(3, 3); else QSV_SEC(3, 2);
        case 4: if (wide) QSV_SEC(4, 4); else QSV_SEC(4, 2);
        case 5: if (wide) QSV_SEC(5, 5); else QSV_SEC(5, 2);
    }
#undef QSV_SEC
    return hipErrorInvalidValue;
}

hipError_t launch_section(qsv_dtype dt, int r, int kmax, void *state, int n, int batch,
                          DevPlanView pv, int sec, int c, size_t lds_bytes, const double *params,
                          int n_params, hipStream_t s) {
    if (dt == QSV_C128)
        return launch_section_dt<double>(r, kmax, state, n, batch, pv, sec, c, lds_bytes, params,
                                         n_params, s);
    return launch_section_dt<float>(r, kmax, state, n, batch, pv, sec, c, lds_bytes, params,
                                    n_params, s);
}

}  // namespace qsv
