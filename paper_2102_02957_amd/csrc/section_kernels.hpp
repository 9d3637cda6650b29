// The section kernel: one blocked section (begin_blocking .. end_blocking,
// Sec. IV-A / IV-C) applied to every chunk of the state.
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

#include "section_core.hpp"

namespace qsv {

using namespace sec;

// KMAX: widest dense op the kernel instance carries code for (register pressure
// of the whole kernel follows the widest case, so narrow plans use KMAX = 2;
// dense-only sections of 3-qubit fused ops have their own KMAX = 3 instance).
// Up to 512 threads per workgroup for R <= 4 (chunk_bits - R <= 9), 256 for R = 5
// (whose amplitude registers need the larger per-thread register budget).
template <int R> constexpr int section_max_threads() { return R <= 4 ? 512 : 256; }

template <typename T, int R, int KMAX, bool DENSE_ONLY>
__global__ void __launch_bounds__(section_max_threads<R>())
k_section(typename Amp<T>::V *__restrict__ state, int n, const DevSection *__restrict__ secs_g,
          int sec, const DevPhase *__restrict__ phases_g, const DevOp *__restrict__ ops_g,
          const typename Amp<T>::V *__restrict__ mats_g, const typename Amp<T>::V *__restrict__ ptab_g,
          int nslots) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *st = state + ((uint64_t)blockIdx.y << n);
    const cptr<V> ptab = (cptr<V>)ptab_g + (size_t)blockIdx.y * 2 * nslots;
    run_chunk<T, R, KMAX, DENSE_ONLY>(st, (cptr<DevSection>)secs_g + sec, (cptr<DevPhase>)phases_g,
                          (cptr<DevOp>)ops_g, (cptr<V>)mats_g, ptab, blockIdx.x,
                          reinterpret_cast<V *>(lds_raw), true);
}

template <typename T, int R, int KMAX, bool DENSE_ONLY>
inline hipError_t launch_section_t(void *state, int n, int batch, DevPlanView pv, int sec, int c,
                                   size_t lds_bytes, const void *ptab, int nslots,
                                   hipStream_t s) {
    using V = typename Amp<T>::V;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_section<T, R, KMAX, DENSE_ONLY>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if ((1 << (c - R)) > section_max_threads<R>() || c < R) return hipErrorInvalidConfiguration;
    const uint64_t nchunks = 1ull << (n - c);
    dim3 block(1u << (c - R));
    dim3 grid((unsigned)nchunks, (unsigned)batch);
    hipLaunchKernelGGL((k_section<T, R, KMAX, DENSE_ONLY>), grid, block, lds_bytes, s, (V *)state, n, pv.secs,
                       sec, pv.phases, pv.ops, (const V *)pv.mats, (const V *)ptab, nslots);
    return hipGetLastError();
}

template <typename T>
inline hipError_t launch_section_dt(int r, int kmax, bool dense_only, void *state, int n, int batch,
                                    DevPlanView pv, int sec, int c, size_t lds_bytes,
                                    const void *ptab, int nslots, hipStream_t s) {
#define QSV_SEC(R_, K_, D_)                                                                  \
    return launch_section_t<T, R_, K_, D_>(state, n, batch, pv, sec, c, lds_bytes, ptab, nslots, s)
    const bool wide = kmax > 2;
    switch (r) {
        case 1: QSV_SEC(1, 1, false);
        case 2: QSV_SEC(2, 2, false);
        case 3: if (wide) QSV_SEC(3, 3, false); else QSV_SEC(3, 2, false);
        case 4:
            if (kmax == 3 && dense_only) QSV_SEC(4, 3, true);
            if (wide) QSV_SEC(4, 4, false);
            else if (dense_only) QSV_SEC(4, 2, true);
            else QSV_SEC(4, 2, false);
        case 5:
            if (wide) QSV_SEC(5, 5, false);
            else if (dense_only) QSV_SEC(5, 2, true);
            else QSV_SEC(5, 2, false);
    }
#undef QSV_SEC
    return hipErrorInvalidValue;
}

}  // namespace qsv
