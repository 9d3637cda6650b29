// Section kernel for paired sections (SEC_PAIRED): two dense 2-qubit ops per
// phase at fixed register positions, 4 register bits (16 amplitudes per thread),
// LDS transpositions between phases, one HBM read and one write per section
// (Sec. IV-C).  With no run-time choice of registers the compiler keeps the
// amplitudes in place, which halves the registers a wave needs compared with the
// general register-phase kernel.
#include <algorithm>

#include "section_core.hpp"

namespace qsv {

using namespace sec;

namespace {

// The FP32 instance fits in 80 VGPRs without spilling, which gives 6 waves per
// SIMD: three workgroups of 512 threads per CU.  At 5 waves it holds only two,
// and FP32 FMAs reach full rate only while two waves per SIMD issue.  The FP64
// instance keeps the compiler's choice (105 VGPRs; 80 would spill).
template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1)))
k_section_paired(typename Amp<T>::V *__restrict__ state, int n, const DevSection *__restrict__ secs_g,
                 int sec, const DevPhase *__restrict__ phases_g, const DevOp *__restrict__ ops_g,
                 const typename Amp<T>::V *__restrict__ mats_g) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *st = state + ((uint64_t)blockIdx.y << n);
    run_chunk_paired<T, 4>(st, (cptr<DevSection>)secs_g + sec, (cptr<DevPhase>)phases_g,
                           (cptr<DevOp>)ops_g, (cptr<V>)mats_g, blockIdx.x,
                           reinterpret_cast<V *>(lds_raw));
}

template <typename T>
hipError_t launch_paired_t(void *state, int n, int batch, DevPlanView pv, int sec, int c,
                           size_t lds_bytes, hipStream_t s) {
    using V = typename Amp<T>::V;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_section_paired<T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (c < 4 || (1 << (c - 4)) > 512) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)(1ull << (n - c)), (unsigned)batch);
    hipLaunchKernelGGL((k_section_paired<T>), grid, dim3(1u << (c - 4)), lds_bytes, s, (V *)state,
                       n, pv.secs, sec, pv.phases, pv.ops, (const V *)pv.mats);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_section_paired(qsv_dtype dt, void *state, int n, int batch, DevPlanView pv,
                                 int sec, int c, size_t lds_bytes, hipStream_t s) {
    if (dt == QSV_C128) return launch_paired_t<double>(state, n, batch, pv, sec, c, lds_bytes, s);
    return launch_paired_t<float>(state, n, batch, pv, sec, c, lds_bytes, s);
}

}  // namespace qsv
