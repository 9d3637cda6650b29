// Section kernel instances for complex128 states.
#include "section_kernels.hpp"

namespace qsv {

hipError_t launch_section_c128(int r, int kmax, bool dense_only, void *state, int n, int batch,
                              DevPlanView pv, int sec, int c, size_t lds_bytes, const void *ptab,
                              int nslots, hipStream_t s) {
    return launch_section_dt<double>(r, kmax, dense_only, state, n, batch, pv, sec, c, lds_bytes, ptab,
                                   nslots, s);
}

}  // namespace qsv
