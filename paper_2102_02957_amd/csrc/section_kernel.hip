// Dispatch of a section launch to the instances of the state's dtype.
#include "device.hpp"

namespace qsv {

hipError_t launch_section_c128(int r, int kmax, bool dense_only, void *state, int n, int batch,
                               DevPlanView pv, int sec, int c, size_t lds_bytes, const void *ptab,
                               int nslots, hipStream_t s);
hipError_t launch_section_c64(int r, int kmax, bool dense_only, void *state, int n, int batch,
                              DevPlanView pv, int sec, int c, size_t lds_bytes, const void *ptab,
                              int nslots, hipStream_t s);

hipError_t launch_section(qsv_dtype dt, int r, int kmax, bool dense_only, void *state, int n,
                          int batch, DevPlanView pv, int sec, int c, size_t lds_bytes,
                          const void *ptab, int nslots, hipStream_t s) {
    if (dt == QSV_C128)
        return launch_section_c128(r, kmax, dense_only, state, n, batch, pv, sec, c, lds_bytes,
                                   ptab, nslots, s);
    return launch_section_c64(r, kmax, dense_only, state, n, batch, pv, sec, c, lds_bytes, ptab,
                              nslots, s);
}

}  // namespace qsv
