// Entry points not yet implemented in this build return QSV_E_UNSUPPORTED.
#include "device.hpp"

extern "C" {

qsv_status qsv_adjoint_grad(qsv_ctx *, const qsv_plan *, const qsv_zterm *, size_t, const double *,
                            int, void *, void *, double *, double *, void *) {
    qsv::set_error("qsv_adjoint_grad: not built");
    return QSV_E_UNSUPPORTED;
}

qsv_status qsv_batch_run(qsv_ctx *, int, const qsv_plan *const *, const uint64_t *, void *,
                         double *, void *) {
    qsv::set_error("qsv_batch_run: not built");
    return QSV_E_UNSUPPORTED;
}
}
