// Device-side helpers and host-callable launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsv_internal.hpp"

namespace qsv {

// amplitude type: (re, im) interleaved, aligned to its size so that one amplitude
// is one 8- or 16-byte memory access.  A plain struct (not HIP's vector types)
// so that arrays of it are promoted to registers.
template <typename T> struct alignas(2 * sizeof(T)) Cplx {
    T x, y;
};
template <typename T> struct Amp { using V = Cplx<T>; };

struct DevPlanView {           // device pointers of one uploaded plan
    const DevSection *secs;
    const DevPhase *phases;
    const DevOp *ops;
    const void *mats;          // V[] in the context's dtype
    const PgOp *pg;
    const PSlot *pslots;
    const int32_t *poff, *plist;   // parameter -> param ops (CSR)
};

// ---- launchers (kernels.hip) ----------------------------------------------

// One section of a blocked plan over `batch` states (state b at state + b * 2^n).
// lds_bytes == 0 when the section has a single phase.
// kmax: widest dense op in the plan (selects the kernel instance); ptab: the
// per-state parameter tables (batch x 2 * nslots amplitudes-typed values) or NULL.
// dense_only: the section's flags carry SEC_DENSE_ONLY (a leaner kernel instance).
hipError_t launch_section(qsv_dtype dt, int r, int kmax, bool dense_only, void *state, int n,
                          int batch, DevPlanView pv, int sec, int c, size_t lds_bytes,
                          const void *ptab, int nslots, hipStream_t s);
// One paired section (SEC_PAIRED): 2^(c-4) threads per chunk, lds_bytes as for
// launch_section (0 for a single phase).
hipError_t launch_section_paired(qsv_dtype dt, void *state, int n, int batch, DevPlanView pv,
                                 int sec, int c, size_t lds_bytes, hipStream_t s);
// One section with the chunk resident in LDS (plans with section_kernel = QSV_KERNEL_LDS or
// QSV_KERNEL_MFMA: one phase per section, op positions = LDS index bits; mfma: dense ops
// of 4 and 5 qubits on the matrix cores, chunk_bits >= 9).
hipError_t launch_section_lds(qsv_dtype dt, int kmax, bool mfma, void *state, int n, int batch,
                              DevPlanView pv, int sec, int c, hipStream_t s);
// ptab[b][2 i], ptab[b][2 i + 1] for every parameterised op i (see OP_PROT / OP_PDIAG)
hipError_t launch_param_table(qsv_dtype dt, const double *params, int n_params,
                              const PSlot *slots, int nslots, int batch, void *ptab, hipStream_t s);
// `hmats`: the plan's FP64 host table (diagonal entries are passed by value);
// `dmats`: its device copy in the state's dtype (dense matrices are read there).
hipError_t launch_pergate_host(qsv_dtype dt, void *state, int n, const PgOp &op, const cd *hmats,
                               const void *dmats, hipStream_t s);
hipError_t launch_fill_basis(qsv_dtype dt, void *state, int n, int batch, uint64_t basis,
                             hipStream_t s);
hipError_t launch_copy(qsv_dtype dt, void *dst, const void *src, int n, hipStream_t s);
hipError_t launch_swap_bits(qsv_dtype dt, void *state, int n, const uint8_t *pa,
                            const uint8_t *pb, int npairs, hipStream_t s);

// FP64 reductions: partials (double, `nblk` * width) then a single-block final sum.
// kind: 0 norm (width 1), 1 overlap (width 4), 2 Z-string expval (width 1)
hipError_t launch_reduce(qsv_dtype dt, int kind, const void *a, const void *b, int n, int batch,
                         const qsv_zterm *terms_dev, int n_terms, double *partials, int nblk,
                         double *out, hipStream_t s);
hipError_t launch_scale_by_norm(qsv_dtype dt, void *state, int n, int batch, const double *norm2,
                                hipStream_t s);
int reduce_blocks(int n);
// density matrix of n qubits (2n-qubit state): kind 0 trace, 1 Z-string expectation
hipError_t launch_dm_reduce(qsv_dtype dt, int kind, const void *rho, int n,
                            const qsv_zterm *terms_dev, int n_terms, double *partials, int nblk,
                            double *out, hipStream_t s);
// device address (for the current device, which must be `device`) and size in
// doubles of the library's fixed reduction-partials array (qsv_overlap_noalloc)
hipError_t noalloc_scratch(int device, double **ptr, size_t *cap);
// copy host Z-string terms to a device table (by value through kernel arguments)
hipError_t launch_store_terms(const qsv_zterm *host, size_t nt, qsv_zterm *dev, hipStream_t s);

// adjoint.hip
hipError_t launch_adjoint_section(qsv_dtype dt, int r, void *psi, void *lam, int n, int batch,
                                  DevPlanView pv, int sec, int c, size_t lds, const void *ptab,
                                  int nslots, double *part, hipStream_t s);
hipError_t launch_apply_zsum(qsv_dtype dt, const void *psi, void *lam, int n, int batch,
                             const qsv_zterm *terms, int nt, hipStream_t s);
hipError_t launch_grad_reduce(const double *part, int nslots, int batch, uint64_t nchunks,
                              double *ssum, const int32_t *off, const int32_t *slots, int nparams,
                              double *grad, hipStream_t s);

}  // namespace qsv
