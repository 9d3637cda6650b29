// Batched trajectories: many independent states of uneven qubit counts (the
// paper's shots / noisy simulation, Sec. III-A and IV-B) run in one persistent
// launch.
//
// Every (trajectory, section, chunk) is a task; tasks are ordered section
// by section (all first sections, then all second sections, ...), and
// workgroups pop them from a global counter.  A task of section s > 0 waits
// until every chunk of section s - 1 of its trajectory has been written
// (per-trajectory completion counters, agent-scope acquire/release).  Since
// tasks are popped in that order, a waiting task only depends on tasks
// already held by running workgroups; the wait is also bounded by a spin
// limit that sets an error flag, so the grid always drains.  The last
// section of a trajectory also writes its chunk's FP64 norm; a second kernel
// sums them (fixed order) and a third rescales every state by 1/sqrt(norm).
// The whole sequence (init, persistent kernel, norm, rescale) is captured
// once into a HIP graph and replayed.
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include <algorithm>

#include "section_core.hpp"

namespace qsv {

using namespace sec;

struct BatchTraj {        // one trajectory (state) of the batch
    uint64_t state_off;   // amplitude offset in the packed buffer
    uint32_t n;           // qubits
    uint32_t sec_begin;   // first section in the combined section table
    uint32_t nsec;
    uint32_t done_base;   // first completion counter (sections 0 .. nsec-2)
    uint32_t part_base;   // first norm partial (one per chunk of the last section)
    uint32_t nchunks;     // chunks per section
};

struct BatchTask {
    uint32_t traj, sec, chunk, pad;
};

constexpr int BATCH_THREADS = 256;
constexpr uint32_t CTR_NEXT = 0, CTR_ERR = 1, CTR_DONE = 2;

template <typename T, int R, int KMAX>
__global__ void __launch_bounds__(BATCH_THREADS)
k_batch(typename Amp<T>::V *__restrict__ states, const BatchTraj *__restrict__ trajs,
        const BatchTask *__restrict__ tasks, uint32_t ntasks, uint32_t *__restrict__ counters,
        double *__restrict__ norm_parts, const DevSection *__restrict__ secs_g,
        const DevPhase *__restrict__ phases_g, const DevOp *__restrict__ ops_g,
        const typename Amp<T>::V *__restrict__ mats_g, uint32_t spin_limit) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *lds = reinterpret_cast<V *>(lds_raw);
    __shared__ uint32_t s_task;
    __shared__ double s_red[BATCH_THREADS];
    const unsigned tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_task = atomicAdd(&counters[CTR_NEXT], 1u);
        __syncthreads();
        const uint32_t t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const BatchTask task = tasks[t];
        const BatchTraj tr = trajs[task.traj];
        if (task.sec > 0) {
            if (tid == 0) {
                uint32_t *ctr = &counters[CTR_DONE + tr.done_base + task.sec - 1];
                uint32_t spins = 0;
                while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
                       tr.nchunks) {
                    // give up after the spin limit, or at once if another wait already did
                    if (++spins > spin_limit ||
                        __hip_atomic_load(&counters[CTR_ERR], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                        atomicOr(&counters[CTR_ERR], 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const cptr<DevSection> S = (cptr<DevSection>)secs_g + (tr.sec_begin + task.sec);
        const bool active = tid < (1u << (S->c - R));
        V *st = states + tr.state_off;
        if (task.sec + 1 == tr.nsec) {
            const double nrm = run_chunk_norm<T, R, KMAX>(
                st, S, (cptr<DevPhase>)phases_g, (cptr<DevOp>)ops_g, (cptr<V>)mats_g, nullptr,
                task.chunk, lds, s_red, active);
            if (tid == 0) norm_parts[tr.part_base + task.chunk] = nrm;
        } else {
            run_chunk<T, R, KMAX>(st, S, (cptr<DevPhase>)phases_g, (cptr<DevOp>)ops_g,
                                  (cptr<V>)mats_g, nullptr, task.chunk, lds, active);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0)
                __hip_atomic_fetch_add(&counters[CTR_DONE + tr.done_base + task.sec], 1u,
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// norms[b] = sum of the trajectory's chunk partials, in chunk order; NaN for
// every trajectory if a dependency wait ran out (the results are then invalid)
__global__ void __launch_bounds__(64)
k_batch_norm(const BatchTraj *__restrict__ trajs, const double *__restrict__ parts,
             const uint32_t *__restrict__ counters, double *__restrict__ norms) {
    const BatchTraj tr = trajs[blockIdx.x];
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (uint32_t g = 0; g < tr.nchunks; ++g) s += parts[tr.part_base + g];
        norms[blockIdx.x] = counters[CTR_ERR] ? __builtin_nan("") : s;
    }
}

// states *= 1/sqrt(norm) (FP64 scale), one workgroup per (trajectory, block of 2^12 amplitudes)
struct ScaleBlock {
    uint32_t traj;
    uint32_t blk;
};

template <typename V>
__global__ void __launch_bounds__(256)
k_batch_scale(V *__restrict__ states, const BatchTraj *__restrict__ trajs,
              const ScaleBlock *__restrict__ blocks, const double *__restrict__ norms) {
    const ScaleBlock sb = blocks[blockIdx.x];
    const BatchTraj tr = trajs[sb.traj];
    const double nn = norms[sb.traj];
    if (!(nn > 0.0) || !isfinite(nn)) return;
    const double f = 1.0 / sqrt(nn);
    const uint64_t len = 1ull << tr.n;
    const uint64_t b0 = (uint64_t)sb.blk << 12;
    V *p = states + tr.state_off;
    for (uint64_t i = b0 + threadIdx.x; i < b0 + 4096 && i < len; i += 256) {
        V v = p[i];
        v.x = (decltype(v.x))((double)v.x * f);
        v.y = (decltype(v.y))((double)v.y * f);
        p[i] = v;
    }
}

template <typename V>
__global__ void __launch_bounds__(256)
k_batch_init(V *__restrict__ states, uint64_t total) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        V v;
        v.x = 0;
        v.y = 0;
        states[i] = v;
    }
}

template <typename V>
__global__ void __launch_bounds__(256)
k_batch_ones(V *__restrict__ states, const BatchTraj *__restrict__ trajs, int count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < count) {
        V v;
        v.x = 1;
        v.y = 0;
        states[trajs[b].state_off] = v;
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------

}  // namespace qsv
#include "batch.hpp"
namespace qsv {

static hipError_t launch_batch_kernel(qsv_dtype dt, const BatchLaunch &L, hipStream_t s,
                                      uint32_t spin_limit);

template <typename T, int R, int KMAX>
static hipError_t launch_batch_t(const BatchLaunch &L, hipStream_t s, uint32_t spin_limit) {
    using V = typename Amp<T>::V;
    if (!s) {  // setup call (outside any stream capture)
        return hipFuncSetAttribute((const void *)k_batch<T, R, KMAX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    }
    hipLaunchKernelGGL((k_batch<T, R, KMAX>), dim3(L.grid), dim3(BATCH_THREADS), L.lds, s,
                       (V *)L.states, L.trajs, L.tasks, L.ntasks, L.counters, L.parts, L.secs,
                       L.phases, L.ops, (const V *)L.mats, spin_limit);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_batch_dt(const BatchLaunch &L, hipStream_t s, uint32_t spin_limit) {
    const bool wide = L.kmax > 2;
    switch (L.r) {
        case 3: return wide ? launch_batch_t<T, 3, 3>(L, s, spin_limit) : launch_batch_t<T, 3, 2>(L, s, spin_limit);
        case 4: return wide ? launch_batch_t<T, 4, 4>(L, s, spin_limit) : launch_batch_t<T, 4, 2>(L, s, spin_limit);
        case 5: return wide ? launch_batch_t<T, 5, 5>(L, s, spin_limit) : launch_batch_t<T, 5, 2>(L, s, spin_limit);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_batch_kernel(qsv_dtype dt, const BatchLaunch &L, hipStream_t s,
                                      uint32_t spin_limit) {
    if (dt == QSV_C128) return launch_batch_dt<double>(L, s, spin_limit);
    return launch_batch_dt<float>(L, s, spin_limit);
}

// resident workgroups of the batch kernel for this configuration
static int batch_grid(qsv_dtype dt, int r, int kmax, size_t lds) {
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
    const bool wide = kmax > 2;
#define QSV_OCC(T_, R_, K_) \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<T_, R_, K_>, BATCH_THREADS, lds)
    if (dt == QSV_C128) {
        if (r == 3) { if (wide) QSV_OCC(double, 3, 3); else QSV_OCC(double, 3, 2); }
        if (r == 4) { if (wide) QSV_OCC(double, 4, 4); else QSV_OCC(double, 4, 2); }
        if (r == 5) { if (wide) QSV_OCC(double, 5, 5); else QSV_OCC(double, 5, 2); }
    } else {
        if (r == 3) { if (wide) QSV_OCC(float, 3, 3); else QSV_OCC(float, 3, 2); }
        if (r == 4) { if (wide) QSV_OCC(float, 4, 4); else QSV_OCC(float, 4, 2); }
        if (r == 5) { if (wide) QSV_OCC(float, 5, 5); else QSV_OCC(float, 5, 2); }
    }
#undef QSV_OCC
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * (cus > 0 ? cus : 1);
}

// Build (or fetch) the batch launch for these plans/buffers; captures the graph.
qsv_status batch_prepare(qsv_dtype dt, int count, const Plan *const *plans,
                         const uint64_t *offsets, void *states, double *norms,
                         BatchLaunch &L, std::string &err, uint32_t spin_limit) {
    const size_t es = dt == QSV_C128 ? 16 : 8;
    const int r = plans[0]->r;
    int kmax = 1;
    size_t lds = 0;
    std::vector<BatchTraj> trajs(count);
    std::vector<DevSection> secs;
    std::vector<DevPhase> phases;
    std::vector<DevOp> ops;
    std::vector<cd> mats;
    uint32_t done = 0, parts = 0, maxS = 0;
    uint64_t total = 0;
    for (int b = 0; b < count; ++b) {
        const Plan &P = *plans[b];
        if (P.dtype != dt) {
            err = "plan " + std::to_string(b) + ": dtype differs from the context";
            return QSV_E_INVALID;
        }
        if (P.r != r) {
            err = "all plans of a batch must use the same register_bits";
            return QSV_E_UNSUPPORTED;
        }
        if (P.n_params > 0 || P.opt.swap_mode != QSV_SWAP_REMAP) {
            err = "batch plans must be remap-mode plans without parameters";
            return QSV_E_UNSUPPORTED;
        }
        if (P.c - r > 8) {
            err = "batch plans need chunk_bits - register_bits <= 8";
            return QSV_E_UNSUPPORTED;
        }
        if (offsets[b] % (256 / es) != 0) {
            err = "state offsets must be 256-byte aligned";
            return QSV_E_INVALID;
        }
        kmax = std::max(kmax, P.kmax);
        BatchTraj &t = trajs[b];
        t.state_off = offsets[b];
        t.n = (uint32_t)P.n;
        t.sec_begin = (uint32_t)secs.size();
        t.nsec = (uint32_t)P.dsec.size();
        t.done_base = done;
        t.part_base = parts;
        t.nchunks = (uint32_t)(1ull << (P.n - P.c));
        done += t.nsec > 0 ? t.nsec - 1 : 0;
        parts += t.nchunks;
        maxS = std::max(maxS, t.nsec);
        total = std::max<uint64_t>(total, offsets[b] + (1ull << P.n));
        const uint32_t ph0 = (uint32_t)phases.size(), op0 = (uint32_t)ops.size(),
                       m0 = (uint32_t)mats.size();
        for (size_t si = 0; si < P.dsec.size(); ++si) {
            DevSection d = P.dsec[si];
            d.phase_begin += ph0;
            d.phase_end += ph0;
            secs.push_back(d);
            if (d.phase_end - d.phase_begin > 1) lds = std::max(lds, (size_t(1) << d.c) * es);
        }
        for (const DevPhase &p : P.dphase) {
            DevPhase q = p;
            q.op_begin += op0;
            q.op_end += op0;
            phases.push_back(q);
        }
        for (const DevOp &o : P.dops) {
            DevOp q = o;
            if (q.type == OP_DENSE || q.type == OP_DIAG) q.arg += (int32_t)m0;
            ops.push_back(q);
        }
        mats.insert(mats.end(), P.dmats.begin(), P.dmats.end());
    }
    // overlapping states are a caller error
    {
        std::vector<std::pair<uint64_t, uint64_t>> iv;
        for (int b = 0; b < count; ++b) iv.push_back({offsets[b], offsets[b] + (1ull << plans[b]->n)});
        std::sort(iv.begin(), iv.end());
        for (size_t i = 1; i < iv.size(); ++i)
            if (iv[i].first < iv[i - 1].second) {
                err = "batch states overlap";
                return QSV_E_INVALID;
            }
    }
    std::vector<BatchTask> tasks;
    for (uint32_t s = 0; s < maxS; ++s)
        for (int b = 0; b < count; ++b)
            if (s < trajs[b].nsec)
                for (uint32_t g = 0; g < trajs[b].nchunks; ++g) tasks.push_back({(uint32_t)b, s, g, 0});
    std::vector<ScaleBlock> sblocks;
    for (int b = 0; b < count; ++b) {
        uint64_t nb = ((1ull << trajs[b].n) + 4095) >> 12;
        for (uint64_t k = 0; k < nb; ++k) sblocks.push_back({(uint32_t)b, (uint32_t)k});
    }
    const uint32_t ncounters = CTR_DONE + done;

    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t o_tr = 0;
    size_t o_tk = align(o_tr + trajs.size() * sizeof(BatchTraj));
    size_t o_ct = align(o_tk + tasks.size() * sizeof(BatchTask));
    size_t o_pt = align(o_ct + ncounters * sizeof(uint32_t));
    size_t o_sb = align(o_pt + std::max<uint32_t>(parts, 1) * sizeof(double));
    size_t o_se = align(o_sb + sblocks.size() * sizeof(ScaleBlock));
    size_t o_ph = align(o_se + secs.size() * sizeof(DevSection));
    size_t o_op = align(o_ph + phases.size() * sizeof(DevPhase));
    size_t o_m = align(o_op + ops.size() * sizeof(DevOp));
    size_t tot = align(o_m + mats.size() * es) + 256;
    std::vector<unsigned char> host(tot, 0);
    std::memcpy(host.data() + o_tr, trajs.data(), trajs.size() * sizeof(BatchTraj));
    std::memcpy(host.data() + o_tk, tasks.data(), tasks.size() * sizeof(BatchTask));
    std::memcpy(host.data() + o_sb, sblocks.data(), sblocks.size() * sizeof(ScaleBlock));
    std::memcpy(host.data() + o_se, secs.data(), secs.size() * sizeof(DevSection));
    std::memcpy(host.data() + o_ph, phases.data(), phases.size() * sizeof(DevPhase));
    std::memcpy(host.data() + o_op, ops.data(), ops.size() * sizeof(DevOp));
    for (size_t i = 0; i < mats.size(); ++i) {
        if (dt == QSV_C128) {
            double v[2] = {mats[i].real(), mats[i].imag()};
            std::memcpy(host.data() + o_m + i * es, v, es);
        } else {
            float v[2] = {(float)mats[i].real(), (float)mats[i].imag()};
            std::memcpy(host.data() + o_m + i * es, v, es);
        }
    }
    hipError_t e = hipMalloc(&L.block, tot);
    if (e != hipSuccess) {
        err = std::string("batch tables: ") + hipGetErrorString(e);
        return QSV_E_NOMEM;
    }
    e = hipMemcpy(L.block, host.data(), tot, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        err = std::string("batch table upload: ") + hipGetErrorString(e);
        return QSV_E_HIP;
    }
    unsigned char *base = (unsigned char *)L.block;
    L.trajs = (BatchTraj *)(base + o_tr);
    L.tasks = (BatchTask *)(base + o_tk);
    L.counters = (uint32_t *)(base + o_ct);
    L.parts = (double *)(base + o_pt);
    L.sblocks = (ScaleBlock *)(base + o_sb);
    L.secs = (DevSection *)(base + o_se);
    L.phases = (DevPhase *)(base + o_ph);
    L.ops = (DevOp *)(base + o_op);
    L.mats = base + o_m;
    L.ntasks = (uint32_t)tasks.size();
    L.ncounters = ncounters;
    L.nsblocks = (uint32_t)sblocks.size();
    L.count = (uint32_t)count;
    L.total_amps = total;
    L.r = r;
    L.kmax = kmax;
    L.lds = lds;
    {
        hipError_t ea = launch_batch_kernel(dt, L, nullptr, spin_limit);  // attributes only
        if (ea != hipSuccess) {
            err = std::string("batch kernel setup: ") + hipGetErrorString(ea);
            return QSV_E_HIP;
        }
    }
    L.grid = std::min<int>(batch_grid(dt, r, kmax, lds), (int)std::max<uint32_t>(1, L.ntasks));
    L.states = states;
    L.norms = norms;

    // capture: counters reset, init, persistent kernel, norms, rescale
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        err = std::string("capture stream: ") + hipGetErrorString(e);
        return QSV_E_HIP;
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const uint64_t nc = ncounters;
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, cs,
                           L.counters, nc);
        const unsigned ig = (unsigned)std::min<uint64_t>((total + 255) / 256, 256ull * 1024);
        if (dt == QSV_C128) {
            hipLaunchKernelGGL((k_batch_init<Cplx<double>>), dim3(ig), dim3(256), 0, cs,
                               (Cplx<double> *)states, total);
            hipLaunchKernelGGL((k_batch_ones<Cplx<double>>), dim3((count + 255) / 256), dim3(256),
                               0, cs, (Cplx<double> *)states, L.trajs, count);
        } else {
            hipLaunchKernelGGL((k_batch_init<Cplx<float>>), dim3(ig), dim3(256), 0, cs,
                               (Cplx<float> *)states, total);
            hipLaunchKernelGGL((k_batch_ones<Cplx<float>>), dim3((count + 255) / 256), dim3(256),
                               0, cs, (Cplx<float> *)states, L.trajs, count);
        }
        (void)launch_batch_kernel(dt, L, cs, spin_limit);
        hipLaunchKernelGGL(k_batch_norm, dim3(count), dim3(64), 0, cs, L.trajs, L.parts, L.counters,
                           norms);
        if (dt == QSV_C128)
            hipLaunchKernelGGL((k_batch_scale<Cplx<double>>), dim3(L.nsblocks), dim3(256), 0, cs,
                               (Cplx<double> *)states, L.trajs, L.sblocks, norms);
        else
            hipLaunchKernelGGL((k_batch_scale<Cplx<float>>), dim3(L.nsblocks), dim3(256), 0, cs,
                               (Cplx<float> *)states, L.trajs, L.sblocks, norms);
        hipError_t e2 = hipStreamEndCapture(cs, &L.graph);
        e = e2 == hipSuccess ? hipGetLastError() : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&L.exec, L.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        err = std::string("batch graph capture: ") + hipGetErrorString(e);
        return QSV_E_HIP;
    }
    return QSV_OK;
}

void batch_release(BatchLaunch &L) {
    if (L.exec) (void)hipGraphExecDestroy(L.exec);
    if (L.graph) (void)hipGraphDestroy(L.graph);
    if (L.block) (void)hipFree(L.block);
    L = BatchLaunch();
}

hipError_t batch_replay(const BatchLaunch &L, hipStream_t s) { return hipGraphLaunch(L.exec, s); }


}  // namespace qsv
