// Batched trajectories: many independent states of uneven qubit counts (the
// paper's shots / noisy simulation, Sec. III-A and IV-B) in one graph launch.
//
// Section depth d of every trajectory that has one runs in one kernel: a
// workgroup per (trajectory, chunk) of that section, so a large trajectory's
// chunks spread over the whole GPU while small trajectories (one chunk, one
// section) finish in the first kernel.  Consecutive depths are ordered by the
// kernel boundaries of the graph (no workgroup ever waits on another).  The
// last section of a trajectory writes each chunk's FP64 norm; a reduction in
// chunk order gives the state's norm and a final kernel rescales every state by
// 1/sqrt(norm).  The whole sequence (init, depth kernels, norms, rescale) is
// captured once into a HIP graph and replayed.
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
    uint32_t nchunks;     // chunks per section
    uint32_t part_off;    // first of its per-chunk norm partials
    uint32_t pad;
};

struct BatchItem {       // one workgroup of a depth kernel
    uint32_t traj;
    uint32_t chunk;
};


constexpr int BATCH_THREADS = 256;

// Section `depth` of every trajectory listed in items: one workgroup per
// (trajectory, chunk).  Transpositions move whole amplitudes (a buffer of the
// chunk's size): trajectory states are small and largely cache-resident, so
// the two extra barriers of a component-wise transposition cost more here than
// the extra workgroup per CU it allows would recover.
template <typename T, int R, int KMAX>
__global__ void __launch_bounds__(BATCH_THREADS)
k_batch_step(typename Amp<T>::V *__restrict__ states, const BatchTraj *__restrict__ trajs,
             const BatchItem *__restrict__ items, uint32_t depth, double *__restrict__ partials,
             const DevSection *__restrict__ secs_g, const DevPhase *__restrict__ phases_g,
             const DevOp *__restrict__ ops_g, const typename Amp<T>::V *__restrict__ mats_g) {
    using V = typename Amp<T>::V;
    extern __shared__ unsigned char lds_raw[];
    V *lds = reinterpret_cast<V *>(lds_raw);
    __shared__ double s_red[BATCH_THREADS];
    const unsigned tid = threadIdx.x;
    const BatchItem it = items[blockIdx.x];
    const BatchTraj tr = trajs[it.traj];
    V *st = states + tr.state_off;
    const cptr<DevSection> S = (cptr<DevSection>)secs_g + (tr.sec_begin + depth);
    const bool active = tid < (1u << (S->c - R));
    // complex64 matrices are read into VGPRs (FP32 FMAs with SGPR operands
    // issue at half rate): 4.6 % faster on the 512-trajectory workload
    if (depth + 1 == tr.nsec) {
        const double nrm = run_chunk_norm<T, R, KMAX, false, sizeof(T) == 4>(st, S, (cptr<DevPhase>)phases_g,
                                                      (cptr<DevOp>)ops_g, (cptr<V>)mats_g, nullptr,
                                                      it.chunk, lds, s_red, active);
        if (tid == 0) partials[tr.part_off + it.chunk] = nrm;
    } else {
        run_chunk<T, R, KMAX, false, false, sizeof(T) == 4>(st, S, (cptr<DevPhase>)phases_g, (cptr<DevOp>)ops_g,
                              (cptr<V>)mats_g, nullptr, it.chunk, lds, active);
    }
}

// norms[b] = sum of trajectory b's chunk partials, in chunk order
__global__ void __launch_bounds__(256)
k_batch_norms(const BatchTraj *__restrict__ trajs, const double *__restrict__ partials,
              double *__restrict__ norms, int count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const BatchTraj tr = trajs[b];
    double s = 0.0;
    for (uint32_t g = 0; g < tr.nchunks; ++g) s += partials[tr.part_off + g];
    norms[b] = s;
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


// ---------------------------------------------------------------------------

}  // namespace qsv
#include "batch.hpp"
namespace qsv {

static hipError_t launch_batch_kernel(qsv_dtype dt, const BatchLaunch &L, uint32_t depth,
                                      hipStream_t s);

template <typename T, int R, int KMAX>
static hipError_t launch_batch_t(const BatchLaunch &L, uint32_t depth, hipStream_t s) {
    using V = typename Amp<T>::V;
    if (!s) {  // setup call (outside any stream capture)
        return hipFuncSetAttribute((const void *)k_batch_step<T, R, KMAX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    }
    hipLaunchKernelGGL((k_batch_step<T, R, KMAX>), dim3(L.depth_count[depth]), dim3(BATCH_THREADS),
                       L.lds, s, (V *)L.states, L.trajs, L.items + L.depth_off[depth], depth,
                       L.partials, L.secs, L.phases, L.ops, (const V *)L.mats);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_batch_dt(const BatchLaunch &L, uint32_t depth, hipStream_t s) {
    const bool wide = L.kmax > 2;
    switch (L.r) {
        case 3: return wide ? launch_batch_t<T, 3, 3>(L, depth, s) : launch_batch_t<T, 3, 2>(L, depth, s);
        case 4: return wide ? launch_batch_t<T, 4, 4>(L, depth, s) : launch_batch_t<T, 4, 2>(L, depth, s);
        case 5: return wide ? launch_batch_t<T, 5, 5>(L, depth, s) : launch_batch_t<T, 5, 2>(L, depth, s);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_batch_kernel(qsv_dtype dt, const BatchLaunch &L, uint32_t depth,
                                      hipStream_t s) {
    if (dt == QSV_C128) return launch_batch_dt<double>(L, depth, s);
    return launch_batch_dt<float>(L, depth, s);
}

// Build (or fetch) the batch launch for these plans/buffers; captures the graph.
qsv_status batch_prepare(qsv_dtype dt, int count, const Plan *const *plans,
                         const uint64_t *offsets, void *states, double *norms,
                         BatchLaunch &L, std::string &err) {
    const size_t es = dt == QSV_C128 ? 16 : 8;
    const int r = plans[0]->r;
    int kmax = 1;
    size_t lds = 0;
    std::vector<BatchTraj> trajs(count);
    std::vector<DevSection> secs;
    std::vector<DevPhase> phases;
    std::vector<DevOp> ops;
    std::vector<cd> mats;
    uint32_t maxS = 0;
    uint64_t total = 0;
    uint64_t npart = 0;
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
        if (P.n_params > 0 || P.opt.swap_mode != QSV_SWAP_REMAP ||
            lds_resident(P.opt)) {
            // paired tables are ordinary register phases (dense ops at fixed positions)
            err = "batch plans must be remap-mode register-phase plans without parameters";
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
        t.nchunks = (uint32_t)(1ull << (P.n - P.c));
        t.part_off = (uint32_t)npart;
        t.pad = 0;
        npart += t.nchunks;
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
    // largest trajectories first (they bound the launch's duration)
    std::vector<uint32_t> order(count);
    for (int k = 0; k < count; ++k) order[k] = (uint32_t)k;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return trajs[x].n > trajs[y].n; });
    // work items of each section depth: (trajectory, chunk), largest trajectories first
    std::vector<BatchItem> items;
    L.depth_off.assign(maxS, 0);
    L.depth_count.assign(maxS, 0);
    for (uint32_t d = 0; d < maxS; ++d) {
        L.depth_off[d] = (uint32_t)items.size();
        for (uint32_t b : order)
            if (d < trajs[b].nsec)
                for (uint32_t g = 0; g < trajs[b].nchunks; ++g) items.push_back({b, g});
        L.depth_count[d] = (uint32_t)items.size() - L.depth_off[d];
    }
    std::vector<ScaleBlock> sblocks;
    for (int b = 0; b < count; ++b) {
        uint64_t nb = ((1ull << trajs[b].n) + 4095) >> 12;
        for (uint64_t k = 0; k < nb; ++k) sblocks.push_back({(uint32_t)b, (uint32_t)k});
    }

    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t o_tr = 0;
    size_t o_sb = align(o_tr + trajs.size() * sizeof(BatchTraj));
    size_t o_it = align(o_sb + sblocks.size() * sizeof(ScaleBlock));
    size_t o_pa = align(o_it + items.size() * sizeof(BatchItem));
    size_t o_se = align(o_pa + npart * sizeof(double));
    size_t o_ph = align(o_se + secs.size() * sizeof(DevSection));
    size_t o_op = align(o_ph + phases.size() * sizeof(DevPhase));
    size_t o_m = align(o_op + ops.size() * sizeof(DevOp));
    size_t tot = align(o_m + mats.size() * es) + 256;
    std::vector<unsigned char> host(tot, 0);
    std::memcpy(host.data() + o_tr, trajs.data(), trajs.size() * sizeof(BatchTraj));
    std::memcpy(host.data() + o_sb, sblocks.data(), sblocks.size() * sizeof(ScaleBlock));
    std::memcpy(host.data() + o_it, items.data(), items.size() * sizeof(BatchItem));
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
    L.sblocks = (ScaleBlock *)(base + o_sb);
    L.items = (BatchItem *)(base + o_it);
    L.partials = (double *)(base + o_pa);
    L.secs = (DevSection *)(base + o_se);
    L.phases = (DevPhase *)(base + o_ph);
    L.ops = (DevOp *)(base + o_op);
    L.mats = base + o_m;
    L.nsblocks = (uint32_t)sblocks.size();
    L.count = (uint32_t)count;
    L.total_amps = total;
    L.r = r;
    L.kmax = kmax;
    L.lds = lds;
    {
        hipError_t ea = launch_batch_kernel(dt, L, 0, nullptr);  // attributes only
        if (ea != hipSuccess) {
            err = std::string("batch kernel setup: ") + hipGetErrorString(ea);
            return QSV_E_HIP;
        }
    }
    L.states = states;
    L.norms = norms;

    // capture: init, one kernel per section depth, norms, rescale
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        err = std::string("capture stream: ") + hipGetErrorString(e);
        return QSV_E_HIP;
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
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
        for (uint32_t d = 0; d < maxS; ++d)
            if (L.depth_count[d] > 0) (void)launch_batch_kernel(dt, L, d, cs);
        hipLaunchKernelGGL(k_batch_norms, dim3((count + 255) / 256), dim3(256), 0, cs, L.trajs,
                           L.partials, norms, count);
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
