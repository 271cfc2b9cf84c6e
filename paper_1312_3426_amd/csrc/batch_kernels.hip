// batch_kernels.hip -- the persistent form of the batching case: one launch
// per step advances every box of a batch (membrane forces, coupling and mesh
// update of every object, then the lattice update of every box; paper,
// Sections "Method" and "Elastic interactions").
//
// The launch holds as many workgroups as fit on the device at once.  Each
// takes tasks from a device ticket counter until the list is done: first the
// membrane tasks, one object each, largest mesh first; then the lattice
// tasks, one block of nodes of one box each, boxes in the order their
// membranes are expected to finish.  A lattice task of box b waits until all
// membrane tasks of box b have finished (a per-box counter), because it reads
// the coupling force they spread; it does not wait for other boxes, so the
// lattice update of a box whose cells are done overlaps the membranes of the
// others, and no launch boundary separates the two phases.
//
// Progress: a task only ever waits for tasks with smaller tickets, which were
// taken by workgroups already running, so the earliest unfinished task can
// always finish.  Each wait is bounded all the same (BatchSched::spin_limit);
// past it the task sets a flag the host reports and goes on, so every
// workgroup reaches the end of the list and the launch ends.
#include "batch_sched.h"
#include "lb_device.h"
#include "mesh_device.h"

namespace oif {
namespace {

using namespace dev;

// Call arguments arrive in vector registers and as generic pointers.  The
// task arguments are uniform across the workgroup and the descriptors they
// point to do not change during a launch, so the callees read them through
// the constant address space: scalar loads into scalar registers, as the
// per-phase kernels read theirs from kernel arguments.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> uniform(const T* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (cptr<T>)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The task bodies as calls rather than inlined: each keeps the register
// allocation it has in its own kernel (inlined side by side in one loop, the
// three membrane variants and the lattice update spilled heavily).
// The object descriptor field by field (a copy through the constant address
// space; a new field of ObjDev must be added here as well).
template <typename R>
__device__ __forceinline__ ObjDev<R> load_obj(cptr<ObjDev<R>> p) {
    static_assert(sizeof(ObjDev<R>) == (sizeof(R) == 8 ? 128 : 112), "ObjDev changed: update load_obj");
    ObjDev<R> o;
    o.t = p->t;
    o.box = p->box;
    o.X = p->X;
    o.V = p->V;
    o.geo = p->geo;
    o.F = p->F;
    o.frep = p->frep;
    o.node0 = p->node0;
    for (int k = 0; k < 3; ++k) o.anchor[k] = p->anchor[k];
    o.inv_mass = p->inv_mass;
    for (int k = 0; k < 3; ++k) o.fext[k] = p->fext[k];
    o.mass = p->mass;
    o.scratch = p->scratch;
    o.qsave = p->qsave;
    return o;
}

template <int P, bool USE_LDS, bool CPL>
__device__ __noinline__ void mesh_task(const ObjDev<typename Prec<P>::R>* O, unsigned char* smem, int parity) {
    const ObjDev<typename Prec<P>::R> o = load_obj(uniform(O));
    mesh_object<P, USE_LDS, true, CPL>(o, smem, uniform(parity), 0);
}
template <int P, bool NT>
__device__ __noinline__ void lb_task(const BoxDev* B, int blk, int nblk, int parity) {
    const cptr<BoxDev> b = uniform(B);
    blk = uniform(blk);
    nblk = uniform(nblk);
    parity = uniform(parity);
    for (int k = 0; k < nblk; ++k)
        lb_node<P, false, true, false, NT>(b, (blk + k) * (int)blockDim.x + (int)threadIdx.x, parity, LB_ALL);
}

template <int P, bool NT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(P == PREC_FP64 ? 1 : 6)))
batch_kernel(const BatchSched* __restrict__ S, int parity) {
    typedef typename Prec<P>::R R;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int ticket;
    const int nbox = S->nbox, nmesh = S->nmesh, ntasks = S->ntasks;
    // this step's counters: next ticket, workgroups done, wait-limit flag,
    // then finished membrane tasks per box (one set per step parity; the set
    // of a launch is cleared by its last workgroup for the launch after next)
    unsigned* ctr = S->ctr + (size_t)(parity & 1) * (3 + nbox);
    // Ordering between the two task kinds, with one device-scope fence per
    // task, issued by thread 0: a membrane task's threads meet at a barrier
    // and thread 0 then counts the task with a release increment; a lattice
    // task's thread 0 polls the count with relaxed loads, then acquires, and
    // the other threads follow it through a barrier.  (A device-scope fence in
    // every wave would write back and invalidate the L2 of its XCD once per
    // wave.)  Thread 0 publishes the finished membrane task in the same branch
    // that takes the next ticket, so each pass of the loop has one
    // single-thread region and it closes at a barrier: with a second such
    // region at the end of the membrane branch the two can be merged across
    // the back edge, which leaves the ticket barrier inside a loop that
    // thread 0 has already left.
    int done_box = -1;
    for (;;) {
        if (threadIdx.x == 0) {
            if (done_box >= 0)
                __hip_atomic_fetch_add(&ctr[3 + done_box], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            ticket = (int)atomicAdd(&ctr[0], 1u);
        }
        __syncthreads();
        // uniform across the workgroup: task descriptors go to scalar registers
        const int t = __builtin_amdgcn_readfirstlane(ticket);
        __syncthreads();  // every thread has read the ticket before it is replaced
        if (t >= ntasks) break;
        if (t < nmesh) {
            const ObjDev<R>* O = (const ObjDev<R>*)S->objs + t;
            const int g = __builtin_amdgcn_readfirstlane(S->group[t]);
            if (g == 0) mesh_task<P, true, false>(O, smem, parity);
            else if (g == 1) mesh_task<P, false, true>(O, smem, parity);
            else mesh_task<P, false, false>(O, smem, parity);
            __syncthreads();  // all threads' spreading is done before thread 0 counts the task
            done_box = __builtin_amdgcn_readfirstlane(S->obj_box[t]);
        } else {
            done_box = -1;
            const int2 w = S->lbwork[t - nmesh];  // (box, first block of nodes)
            if (threadIdx.x == 0) {
                const unsigned want = (unsigned)S->box_nmesh[w.x];
                unsigned long long spins = 0;
                while (__hip_atomic_load(&ctr[3 + w.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                    if (++spins > S->spin_limit) {
                        atomicOr(&ctr[2], 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the box's spread forces
            }
            __syncthreads();
            lb_task<P, NT>(S->boxes + w.x, w.y, S->lb_chunk, parity);
        }
    }
    // the last workgroup to finish clears this parity's counters (the flag
    // stays for the host)
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&ctr[1], 1u) == gridDim.x - 1) {
            for (int b = 0; b < nbox; ++b) ctr[3 + b] = 0u;
            ctr[0] = 0u;
            ctr[1] = 0u;
            __threadfence();
        }
    }
}

template <int P, bool NT>
const void* batch_fn() {
    return (const void*)batch_kernel<P, NT>;
}

const void* batch_fn(int precision, int nt) {
    switch (precision) {
        case PREC_FP64: return nt ? batch_fn<PREC_FP64, true>() : batch_fn<PREC_FP64, false>();
        case PREC_FP32: return nt ? batch_fn<PREC_FP32, true>() : batch_fn<PREC_FP32, false>();
        case PREC_FP16: return nt ? batch_fn<PREC_FP16, true>() : batch_fn<PREC_FP16, false>();
        case PREC_BF16: return nt ? batch_fn<PREC_BF16, true>() : batch_fn<PREC_BF16, false>();
        default: return nullptr;
    }
}

}  // namespace

hipError_t batch_blocks_per_cu(int precision, int nt, int block, size_t lds_bytes, int* per_cu) {
    const void* f = batch_fn(precision, nt);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, block, lds_bytes);
}

hipError_t launch_batch(const BatchLaunch& L) {
    const void* f = batch_fn(L.precision, L.nt);
    if (!f || L.grid <= 0) return hipErrorInvalidValue;
    void* args[] = {(void*)&L.sched, (void*)&L.parity};
    return hipLaunchKernel(f, dim3(L.grid), dim3(L.block), args, L.lds_bytes, L.stream);
}

}  // namespace oif
