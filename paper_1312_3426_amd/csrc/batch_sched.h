// batch_sched.h -- task list of the persistent batch kernel (batch_kernels.hip)
// and its launcher.  Internal to liboif.so.
#pragma once

#include "oif_device.h"

namespace oif {

struct BatchSched {
    int ntasks;                  // membrane tasks, then lattice tasks
    int nmesh;                   // membrane tasks (one object each)
    int nbox;
    const void* objs;            // ObjDev<real>[nmesh] in task order
    const unsigned char* group;  // [nmesh] 0: mesh in LDS; 1: mesh in the scratch, coupling area in
                                 // LDS; 2: all in the scratch
    const int* obj_box;          // [nmesh] box of each membrane task
    const int2* lbwork;          // [ntasks - nmesh] (box, first block of blockDim nodes)
    int lb_chunk;                // blocks of nodes per lattice task
    const BoxDev* boxes;         // [nbox]
    const int* box_nmesh;        // [nbox] membrane tasks per box
    unsigned* ctr;               // [2][3 + nbox] per step parity: next ticket, workgroups done,
                                 // wait-limit flag, finished membrane tasks per box
    unsigned long long spin_limit;  // polls of a lattice task's wait before it gives up
};

struct BatchLaunch {
    const BatchSched* sched;     // device copy
    int grid, block;
    size_t lds_bytes;
    int parity;
    int precision;
    int nt;                      // non-temporal population reads
    hipStream_t stream;
};

// Workgroups of `block` threads with `lds_bytes` of dynamic LDS that fit on one
// compute unit (also allows that much dynamic LDS for the kernel).
hipError_t batch_blocks_per_cu(int precision, int nt, int block, size_t lds_bytes, int* per_cu);
hipError_t launch_batch(const BatchLaunch& L);

}  // namespace oif
