// Launch descriptors and launchers of the pipeline kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace esp {

// Systems sharing one window width P: one spread and one gather launch.
struct Group {
    int P;
    int off;         // first bin work item of the group
    int count;       // bin work items
    int lds_spread;  // LDS bytes per spread block, E^3 64-bit accumulators
    int lds_gather;  // LDS bytes per gather block, E^3 reals
};

// One launch set: the device descriptor table of the active systems, the
// work-item lists of every phase and the launch shapes. Buffers the systems
// use are reached through their descriptors.
struct Launch {
    int prec;             // 32 or 64
    int nsys;
    hipStream_t stream;
    const SysDesc* sys;
    const int2* pitems;   // particle chunks
    int n_pitems;
    const int2* titems;   // bins, grouped by P
    const int2* planes;   // (sys, x)
    int n_planes;
    const int4* cols;     // (sys, ky, kz0, width)
    int n_cols;
    int plane_bd, plane_maxit, plane_lds;
    int col_maxit, col_lds;
    int hist_lds;         // LDS bytes of the per-chunk histogram
    double* bpart;        // per particle chunk: sum q, sum |q|, sum q^2, max |q|
    double* epart;        // per x-column item: k-space energy partial
};

// Preparation phases: 0 per-chunk bin histograms, 1 scan, 2 scatter into
// bin order.
hipError_t launch_prepare(const Launch& L, int phase);
hipError_t launch_spread(const Launch& L, const Group& G);
// Diagnostics: fold the spread tiles into the real grid.
hipError_t launch_fold(const Launch& L);
// which: 0 forward z/y planes (mode 3: read the real grid instead of the
// spread tiles), 1 x-columns with scaling (mode 0 full, 1 forward only,
// 2 forward + scaling), 2 inverse y/z planes.
hipError_t launch_fft(const Launch& L, int which, int mode);
hipError_t launch_gather(const Launch& L, const Group& G);
hipError_t launch_finalize(const Launch& L, double* E_dev);
// Serving: apply each system's drift step to its resident FP32 positions.
hipError_t launch_drift(const Launch& L);

}  // namespace esp
