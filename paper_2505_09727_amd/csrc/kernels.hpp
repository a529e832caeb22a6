// Launch descriptors and launchers of the pipeline kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace esp {

// Systems of one lane sharing one window width P: one spread and one gather
// launch.
struct Group {
    int P;
    int lane;        // the pipeline lane of its systems
    int off;         // first entry of the group in the XCD-ordered bin list
    int count;       // its entries: kXcds runs of count / kXcds, padding (-1, -1) included
    int lds_spread;  // LDS bytes per spread block: E^3 accumulators, coefficients
    int lds_gather;  // LDS bytes per gather block: E^3 reals, coefficients, E^2 row offsets
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
    int n_titems;
    const int2* xitems;   // the same bins per group in XCD order, for the spread and the gather
    const int2* planes;   // (sys, x), grouped by grid size
    int n_planes;
    const int4* cols;     // (sys, first column, columns, 0), grouped by grid size
    int n_cols;
    const int2* fsys;     // (sys, 0) of systems on the one-block transform, grouped by grid size
    int hist_lds;         // LDS bytes of the per-chunk histogram
    int any_ik;           // some system takes ik forces (x pass keeps two column buffers)
    int n_large;          // systems binned by the chunked kernels
    const int2* bsys;     // (sys, 0) of systems binned by one block
    int n_small;
    int small_lds;        // LDS bytes of the one-block binning
    double* bpart;        // per particle chunk: sum q, sum |q|, sum q^2, max |q|
    double* epart;        // per x-column item: k-space energy partial
    const int2* litems;   // local pass: (sys, bin x (lcs/lsa)^3 + block within the bin)
    int n_litems;
    double* lpart;        // per local item: local-part energy partial, sum q u^l
    int any_local;        // some system evaluates the local part
    int scan_rows_fused;  // every chunked system has <= kScanRowsMax bins and chunks: k_scan scans the rows
    int any_fin_kernel;   // some system is finalized by k_finalize (fused FFT), not by k_inv_yz
    int local_cap;        // particles of a bin's halo the local pass stages in LDS
    int local_cells;      // largest halo sub-cell count, (lcs + 2 lR)^3
    int local_deg;        // largest local-part polynomial degree
};

// Systems sharing one grid size n: one launch per FFT pass.
struct FftGroup {
    int n;
    int lane;                    // the pipeline lane of its systems
    int fused;                   // 1: one block per system for the whole transform
    int xreg;                    // 1: x pass with one column per thread (k_fft_x_reg)
    int plane_off, plane_count;  // x-plane work items (three-pass path)
    int col_off, col_count;      // x-column chunk work items (three-pass path)
    int sys_off, sys_count;      // system work items (fused path)
};

// Grid sizes with FFT kernels (even 2^a 3^b up to 144).
inline bool fft_size_supported(int n) {
    static const int sizes[] = {8, 12, 16, 18, 24, 32, 36, 48, 54, 64, 72, 96, 108, 128, 144};
    for (int s : sizes)
        if (s == n) return true;
    return false;
}
// Columns per x-pass block: 256-byte runs of complex values.
inline int fft_x_columns(int prec) { return prec == 64 ? 16 : 32; }
// Grid sizes whose x pass keeps each column in one thread's registers
// (k_fft_x_reg; systems with AD forces), with its columns per block (one
// wave): FP32 n in [40, 64]; smaller grids run faster on the LDS stages.
inline bool fft_x_in_registers(int n, int prec) { return prec == 32 && n >= 40 && n <= 64; }
constexpr int kXRegColumns = 64;
// Dynamic LDS bytes of the plane passes (twiddles, one half-spectrum plane,
// covering tables of the halo fold) and of the x pass.
inline int fft_plane_lds(int n, int prec) {
    const int rb = prec == 64 ? 8 : 4;
    return (n + n * (n / 2 + 1)) * 2 * rb + (n + 1) * 9 * 4;
}
inline int fft_x_lds(int n, int prec, bool ik = false) {
    const int rb = prec == 64 ? 8 : 4;
    return (n + (ik ? 2 : 1) * n * fft_x_columns(prec)) * 2 * rb;
}
// Dynamic LDS of the one-block transform (twiddles, the whole half spectrum,
// covering tables); the path is taken when this fits in 160 KB.
inline int fft_fused_lds(int n, int prec) {
    const int rb = prec == 64 ? 8 : 4;
    return (n + n * n * (n / 2 + 1)) * 2 * rb + (n + 1) * 9 * 4;
}

// Preparation phases: 0 per-chunk bin histograms, 1 scan, 2 scatter into
// bin order and deal each bin into LDS bank classes. Phase 0 also bins the
// systems binned by one block (k_bin_small) unless with_small is false, in
// which case launch_bin_small does that, say on another stream.
hipError_t launch_prepare(const Launch& L, int phase, bool with_small = true);
hipError_t launch_bin_small(const Launch& L);
hipError_t launch_spread(const Launch& L, const Group& G);
// Diagnostics: fold the spread tiles into the real grid.
hipError_t launch_fold(const Launch& L);
// which: 0 forward z/y planes, 1 x-columns with scaling, 2 inverse y/z
// planes. For which = 0, mode & 3 == 3 reads the real grid instead of the
// spread tiles and mode >> 2 is the x-pass mode; for which = 1 the mode is
// 0 full, 1 forward only, 2 forward + scaling. A fused group runs its whole
// transform at which = 0 (with mode >> 2) and nothing at 1 and 2.
// which 2 (the last pass) also finalizes the energy of systems with fin_fft,
// writing E_dev[sys] when E_dev is non-null.
hipError_t launch_fft(const Launch& L, const FftGroup& G, int which, int mode, double* E_dev = nullptr);
hipError_t launch_gather(const Launch& L, const Group& G);
hipError_t launch_finalize(const Launch& L, double* E_dev);
// Local part of the split (systems with local = 1): sub-cell order, then the
// pair sums into the per-particle buffer the gather adds and the per-bin
// energy partials k_finalize adds.
hipError_t launch_local(const Launch& L);
// Serving: apply each system's drift step to its resident FP32 positions.
hipError_t launch_drift(const Launch& L);

}  // namespace esp
