// Descriptors shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace esp {

// One system of a (possibly batched) plan. Every kernel reads the descriptor of
// its work item's system, so systems of different sizes share one launch.
struct SysDesc {
    int n;            // grid points per side
    int P;            // window width
    int N;            // particles
    int part_off;     // first particle in the concatenated arrays
    int tile_off;     // first bin in the bin arrays
    int tiles1;       // bins per side = ceil(n / T)
    int T;            // bin edge in grid points
    int degree;       // window polynomial degree
    long long grid_off;  // first real of the grid, n * n * (n + 2) reals
    int ts_off;       // radial influence table (3 (n/2)^2 + 1 entries)
    int tphi_off;     // per-axis influence table (n/2 + 1 entries)
    int poly_off;     // window polynomials, P * (degree + 1)
    int tw_off;       // twiddles exp(2 pi i t/n), n complex
    int col_off;      // first x-column work item of this system
    int ncol;         // number of x-column work items
    int pitem_off;    // first particle work item
    int npitem;       // number of particle work items
    int E;            // edge of a bin's window tile, T + P - 1 + (P odd)
    int hist_off;     // bin-major histogram / offset matrix, nbins x npitem
    long long tb_off; // first real of this system's bin tiles, nbins x E^3
    double inv_L;     // 1/L
    double s0;        // self constant S(0)
    double wmax3;     // cube of the window's peak value (fixed-point range)
};

// Work items: .x = system, .y (.z) = item coordinates inside the system.
//   particle chunk: (sys, first particle of a 256-chunk)
//   bin:            (sys, bin index within the system)
//   plane:          (sys, x)
//   x-column block: (sys, ky, kz0, width)

constexpr int kParticleChunk = 256;
constexpr int kMaxColumns = 16;

}  // namespace esp
