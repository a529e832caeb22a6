// Descriptors shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace esp {

// One system of a launch. Every kernel reads the descriptor of its work
// item's system, so systems of different sizes, whose buffers may live
// anywhere in device memory, share one launch per pipeline phase.
struct SysDesc {
    int n;            // grid points per side
    int P;            // window width
    int N;            // particles
    int T;            // bin edge in grid points (divides n)
    int tiles1;       // bins per side, n / T
    int E;            // edge of a bin's window tile, T + P - 1 + (P odd)
    int degree;       // window polynomial degree
    int npitem;       // particle-chunk work items of this system ...
    int pitem_off;    // ... starting at this index of the launch's list
    int ncol;         // x-column work items ...
    int col_off;      // ... starting here
    int small;        // 1: binned by one block (k_bin_small), 0: chunked kernels
    int mT;           // ceil(2^20 / T): x / T == (x mT) >> 20 for 0 <= x < 2^20 / T
    int mt1;          // ceil(2^20 / tiles1), likewise
    int ik;           // 1: forces by spectral derivatives (three gradient grids)
    int local;        // 1: local part of the split on the device (k_cellsort, k_local)
    int lcs;          // local: sub-cells per bin side (edge T / lcs >= rho / 2)
    int lR;           // local: stencil radius in sub-cells
    int ldeg;         // local: polynomial degree in x = r^2 / rho^2 (one piece on [0, 1))
    int lsa;          // local: sub-cells per side of a local work item's block (divides lcs)
    int litem_off;    // local: first local work item of the system in the launch's list ...
    int nlitem;       // ... and their count (bins x (lcs / lsa)^3)
    int fin_fft;      // 1: the last FFT pass (k_inv_yz) finalizes the energy; 0: k_finalize
    double inv_L;     // 1/L (x side)
    double inv_Ly;    // 1/Ly
    double inv_Lz;    // 1/Lz
    double side[3];   // L, Ly, Lz
    double nside[3];  // n/L, n/Ly, n/Lz (grid coordinate per length unit in a box)
    int tilt;         // 1: triclinic cell (grid coordinates n mod(H^-1 r, 1))
    double lay, laz;  // local: h_y/h_x, h_z/h_x (1 for a cubic box)
    // triclinic cell H = [a b c] = [[L, xy, xz], [0, Ly, yz], [0, 0, Lz]]: the
    // off-diagonal entries of H^-1 (grid coordinates u = n H^-1 r) and of
    // H / L (a grid-unit displacement in units of h_x = L/n); 0 otherwise
    double ixy, ixz, iyz;
    double mxy, mxz, myz;
    // ik: scale of the spectral derivative along each index axis, 1/L_d in a
    // box (Cartesian derivatives), 1 in a tilted cell (derivatives along the
    // fractional coordinates, mapped to Cartesian ones by H^-T in the gather)
    double ikx, iky, ikz;
    double s0;        // self constant S(0) of this box
    double pscale;    // influence scale: tables are made for a box of side n, p ~ 1/L
    double wmax3;     // cube of the window's peak value (fixed-point range)
    double lsT;       // local: lcs / T (sub-cell coordinate per grid unit)
    double lrho2;     // local: (rc / h)^2
    // tables shared by the systems of one parameter class
    const void* TS;   // radial influence table, 3 (n/2)^2 + 1 entries
    const void* Tphi; // per-axis influence table, n/2 + 1 entries
    const void* poly; // window polynomials, P * (degree + 1)
    const void* tw;   // twiddles exp(2 pi i t/n), n complex
    const void* lcoef;  // local: polynomials A then B, each zero-padded to 17 coefficients
    const void* p3;   // orthorhombic box: influence table p over the half spectrum,
                      // (x, ky, kz) like the grid; null for a cubic box (factored tables)
    // particles in the caller's order (this system's slice) and outputs
    const void* pos;  // N x 3
    const void* q;    // N
    void* phi;        // N or null
    void* F;          // N x 3 or null
    // scratch owned by the plan or server
    void* sorted;     // N x (v_x, v_y, v_z, q) in bin order, v = u - T (bin coordinates):
                      // grid coordinates relative to the bin's first cell
    int* perm;        // N: caller index of each sorted particle
    int* rank;        // N: rank within (chunk, bin)
    int* hist;        // nbins x npitem counts, then offsets
    int* bin_start;   // nbins + 1
    void* grid;       // n x n x (n + 2) reals (half spectrum in place)
    void* tiles;      // nbins x E^3 reals; before the spread, the scatter's staging
                      // (N 4-vectors, then N ints at the next 256-byte boundary)
    void* grad;       // ik only: three grids like `grid` (d/dx, d/dy, d/dz), each
                      // n x n x (n + 2) reals, one after another
    // local part (null unless local): particles reordered by sub-cell within
    // each bin, canonical order by caller index inside a sub-cell
    void* cpos;       // N x (u_x, u_y, u_z, q), sub-cell order
    int* cidx;        // N: sorted index of each sub-cell-ordered particle
    int* cstart;      // nbins lcs^3 + 1: first particle of every sub-cell
    void* loc;        // N x (u^l, F^l_x, F^l_y, F^l_z) in sorted order (the gather adds it)
    double* out;      // 8 doubles: E, sum q, sum |q|, sum q^2, fixed-point scale
    // serving: per-step drift of the resident positions (k_drift)
    unsigned long long seed;  // drift stream of the request
    int step;         // index of the drift to apply (0: none this iteration)
    float drift;      // amplitude: each coordinate moves by U(-drift, drift)
};

// Work items: .x = system index in the launch, .y (.z, .w) = position inside it.
//   particle chunk: (sys, first particle of a chunk of kParticleChunk)
//   bin:            (sys, bin index within the system)
//   plane:          (sys, x)
//   x-column block: (sys, first flattened (ky, kz) column, columns, 0)

#ifndef ESP_SMALL_MAX_N
#define ESP_SMALL_MAX_N 65536
#endif
constexpr int kSmallMaxN = ESP_SMALL_MAX_N;  // systems up to this size ...
constexpr int kSmallMaxBins = 512;    // ... and bin count are binned by one block
constexpr int kSmallRounds = 8192;    // deal rounds a one-block binning can hold
constexpr int kSmallMinSystems = 64;  // one-block binning pays only with this many systems,
constexpr int kSmallAlwaysN = 4096;   // or for systems this small (one launch instead of five)
// FP32 systems up to kSmallKeep x 1024 particles keep each particle's bin
// coordinates, bin, class and rank in registers from the one-block binning's
// counting pass to its placing pass, which then computes nothing again and
// reads no input (9 per thread: the 1024-thread block's 128 registers hold no
// more without spilling)
constexpr int kSmallKeep = 9;
constexpr int kParticleChunk = 1024;  // particles per chunk work item
constexpr int kScanRowsMax = 64;      // bins and chunks per system for k_scan to scan the rows itself
constexpr int kChunkThreads = 256;    // threads of a chunk block (4 particles each)
constexpr int kXcds = 8;              // accelerator complex dies (one L2 each) of the chip
// LDS bytes of a spread / gather block's window coefficients and their
// derivatives: 2 x P x 17 reals at most (P <= 12, degree <= 16, 8-byte reals)
constexpr int kCoefBytes = 2 * 12 * 17 * 8;
// A gather block's coefficient tables (window and derivative, 17 x P each),
// 16-byte aligned: the tile row offsets follow them in LDS
constexpr int gather_coef_bytes(int P, int rb) { return (2 * 17 * P * rb + 15) & ~15; }
constexpr int kOutDoubles = 8;
constexpr int kLocalCoefStride = 17;       // padded coefficients per local polynomial (degree <= 16)
constexpr int kLocalThreads = 256;          // threads of a local-part block
constexpr int kCellSortCap = 4096;          // particles of a bin sorted in LDS
constexpr double kLocalHaloTarget = 3000.0; // expected halo particles a local work item stages

}  // namespace esp
