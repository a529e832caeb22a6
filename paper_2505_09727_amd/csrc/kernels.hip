// HIP kernels of the ESP long-range pipeline for gfx950 (CDNA4, wave64).
//
// Pipeline (Methods, "Fast algorithm for the spectral part"):
//   bin + counting sort -> spread (eq. spread) -> forward 3D FFT ->
//   diagonal scaling by p_k (eq. pk) with the k-space energy ->
//   inverse 3D FFT -> interpolation with analytic window derivatives (eq. interp,
//   AD forces) -> energy finalisation.
//
// Every kernel walks a work-item list, so one launch serves a batch of systems
// of different sizes. Real grids are stored n x n x (n+2) so that the half
// spectrum n x n x (n/2+1) of each x-plane overwrites that plane in place.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace esp {

// x / d for 0 <= x < 2^20 / d with m = ceil(2^20 / d) (the error term of m
// times x stays below 2^20).
__device__ __forceinline__ int fdiv(int x, int m) {
    return (int)(((unsigned long long)(unsigned)x * (unsigned)m) >> 20);
}

// x mod L for L > 0, as the definition takes it (fmod, then + L for a
// negative remainder); x itself inside [0, L).
__device__ __forceinline__ double mod_side(double x, double L) {
    if (x >= 0.0 && x < L) return x;
    double t = fmod(x, L);
    if (t < 0.0) t = __dadd_rn(t, L);
    return t;
}

// Grid coordinates of a particle and its bin, in FP64 with the definition's
// operations: u_d = mod(x_d, L_d) (n / L_d) in a box, u = n mod(H^-1 r, 1) in
// a triclinic cell (H^-1 upper triangular, each row summed left to right),
// u in [0, n) (u = n, a rounding of the last representable position, is the
// periodic image 0). The cells floor(u), and with them the bin and the first
// point of every window (l0 = floor(u - P/2) + 1), are therefore decided in
// FP64. The coordinates are kept relative to the bin's first cell, v = u -
// T t_d in [0, T), rounded toward zero in FP32: the window boundaries (whole
// and half grid points) are representable, so floor(v - P/2) is the FP64
// decision exactly, and v keeps T/n times the absolute precision of u.
template <typename R>
struct BinCoords {
    R vx, vy, vz;
    int tx, ty, tz, bin;
};

template <typename R>
__device__ __forceinline__ R to_bin_real(double v);
template <>
__device__ __forceinline__ float to_bin_real<float>(double v) {
    return __double2float_rz(v);
}
template <>
__device__ __forceinline__ double to_bin_real<double>(double v) {
    return v;
}

template <typename R>
__device__ __forceinline__ BinCoords<R> bin_coords_of(const SysDesc& S, double x, double y, double z) {
    const double n = (double)S.n;
    double u[3];
    if (S.tilt) {
        const double sx = __dadd_rn(__dadd_rn(__dmul_rn(x, S.inv_L), __dmul_rn(y, S.ixy)), __dmul_rn(z, S.ixz));
        const double sy = __dadd_rn(__dmul_rn(y, S.inv_Ly), __dmul_rn(z, S.iyz));
        const double sz = __dmul_rn(z, S.inv_Lz);
        u[0] = __dmul_rn(mod_side(sx, 1.0), n);
        u[1] = __dmul_rn(mod_side(sy, 1.0), n);
        u[2] = __dmul_rn(mod_side(sz, 1.0), n);
    } else {
        u[0] = __dmul_rn(mod_side(x, S.side[0]), S.nside[0]);
        u[1] = __dmul_rn(mod_side(y, S.side[1]), S.nside[1]);
        u[2] = __dmul_rn(mod_side(z, S.side[2]), S.nside[2]);
    }
    BinCoords<R> b;
    int t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (u[d] >= n) u[d] = __dadd_rn(u[d], -n);
        const int c = min((int)u[d], S.n - 1);
        t[d] = fdiv(c, S.mT);
    }
    b.tx = t[0];
    b.ty = t[1];
    b.tz = t[2];
    b.vx = to_bin_real<R>(__dadd_rn(u[0], -(double)(t[0] * S.T)));
    b.vy = to_bin_real<R>(__dadd_rn(u[1], -(double)(t[1] * S.T)));
    b.vz = to_bin_real<R>(__dadd_rn(u[2], -(double)(t[2] * S.T)));
    b.bin = (t[0] * S.tiles1 + t[1]) * S.tiles1 + t[2];
    return b;
}

// Coordinates (tx, ty, tz) of bin t.
__device__ __forceinline__ void bin_coords(int t, const SysDesc& S, int& tx, int& ty, int& tz) {
    const int r = fdiv(t, S.mt1);
    tz = t - r * S.tiles1;
    tx = fdiv(r, S.mt1);
    ty = r - tx * S.tiles1;
}

// ---------------------------------------------------------------------------
// Binning without global atomics.
//
// k_hist: one block per chunk of kParticleChunk particles of one system. Grid
// coordinates, bin id, and the rank of the particle among the chunk's
// particles of the same bin (LDS atomics); the chunk's bin counts go to column
// `item` of the system's bin-major count matrix (plain stores). Also the chunk
// sums of q, |q|, q^2 and max |q| (neutrality check, self energy, fixed-point
// range of the spread).
template <typename R>
__global__ void __launch_bounds__(kChunkThreads) k_hist(const SysDesc* __restrict__ sys,
                                                        const int2* __restrict__ items, double* __restrict__ bpart) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int* cnt = reinterpret_cast<int*>(smem_raw);
    __shared__ double red[64];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (S.small) return;  // uniform over the block
    const int t1 = S.tiles1, nb = t1 * t1 * t1;
    for (int b = threadIdx.x; b < nb; b += kChunkThreads) cnt[b] = 0;
    __syncthreads();
    double sq = 0.0, sa = 0.0, s2 = 0.0, qm = 0.0;
    const R* pos = reinterpret_cast<const R*>(S.pos);
    const R* q = reinterpret_cast<const R*>(S.q);
#pragma unroll
    for (int k = 0; k < kParticleChunk / kChunkThreads; ++k) {
        const int il = wi.y + threadIdx.x + k * kChunkThreads;
        if (il < S.N) {
            const BinCoords<R> bc = bin_coords_of<R>(S, pos[3 * il + 0], pos[3 * il + 1], pos[3 * il + 2]);
            S.rank[il] = atomicAdd(&cnt[bc.bin], 1);
            const double qq = (double)q[il];
            sq += qq;
            sa += fabs(qq);
            s2 += qq * qq;
            qm = fmax(qm, fabs(qq));
        }
    }
    __syncthreads();
    const int it = blockIdx.x - S.pitem_off;
    for (int b = threadIdx.x; b < nb; b += kChunkThreads) S.hist[b * S.npitem + it] = cnt[b];
    block_sum3_max(sq, sa, s2, qm, red);
    if (threadIdx.x == 0) {
        bpart[4 * blockIdx.x + 0] = sq;
        bpart[4 * blockIdx.x + 1] = sa;
        bpart[4 * blockIdx.x + 2] = s2;
        bpart[4 * blockIdx.x + 3] = qm;
    }
}

// Exclusive scan of each bin's row of the count matrix (one wave per bin):
// entry (bin, item) becomes the first slot of that chunk's particles within
// the bin, and the bin's total goes to bin_start[bin] (turned into the bin's
// first slot by k_scan).
__global__ void __launch_bounds__(256) k_scan_rows(const SysDesc* __restrict__ sys, const int2* __restrict__ items,
                                                   int n_items) {
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_items) return;  // uniform over the wave
    const int2 wi = items[w];
    const SysDesc& S = sys[wi.x];
    if (S.small) return;  // uniform over the wave
    const int lane = threadIdx.x & 63;
    int* row = S.hist + (size_t)wi.y * S.npitem;
    int carry = 0;
    for (int base = 0; base < S.npitem; base += 64) {
        const int l = base + lane;
        const int v = l < S.npitem ? row[l] : 0;
        int x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (l < S.npitem) row[l] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    if (lane == 0) S.bin_start[wi.y] = carry;
}

// Per system (one block): exclusive scan of the bin totals into the bins'
// first slots, and the fixed-point scale of the FP32 spread: 2^F with every
// single term |q w_x w_y w_z| 2^F <= 2^30, so it is exact through int32.
// With `rows` (every chunked system has at most kScanRowsMax bins and chunks)
// the block first does k_scan_rows' work itself, one wave per bin with all of
// its rows' loads issued first, and keeps the totals in LDS: one launch fewer.
__global__ void __launch_bounds__(1024) k_scan(const SysDesc* __restrict__ sys, const double* __restrict__ bpart,
                                               int rows) {
    __shared__ int warp_tot[16];
    __shared__ double red[16];
    __shared__ int tot[kScanRowsMax];
    const SysDesc& S = sys[blockIdx.x];
    if (S.small) return;  // uniform over the block
    if (rows) {
        constexpr int RW = kScanRowsMax / 16;  // rows per wave
        const int nbr = S.tiles1 * S.tiles1 * S.tiles1, np = S.npitem;
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        int v[RW];
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int b = wid + 16 * k;
            v[k] = b < nbr && lane < np ? S.hist[(size_t)b * np + lane] : 0;
        }
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int b = wid + 16 * k;
            if (b < nbr) {  // uniform over the wave
                int x = v[k];
                for (int off = 1; off < 64; off <<= 1) {
                    const int y = __shfl_up(x, off, 64);
                    if (lane >= off) x += y;
                }
                if (lane < np) S.hist[(size_t)b * np + lane] = x - v[k];
                if (lane == 63) tot[b] = x;
            }
        }
        __syncthreads();
    }
    auto total = [&](int b) { return rows ? tot[b] : S.bin_start[b]; };
    {
        double qm = 0.0;
        for (int i = threadIdx.x; i < S.npitem; i += blockDim.x) qm = fmax(qm, bpart[4 * (S.pitem_off + i) + 3]);
        qm = block_max(qm, red);
        if (threadIdx.x == 0) {
            const double bound = qm * S.wmax3;
            const int F = bound > 0.0 ? 30 - (int)ceil(log2(bound)) : 30;
            S.out[4] = ldexp(1.0, max(-100, min(100, F)));
        }
    }
    const int t1 = S.tiles1, nb = t1 * t1 * t1;
    // each thread owns a contiguous run of bins (at most a few)
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    int run = 0;
    for (int b = b0; b < b1; ++b) run += total(b);
    int x = run;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) warp_tot[wid] = x;
    __syncthreads();
    int off = x - run;
    for (int w = 0; w < wid; ++w) off += warp_tot[w];
    for (int b = b0; b < b1; ++b) {
        const int v = total(b);
        S.bin_start[b] = off;
        off += v;
    }
    if (threadIdx.x == 0) S.bin_start[nb] = S.N;
}

// Staging of the scatter's output in the tile buffer (the tiles are written
// later, by the spread).
template <typename R>
__device__ __forceinline__ typename Vec4<R>::type* stage_vals(const SysDesc& S) {
    return reinterpret_cast<typename Vec4<R>::type*>(S.tiles);
}
template <typename R>
__device__ __forceinline__ int* stage_perm(const SysDesc& S) {
    const size_t off = ((size_t)S.N * sizeof(typename Vec4<R>::type) + 255) & ~size_t(255);
    return reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(S.tiles) + off);
}

// Scatter particles into bin order as (v_x, v_y, v_z, q) (bin coordinates)
// with their caller indices, into the staging area; the dealing pass writes
// the final order.
template <typename R>
__global__ void __launch_bounds__(kChunkThreads) k_scatter(const SysDesc* __restrict__ sys,
                                                           const int2* __restrict__ items) {
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (S.small) return;  // uniform over the block
    const R* pos = reinterpret_cast<const R*>(S.pos);
    const int* hcol = S.hist + (blockIdx.x - S.pitem_off);
#pragma unroll
    for (int k = 0; k < kParticleChunk / kChunkThreads; ++k) {
        const int il = wi.y + threadIdx.x + k * kChunkThreads;
        if (il < S.N) {
            const BinCoords<R> bc = bin_coords_of<R>(S, pos[3 * il + 0], pos[3 * il + 1], pos[3 * il + 2]);
            const int bin = bc.bin;
            const int dst = S.bin_start[bin] + hcol[bin * S.npitem] + S.rank[il];
            typename Vec4<R>::type v;
            v.x = bc.vx;
            v.y = bc.vy;
            v.z = bc.vz;
            v.w = reinterpret_cast<const R*>(S.q)[il];
            stage_vals<R>(S)[dst] = v;
            stage_perm<R>(S)[dst] = il;
        }
    }
}

// Dealing: write the particles of each bin from the staging area to the
// sorted arrays in an order where consecutive particles fall in distinct LDS
// bank classes. A particle's class is the linear index, in its bin's E^3
// tile, of the first entry of its window, mod 32; every tile access of the
// spread and the gather is that index plus an offset common to all
// particles, so lanes holding particles of distinct classes hit distinct
// banks on every access. The order lists round j = 0, 1, ... where round j
// holds the j-th staged particle of every class that has one, in class order.
// Any order within a bin gives the same results; a bin whose largest class
// exceeds kDealRounds keeps the staged order.
// Threads per spread / gather block (one block per bin). Waves past a bin's
// last particle exit their particle loop at once, so a fixed block costs
// little for small bins. The gather's registers (about 120 per thread) allow
// 16 waves per compute unit: in blocks of 256 threads that is 4 bins at once
// (the LDS holds 4 FP32 P = 6 tiles), against 2 with blocks of 512 (measured:
// the ensemble's largest gather launch 48 against 53 us). A launch of fewer
// than 4 bins per compute unit keeps 512 threads per bin (the 300,000-atom
// box's 512 bins: 36 against 46 us with 256).
constexpr int kSpreadThreads = 512;
constexpr int kGatherThreadsMany = 256;
constexpr int kGatherThreadsFew = 512;
constexpr int kComputeUnits = 256;  // MI355X

constexpr int kDealRounds = 1024;
constexpr int kDealRegs = 8;  // staged particles per thread held in registers

// Bank class of a particle at bin coordinates v: the tile index of its
// window's first entry, l0 - (bin origin + lo) per axis, mod 32.
template <typename R>
__device__ __forceinline__ int deal_class(R vx, R vy, R vz, R hp, int lo, int E) {
    const int bx = (int)floor(vx - hp) + 1 - lo;
    const int by = (int)floor(vy - hp) + 1 - lo;
    const int bz = (int)floor(vz - hp) + 1 - lo;
    return ((bx * E + by) * E + bz) & 31;
}

template <typename R>
__global__ void __launch_bounds__(256) k_deal(const SysDesc* __restrict__ sys, const int2* __restrict__ items) {
    using V = typename Vec4<R>::type;
    constexpr int BD = 256;
    __shared__ int start[kDealRounds];        // first slot of round j
    __shared__ unsigned mask[kDealRounds];    // classes present in round j
    __shared__ int cnt[32];
    __shared__ int maxc_s;
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (S.small) return;  // uniform over the block
    const int t = wi.y, E = S.E;
    const int beg = S.bin_start[t], count = S.bin_start[t + 1] - beg;
    if (count == 0) return;  // uniform over the block
    const V* src = stage_vals<R>(S) + beg;
    const int* srcp = stage_perm<R>(S) + beg;
    V* dst = reinterpret_cast<V*>(S.sorted) + beg;
    int* dstp = S.perm + beg;
    int* key = S.rank + beg;  // free after the scatter; keys beyond the registers
    const int lo = -((S.P - 1) / 2);
    const R hp = R(0.5) * R(S.P);
    if (threadIdx.x < 32) cnt[threadIdx.x] = 0;
    __syncthreads();
    // key = class << 16 | rank of the particle within its class
    V vr[kDealRegs];
    int pr[kDealRegs], kr[kDealRegs];
#pragma unroll
    for (int k = 0; k < kDealRegs; ++k) {
        const int i = threadIdx.x + k * BD;
        if (i < count) {
            vr[k] = src[i];
            pr[k] = srcp[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kDealRegs; ++k) {
        const int i = threadIdx.x + k * BD;
        if (i < count) {
            const int c = deal_class<R>(vr[k].x, vr[k].y, vr[k].z, hp, lo, E);
            kr[k] = (c << 16) | atomicAdd(&cnt[c], 1);
        }
    }
    for (int i = threadIdx.x + kDealRegs * BD; i < count; i += BD) {
        const V s = src[i];
        const int c = deal_class<R>(s.x, s.y, s.z, hp, lo, E);
        key[i] = (c << 16) | atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    // one wave: largest class, then per round the mask of classes present and
    // the first slot (running sum of the round sizes)
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int cl = lane < 32 ? cnt[lane] : 0;
        int m = cl;
        for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
        if (lane == 0) maxc_s = m;
        if (m <= kDealRounds) {
            int run = 0;
            for (int j = 0; j < m; ++j) {
                const unsigned b = (unsigned)__ballot(cl > j);
                if (lane == 0) {
                    mask[j] = b;
                    start[j] = run;
                }
                run += __popc(b);
            }
        }
    }
    __syncthreads();
    const int maxc = maxc_s;
    const bool deal = maxc <= kDealRounds;  // else keep the staged order
#pragma unroll
    for (int k = 0; k < kDealRegs; ++k) {
        const int i = threadIdx.x + k * BD;
        if (i < count) {
            int pos = i;
            if (deal) {
                const int c = kr[k] >> 16, r = kr[k] & 0xFFFF;
                pos = start[r] + __popc(mask[r] & ((1u << c) - 1u));
            }
            dst[pos] = vr[k];
            dstp[pos] = pr[k];
        }
    }
    for (int i = threadIdx.x + kDealRegs * BD; i < count; i += BD) {
        int pos = i;
        if (deal) {
            const int kk = key[i], c = kk >> 16, r = kk & 0xFFFF;
            pos = start[r] + __popc(mask[r] & ((1u << c) - 1u));
        }
        dst[pos] = src[i];
        dstp[pos] = srcp[i];
    }
}

// ---------------------------------------------------------------------------
// Window polynomial coefficients of one system staged in LDS, transposed so
// the P coefficients of one power of y are contiguous: ct[m * P + j]. The
// global table holds coef[j * (deg + 1) + m] (window piece j, power m). With
// ctd != nullptr the derivative coefficients (m + 1) c[m + 1][j] go to
// ctd[m * P + j] for m < deg, and row deg of ctd is zero.
template <typename R, int P>
__device__ __forceinline__ void stage_coef(R* __restrict__ ct, R* __restrict__ ctd, const R* __restrict__ coef,
                                           int deg) {
    const int d1 = deg + 1;
    for (int i = threadIdx.x; i < P * d1; i += blockDim.x) {
        const int j = i / d1, m = i - j * d1;
        ct[m * P + j] = coef[i];
        if (ctd) ctd[(m > 0 ? m - 1 : deg) * P + j] = m > 0 ? R(m) * coef[i] : R(0);  // row deg is zero
    }
}

// Window weights of the three axes of one particle (eq. spread): the P
// polynomial pieces at y = frac(u - P/2) - 1/2 (|y| <= 1/2), summed as
// sum_m c[m][j] y^m with a running power of y, so every term is one
// accumulate and each power's coefficients are read from LDS once for all
// three axes (the sums start at c[0] + c[1] y, degree >= 4). Weights are
// clamped at zero (the window is positive on its support; the clamp only
// removes rounding noise at the support's edge, and the fixed-point spread
// relies on it). l0[a] is the first grid index of axis a's support.
template <typename R, int P, bool CLAMP = true>
__device__ __forceinline__ void windows3(R ux, R uy, R uz, const R* __restrict__ ct, int deg, R (&w)[3][P],
                                         int (&l0)[3]) {
    const R hp = R(0.5) * R(P);
    const R u[3] = {ux, uy, uz};
    R y[3], yp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R f = floor(u[a] - hp);
        y[a] = (u[a] - hp) - f - R(0.5);
        l0[a] = (int)f + 1;
        yp[a] = y[a] * y[a];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const R c0 = ct[j], c1 = ct[P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a][j] = c1 * y[a] + c0;
    }
#pragma unroll 1
    for (int m = 2; m <= deg; ++m) {
        R c[P];
#pragma unroll
        for (int j = 0; j < P; ++j) c[j] = ct[m * P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int j = 0; j < P; ++j) w[a][j] += c[j] * yp[a];
            yp[a] *= y[a];
        }
    }
    if constexpr (CLAMP) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int j = 0; j < P; ++j) w[a][j] = fmax(w[a][j], R(0));
    }
}

// As windows3 without the clamp, with the derivatives d w / d u from the
// staged derivative coefficients ctd (sum_m (m + 1) c[m + 1][j] y^m).
template <typename R, int P>
__device__ __forceinline__ void windows3_d(R ux, R uy, R uz, const R* __restrict__ ct, const R* __restrict__ ctd,
                                           int deg, R (&w)[3][P], R (&dw)[3][P], int (&l0)[3]) {
    const R hp = R(0.5) * R(P);
    const R u[3] = {ux, uy, uz};
    R y[3], yp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R f = floor(u[a] - hp);
        y[a] = (u[a] - hp) - f - R(0.5);
        l0[a] = (int)f + 1;
        yp[a] = y[a] * y[a];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const R c0 = ct[j], c1 = ct[P + j], d0 = ctd[j], d1 = ctd[P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w[a][j] = c1 * y[a] + c0;
            dw[a][j] = d1 * y[a] + d0;
        }
    }
#pragma unroll 1
    for (int m = 2; m <= deg; ++m) {
        R c[P], d[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            c[j] = ct[m * P + j];
            d[j] = ctd[m * P + j];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int j = 0; j < P; ++j) {
                w[a][j] += c[j] * yp[a];
                dw[a][j] += d[j] * yp[a];
            }
            yp[a] *= y[a];
        }
    }
}

__device__ __forceinline__ int wrapi(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

// Periodic index for -n <= g < 2n (tile origins and offsets: a tile starts at
// most 6 points before 0 and spans at most T + 12 <= n + 12 points, n >= 8).
__device__ __forceinline__ int wrap_near(int g, int n) {
    g += g < 0 ? n : 0;
    return g >= n ? g - n : g;
}

// The bin of this block in a spread / gather launch over a group's XCD-ordered
// list of kXcds runs of `per` entries. Blocks go to the chip's XCDs round
// robin (block b to XCD b mod kXcds), so XCD x takes run x, which holds whole
// systems: the neighbouring bins of a system share that XCD's L2, which then
// serves the halos their tiles have in common. (-1, -1) marks padding.
__device__ __forceinline__ int2 xcd_item(const int2* __restrict__ items, int per) {
    return items[(int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds)];
}

// Spread (eq. spread): one block per bin of T^3 grid cells. The block
// accumulates its particles' P^3 windows into an LDS tile of E^3 points
// (E = T + P - 1 + (P odd)) and stores the whole tile, halo included, to the
// bin's slot of the tile buffer with plain stores. The halos of neighbouring
// bins are summed when the forward FFT loads its planes (fold_point), so no
// global atomics are needed.
//
// LDS accumulator. FP32 systems accumulate in fixed point (LDS float atomics
// are ~40x slower than integer ones on gfx950, and integer sums are
// order-independent, so the spread is deterministic):
//   * windows up to P = 6 (tol >= 1e-4): 32-bit (ds_add_u32, about 1.45x the
//     rate of 64-bit adds, and half the LDS, so twice the blocks per CU).
//     A bin of `count` particles takes the scale 2^F / 2^ceil(log2 count):
//     no point can then collect more than 2^30 in magnitude, and each term,
//     rounded to the nearest unit, is kept to about 2^-20 of the largest
//     single term (a few 1e-7 of the grid values, below FP32 rounding of the
//     later stages times the tolerance);
//   * wider windows (tol < 1e-4): 64-bit (ds_add_u64) with the system's scale
//     2^F, every term below 2^30 and truncated toward zero (a bias below one
//     unit, ~1e-9 of the largest term).
// The tile goes back to float when stored. FP64 systems accumulate with
// ds_add_f64.
template <typename R, int P> struct SpreadAcc {
    using type = R;
};
template <int P> struct SpreadAcc<float, P> {
    using type = typename std::conditional<(P <= 6), unsigned, unsigned long long>::type;
};

template <typename R, int P>
__global__ void __launch_bounds__(kSpreadThreads) k_spread(const SysDesc* __restrict__ sys, const int2* __restrict__ items,
                                                           int per) {
    using A = typename SpreadAcc<R, P>::type;
    constexpr bool kFixed = !std::is_floating_point<A>::value;
    constexpr bool kNarrow = sizeof(A) == 4 && kFixed;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A* lds = reinterpret_cast<A*>(smem_raw);
    const int2 wi = xcd_item(items, per);
    if (wi.x < 0) return;
    const SysDesc& S = sys[wi.x];
    const int t = wi.y;
    const int lo = -((P - 1) / 2);
    const int E = S.E, E3 = E * E * E;
    const int beg = S.bin_start[t], end = S.bin_start[t + 1];
    const auto out = gptr(reinterpret_cast<R*>(S.tiles) + (long long)t * E3);
    if (beg == end) {  // uniform over the block
        for (int i = threadIdx.x; i < E3; i += blockDim.x) out[i] = R(0);
        return;
    }
    // each thread's first particle loads while the tile is cleared, the next
    // ones while the current one is spread
    typename Vec4<R>::type vn{};
    if (beg + (int)threadIdx.x < end) vn = gload4<R>(S.sorted, beg + threadIdx.x);
    // 32-bit: the system's scale over the bin's count rounded up to a power of two
    const R scale = !kFixed ? R(1)
                  : kNarrow ? R(ldexp(S.out[4], -(32 - __clz((unsigned)(end - beg - 1)))))
                            : R(S.out[4]);
    R* ct = reinterpret_cast<R*>(smem_raw + (size_t)E3 * sizeof(A));
    stage_coef<R, P>(ct, nullptr, reinterpret_cast<const R*>(S.poly), S.degree);
    {
        // clear the tile 16 bytes at a time, then the tail
        const int n16 = (int)(((size_t)E3 * sizeof(A)) / 16);
        for (int i = threadIdx.x; i < n16; i += blockDim.x) reinterpret_cast<uint4*>(lds)[i] = make_uint4(0, 0, 0, 0);
        for (int i = n16 * (16 / (int)sizeof(A)) + threadIdx.x; i < E3; i += blockDim.x) lds[i] = A(0);
    }
    __syncthreads();
    const int deg = S.degree;
    for (int k = beg + threadIdx.x; k < end; k += blockDim.x) {
        const typename Vec4<R>::type v = vn;
        if (k + (int)blockDim.x < end) vn = gload4<R>(S.sorted, k + blockDim.x);
        R w[3][P];
        int l0[3];
        windows3<R, P>(v.x, v.y, v.z, ct, deg, w, l0);
        const int bx = l0[0] - lo, by = l0[1] - lo, bz = l0[2] - lo;  // bin coordinates
        const R qs = v.w * scale;
        // fixed point: every term of a particle has the sign of its charge
        // (weights >= 0), so the high word of the 64-bit addend is that sign
        // and the low word is the term truncated toward zero, shifted by -1 for
        // negative charges so that it is never 0 there (a bias below one unit
        // 2^-F per term)
        const bool neg = v.w < R(0);
        const R shift = neg ? R(-1) : R(0);
        const unsigned long long hi = neg ? 0xFFFFFFFF00000000ull : 0ull;
#pragma unroll
        for (int a = 0; a < P; ++a) {
            const R qa = qs * w[0][a];
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const R qab = qa * w[1][b];
                A* row = lds + ((bx + a) * E + (by + b)) * E + bz;
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    if constexpr (kNarrow)
                        atomicAdd(row + c, (A)__float2int_rn(qab * w[2][c]));  // two's complement
                    else if constexpr (kFixed)
                        atomicAdd(row + c, (A)(hi | (unsigned)(int)(qab * w[2][c] + shift)));
                    else
                        atomicAdd(row + c, qab * w[2][c]);
                }
            }
        }
    }
    __syncthreads();
    if constexpr (kNarrow) {
        // |value| < 2^31 and the scale a power of two: one rounding, as in FP64
        const R inv = R(1) / scale;
        for (int i = threadIdx.x; i < E3; i += blockDim.x) out[i] = R((int)lds[i]) * inv;
    } else if constexpr (kFixed) {
        const R inv = R(1) / scale;
        for (int i = threadIdx.x; i < E3; i += blockDim.x) out[i] = R((double)(long long)lds[i] * (double)inv);
    } else {
        for (int i = threadIdx.x; i < E3; i += blockDim.x) out[i] = lds[i];
    }
}

// Diagnostics: fold the bin tiles into the padded real grid (b_l of eq. spread).
template <typename R>
__global__ void __launch_bounds__(256) k_fold(const SysDesc* __restrict__ sys, const int2* __restrict__ items) {
    __shared__ CoverTab tab[145];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int n = S.n;
    build_cover(tab, S, -((S.P - 1) / 2));
    __syncthreads();
    const CoverTab cx = tab[wi.y];
    const R* tiles = reinterpret_cast<const R*>(S.tiles);
    R* plane = reinterpret_cast<R*>(S.grid) + (long long)wi.y * n * (n + 2);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int y = idx / n, z = idx - y * n;
        plane[y * (n + 2) + z] = fold_point(tiles, S, cx, tab[y], tab[z]);
    }
}

// The E^3 window tile of a bin (origin ox, oy, oz, periodic) from a grid
// stored n x n x (n + 2) (E <= 28): element r E + c of the tile, row
// r = a E + b, is grid point (ox + a, oy + b, oz + c) mod n. The E^2 row
// offsets go to `rows` (LDS) first. Then the first floor(blockDim / E) E
// threads each own one column c = tid mod E, whose periodic z offset they
// compute once, and walk the rows r = tid / E, + floor(blockDim / E), ...,
// four loads in flight. Starts and ends with a block barrier.
template <typename R>
__device__ __forceinline__ void load_tile(R* __restrict__ lds, int* __restrict__ rows, const R* __restrict__ g, int n,
                                          int E, int ox, int oy, int oz) {
    const int rl = n + 2, E2 = E * E;
    for (int r = threadIdx.x; r < E2; r += blockDim.x) {
        const int a = r / E, b = r - a * E;
        rows[r] = (wrap_near(ox + a, n) * n + wrap_near(oy + b, n)) * rl;
    }
    __syncthreads();
    const int rstep = blockDim.x / E;
    const int r0 = threadIdx.x / E, c = threadIdx.x - r0 * E;
    if (r0 < rstep) {
        const unsigned zoff = (unsigned)wrap_near(oz + c, n);
        const auto gg = gptr(g);
        int r = r0;
        for (; r + 3 * rstep < E2; r += 4 * rstep) {
            R v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = gg[(unsigned)rows[r + u * rstep] + zoff];
#pragma unroll
            for (int u = 0; u < 4; ++u) lds[(r + u * rstep) * E + c] = v[u];
        }
        for (; r < E2; r += rstep) lds[r * E + c] = gg[(unsigned)rows[r] + zoff];
    }
    __syncthreads();
}

// Gather with ik forces (Methods, force paragraph): four passes over the
// bin's particles, each interpolating one grid with the window itself:
// the potential (phi_i = u~_i - q_i S(0)) and the three gradient grids
// (F_i = -q_i times the interpolated gradient). In a box the grids hold
// Cartesian derivatives; in a tilted cell they hold derivatives g_d along the
// fractional coordinates and F = -q H^-T g, accumulated over the passes (H^-1
// upper triangular: pass d adds to components d and beyond).
template <typename R, int P>
__device__ __forceinline__ void gather_ik(const SysDesc& S, R* __restrict__ lds, int* __restrict__ rows, const R* __restrict__ ct,
                          int ox, int oy, int oz, int beg, int end) {
    const int n = S.n, E = S.E, deg = S.degree;
    const long long G = (long long)n * n * (n + 2);
    const typename Vec4<R>::type* sorted = reinterpret_cast<const typename Vec4<R>::type*>(S.sorted);
    R* phi = reinterpret_cast<R*>(S.phi);
    R* F = reinterpret_cast<R*>(S.F);
    const R s0 = R(S.s0);
    const bool tilt = S.ixy != 0.0 || S.ixz != 0.0 || S.iyz != 0.0;  // uniform
    // column pass - 1 of H^-T: the factors of g_{pass-1} in F_x, F_y, F_z
    const R hinv[3][3] = {{R(S.inv_L), R(S.ixy), R(S.ixz)}, {R(0), R(S.inv_Ly), R(S.iyz)}, {R(0), R(0), R(S.inv_Lz)}};
    for (int pass = 0; pass < 4; ++pass) {
        if (pass == 0 && !phi) continue;
        if (pass > 0 && !F) break;
        const R* src = pass == 0 ? reinterpret_cast<const R*>(S.grid)
                                 : reinterpret_cast<const R*>(S.grad) + (pass - 1) * G;
        __syncthreads();
        load_tile<R>(lds, rows, src, n, E, ox, oy, oz);
        for (int k = beg + threadIdx.x; k < end; k += blockDim.x) {
            const typename Vec4<R>::type v = sorted[k];
            R w[3][P];
            int l0[3];
            windows3<R, P, false>(v.x, v.y, v.z, ct, deg, w, l0);
            const int lo = -((P - 1) / 2);
            const int bx = l0[0] - lo, by = l0[1] - lo, bz = l0[2] - lo;  // bin coordinates
            R u = 0;
#pragma unroll 1
            for (int a = 0; a < P; ++a) {
                R su = 0;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const R* row = lds + ((bx + a) * E + (by + b)) * E + bz;
                    R s = 0;
#pragma unroll
                    for (int c = 0; c < P; ++c) s += row[c] * w[2][c];
                    su += s * w[1][b];
                }
                u += su * w[0][a];
            }
            const int o = S.perm[k];
            R l = 0;  // local part (k_local), component `pass`
            if (S.local) l = reinterpret_cast<const R*>(S.loc)[4LL * k + pass];
            if (pass == 0) {
                phi[o] = u - v.w * s0 + l;
            } else if (!tilt) {
                F[3LL * o + (pass - 1)] = -v.w * u + l;
            } else {
                // the same thread owns particle k in every pass
                const int d = pass - 1;
                for (int j = d; j < 3; ++j) {
                    const R t = -v.w * (hinv[d][j] * u) + (j == d ? l : R(0));
                    F[3LL * o + j] = d == 0 ? t : F[3LL * o + j] + t;
                }
            }
        }
    }
}

// Gather (eq. interp) with analytic window derivatives (AD forces):
// phi_i = u~_i - q_i S(0), F_i = -q_i (n/L) grad_u u~_i, written in caller order.
// BT threads per block (see kGatherThreadsMany). FP32 windows of 7 and 8
// points are held to 128 registers (4 waves per SIMD, two 512-thread blocks
// per compute unit), which they exceed by a few otherwise; the others keep
// the compiler's choice (P = 6: 121, and a cap there costs speed).
template <typename R, int P, int BT>
__global__ void __launch_bounds__(BT, (sizeof(R) == 4 && P >= 7 && P <= 8) ? 4 : 1) k_gather(const SysDesc* __restrict__ sys, const int2* __restrict__ items,
                                               int per) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* lds = reinterpret_cast<R*>(smem_raw);
    const int2 wi = xcd_item(items, per);
    if (wi.x < 0) return;
    const SysDesc& S = sys[wi.x];
    const int t = wi.y, T = S.T, t1 = S.tiles1, n = S.n;
    int tx, ty, tz;
    bin_coords(t, S, tx, ty, tz);
    const int lo = -((P - 1) / 2);
    const int E = S.E, E3 = E * E * E;
    const int ox = tx * T + lo, oy = ty * T + lo, oz = tz * T + lo;
    const int beg = S.bin_start[t], end = S.bin_start[t + 1];
    if (beg == end) return;
    // LDS: the tile, the window coefficients and their derivatives, the
    // tile's row offsets
    R* ct = reinterpret_cast<R*>(smem_raw + (((size_t)E3 * sizeof(R) + 15) & ~size_t(15)));
    R* ctd = ct + 17 * P;
    int* rows = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(ct) + gather_coef_bytes(P, (int)sizeof(R)));
    stage_coef<R, P>(ct, ctd, reinterpret_cast<const R*>(S.poly), S.degree);
    if (S.ik) {  // uniform over the block
        gather_ik<R, P>(S, lds, rows, ct, ox, oy, oz, beg, end);
        return;
    }
    // each thread's first particle and its caller index load during the
    // tile's load, the next ones while the current particle is gathered
    using V = typename Vec4<R>::type;
    const int BD = blockDim.x;
    int k = beg + threadIdx.x;
    V vn{};
    int on = 0;
    if (k < end) {
        vn = gload4<R>(S.sorted, k);
        on = gptr(S.perm)[k];
    }
    load_tile<R>(lds, rows, reinterpret_cast<const R*>(S.grid), n, E, ox, oy, oz);
    const int deg = S.degree;
    const R scx = R(S.n) * R(S.inv_L), scy = R(S.n) * R(S.inv_Ly), scz = R(S.n) * R(S.inv_Lz);
    // grad_r = n H^-T grad_u: the off-diagonal terms of a triclinic cell (0 otherwise)
    const R sxy = R(S.n) * R(S.ixy), sxz = R(S.n) * R(S.ixz), syz = R(S.n) * R(S.iyz);
    const R s0 = R(S.s0);
    const auto phi = gptr(reinterpret_cast<R*>(S.phi));
    const auto F = gptr(reinterpret_cast<R*>(S.F));
    for (; k < end; k += BD) {
        const V v = vn;
        const int o = on;
        if (k + BD < end) {
            vn = gload4<R>(S.sorted, k + BD);
            on = gptr(S.perm)[k + BD];
        }
        R w[3][P], dw[3][P];
        int l0[3];
        windows3_d<R, P>(v.x, v.y, v.z, ct, ctd, deg, w, dw, l0);
        const int bx = l0[0] - lo, by = l0[1] - lo, bz = l0[2] - lo;  // bin coordinates
        const R(&wx)[P] = w[0];
        const R(&wy)[P] = w[1];
        const R(&wz)[P] = w[2];
        const R(&dx)[P] = dw[0];
        const R(&dy)[P] = dw[1];
        const R(&dz)[P] = dw[2];
        R u = 0, gxs = 0, gys = 0, gzs = 0;
        // outer loop kept rolled: a is uniform across the wavefront, and
        // unrolling all P^3 loads would exhaust the register file
#pragma unroll 1
        for (int a = 0; a < P; ++a) {
            R su = 0, sdy = 0, sdz = 0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const R* row = lds + ((bx + a) * E + (by + b)) * E + bz;
                R s = 0, sd = 0;
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    const R gv = row[c];
                    s += gv * wz[c];
                    sd += gv * dz[c];
                }
                su += s * wy[b];
                sdy += s * dy[b];
                sdz += sd * wy[b];
            }
            u += su * wx[a];
            gxs += su * dx[a];
            gys += sdy * wx[a];
            gzs += sdz * wx[a];
        }
        V l = {0, 0, 0, 0};  // local part (k_local)
        if (S.local) l = gload4<R>(S.loc, k);
        if (phi) phi[o] = u - v.w * s0 + l.x;
        if (F) {
            F[3LL * o + 0] = -v.w * scx * gxs + l.y;
            F[3LL * o + 1] = -v.w * scy * gys - v.w * (sxy * gxs) + l.z;
            F[3LL * o + 2] = -v.w * scz * gzs - v.w * (sxz * gxs + syz * gys) + l.w;
        }
    }
}

// Energy per system (finalize_system) for the systems whose FFT ran as one
// fused kernel; the others are finalized by their last FFT pass (k_inv_yz).
// One wave per system.
__global__ void __launch_bounds__(64) k_finalize(const SysDesc* __restrict__ sys, const double* __restrict__ epart,
                                                 const double* __restrict__ bpart, const double* __restrict__ lpart,
                                                 double* __restrict__ E_dev) {
    const SysDesc& S = sys[blockIdx.x];
    if (S.fin_fft) return;  // uniform over the block
    finalize_system(S, epart, bpart, lpart, E_dev, blockIdx.x);
}

// Serving: move the resident positions of every system with step > 0 by the
// drift of that step. Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA
// 2014): the uniform variate of (step k, particle i, component c) is
// mix(seed + (k * 2^40 + 3 i + c + 1) * 0x9E3779B97F4A7C15) / 2^64, so the
// host reproduces every position exactly.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kChunkThreads) k_drift(const SysDesc* __restrict__ sys,
                                                         const int2* __restrict__ items) {
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (S.step <= 0) return;
    float* pos = reinterpret_cast<float*>(const_cast<void*>(S.pos));
    const float L = (float)(1.0 / S.inv_L);
    for (int k = 0; k < kParticleChunk / kChunkThreads; ++k) {
        const int il = wi.y + threadIdx.x + k * kChunkThreads;
        if (il >= S.N) return;
        for (int c = 0; c < 3; ++c) {
            const unsigned long long ctr = ((unsigned long long)S.step << 40) + 3ULL * il + c + 1ULL;
            const unsigned long long z = splitmix64(S.seed + ctr * 0x9E3779B97F4A7C15ULL);
            const double u = (double)(z >> 11) * 0x1.0p-53;
            const float d = (float)((double)S.drift * (2.0 * u - 1.0));
            float x = pos[3 * il + c] + d;
            if (x >= L) x -= L;
            if (x < 0.0f) x += L;
            pos[3 * il + c] = x;
        }
    }
}

// ---------------------------------------------------------------------------
// Binning of a small system by one block, in place of k_hist, the scans, the
// scatter and the deal: LDS counters per (bin, bank class), the bins' first
// slots, the deal's rounds per bin, and one write of every particle to its
// dealt slot. The order is the one k_deal produces (round j of a bin holds the
// j-th particle of every class present, in class order), up to the order of
// particles within a (bin, class), which the LDS counters leave open and which
// no result depends on. If the rounds exceed kSmallRounds the bins are written
// class by class instead. The charge statistics go to the system's first
// chunk slot (the others are zeroed) and the fixed-point scale to out[4].

constexpr int kSmallBatch = 8;

template <typename R>
__device__ __forceinline__ BinCoords<R> small_bin_class(const SysDesc& S, R x, R y, R z, R hp, int lo, int& c) {
    const BinCoords<R> bc = bin_coords_of<R>(S, x, y, z);
    c = deal_class<R>(bc.vx, bc.vy, bc.vz, hp, lo, S.E);
    return bc;
}

template <typename R>
__global__ void __launch_bounds__(1024) k_bin_small(const SysDesc* __restrict__ sys, const int2* __restrict__ items,
                                                    double* __restrict__ bpart) {
    using V = typename Vec4<R>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[64];
    __shared__ int deal_s;
    const SysDesc& S = sys[items[blockIdx.x].x];
    const int t1 = S.tiles1, nb = t1 * t1 * t1, N = S.N;
    int* cnt = reinterpret_cast<int*>(smem_raw);  // nb x 32
    int* binoff = cnt + nb * 32;                  // nb + 1
    int* rbase = binoff + nb + 1;                 // nb + 1: first round of each bin
    int* rstart = rbase + nb + 1;                 // kSmallRounds
    unsigned* rmask = reinterpret_cast<unsigned*>(rstart + kSmallRounds);
    const R* pos = reinterpret_cast<const R*>(S.pos);
    const R* q = reinterpret_cast<const R*>(S.q);
    const R hp = R(0.5) * R(S.P);
    const int lo = -((S.P - 1) / 2);
    for (int i = threadIdx.x; i < nb * 32; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    double sq = 0.0, sa = 0.0, s2 = 0.0, qm = 0.0;
    constexpr int KK = sizeof(R) == 4 ? kSmallKeep : 1;
    const bool keep = sizeof(R) == 4 && N <= KK * 1024;  // uniform over the block
    R kx[KK], ky[KK], kz[KK], kq[KK];
    int kk[KK];  // rank within (bin, class) << 14 | bin x 32 + class (bins <= 512)
    if (keep) {
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            const int i = k * 1024 + threadIdx.x;
            if (i < N) {
                kx[k] = pos[3 * i + 0];
                ky[k] = pos[3 * i + 1];
                kz[k] = pos[3 * i + 2];
                kq[k] = q[i];
            }
        }
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            const int i = k * 1024 + threadIdx.x;
            if (i < N) {
                int c;
                const BinCoords<R> bc = small_bin_class<R>(S, kx[k], ky[k], kz[k], hp, lo, c);
                kx[k] = bc.vx;
                ky[k] = bc.vy;
                kz[k] = bc.vz;
                const int bcl = bc.bin * 32 + c;
                kk[k] = (atomicAdd(&cnt[bcl], 1) << 14) | bcl;
                const double qq = (double)kq[k];
                sq += qq;
                sa += fabs(qq);
                s2 += qq * qq;
                qm = fmax(qm, fabs(qq));
            }
        }
    }
    // batches of kSmallBatch particles per thread: every load of a batch is
    // issued before any is used
    for (int base = 0; !keep && base < N; base += kSmallBatch * 1024) {
        R px[kSmallBatch], py[kSmallBatch], pz[kSmallBatch], pq[kSmallBatch];
#pragma unroll
        for (int k = 0; k < kSmallBatch; ++k) {
            const int i = base + k * 1024 + threadIdx.x;
            if (i < N) {
                px[k] = pos[3 * i + 0];
                py[k] = pos[3 * i + 1];
                pz[k] = pos[3 * i + 2];
                pq[k] = q[i];
            }
        }
#pragma unroll
        for (int k = 0; k < kSmallBatch; ++k) {
            const int i = base + k * 1024 + threadIdx.x;
            if (i < N) {
                int c;
                const int b = small_bin_class<R>(S, px[k], py[k], pz[k], hp, lo, c).bin;
                S.rank[i] = atomicAdd(&cnt[b * 32 + c], 1);
                const double qq = (double)pq[k];
                sq += qq;
                sa += fabs(qq);
                s2 += qq * qq;
                qm = fmax(qm, fabs(qq));
            }
        }
    }
    block_sum3_max(sq, sa, s2, qm, red);  // also orders the counters
    if (threadIdx.x == 0) {
        double* bp = bpart + 4 * S.pitem_off;
        bp[0] = sq;
        bp[1] = sa;
        bp[2] = s2;
        bp[3] = qm;
        const double bound = qm * S.wmax3;
        const int F = bound > 0.0 ? 30 - (int)ceil(log2(bound)) : 30;
        S.out[4] = ldexp(1.0, max(-100, min(100, F)));
    }
    for (int k = 1 + threadIdx.x; k < S.npitem; k += blockDim.x)
        for (int j = 0; j < 4; ++j) bpart[4 * (S.pitem_off + k) + j] = 0.0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // per bin (one wave per bin): particle total and largest class
    for (int b = wid; b < nb; b += nw) {
        const int cl = lane < 32 ? cnt[b * 32 + lane] : 0;
        int t = cl, m = cl;
        for (int off = 32; off > 0; off >>= 1) {
            t += __shfl_xor(t, off, 64);
            m = max(m, __shfl_xor(m, off, 64));
        }
        if (lane == 0) {
            binoff[b] = t;
            rbase[b] = m;
        }
    }
    __syncthreads();
    // exclusive scans over bins of the totals and of the round counts (wave 0)
    if (wid == 0) {
        int ct = 0, cr = 0;
        for (int base = 0; base < nb; base += 64) {
            const int l = base + lane;
            const int vt = l < nb ? binoff[l] : 0, vr = l < nb ? rbase[l] : 0;
            int xt = vt, xr = vr;
            for (int off = 1; off < 64; off <<= 1) {
                const int yt = __shfl_up(xt, off, 64), yr = __shfl_up(xr, off, 64);
                if (lane >= off) {
                    xt += yt;
                    xr += yr;
                }
            }
            if (l < nb) {
                binoff[l] = ct + xt - vt;
                rbase[l] = cr + xr - vr;
            }
            ct += __shfl(xt, 63, 64);
            cr += __shfl(xr, 63, 64);
        }
        if (lane == 0) {
            binoff[nb] = ct;
            rbase[nb] = cr;
            deal_s = cr <= kSmallRounds;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b <= nb; b += blockDim.x) S.bin_start[b] = binoff[b];
    const bool deal = deal_s;
    for (int b = wid; b < nb; b += nw) {
        const int cl = lane < 32 ? cnt[b * 32 + lane] : 0;
        if (deal) {
            const int r0 = rbase[b], nr = rbase[b + 1] - r0;
            int run = 0;
            for (int j = 0; j < nr; ++j) {
                const unsigned m = (unsigned)__ballot(cl > j);
                if (lane == 0) {
                    rstart[r0 + j] = run;
                    rmask[r0 + j] = m;
                }
                run += __popc(m);
            }
        } else {
            // class-major order: exclusive scan of the class counts of the bin
            int x = cl;
            for (int off = 1; off < 32; off <<= 1) {
                const int y = __shfl_up(x, off, 64);
                if (lane >= off) x += y;
            }
            if (lane < 32) cnt[b * 32 + lane] = x - cl;
        }
    }
    __syncthreads();
    V* sorted = reinterpret_cast<V*>(S.sorted);
    if (keep) {
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            const int i = k * 1024 + threadIdx.x;
            if (i < N) {
                const int bcl = kk[k] & 16383, r = kk[k] >> 14, b = bcl >> 5, c = bcl & 31;
                int p = binoff[b];
                if (deal) {
                    const int j = rbase[b] + r;
                    p += rstart[j] + __popc(rmask[j] & ((1u << c) - 1u));
                } else {
                    p += cnt[bcl] + r;
                }
                V v;
                v.x = kx[k];
                v.y = ky[k];
                v.z = kz[k];
                v.w = kq[k];
                sorted[p] = v;
                S.perm[p] = i;
            }
        }
        return;
    }
    for (int base = 0; base < N; base += kSmallBatch * 1024) {
        R px[kSmallBatch], py[kSmallBatch], pz[kSmallBatch], pq[kSmallBatch];
        int pr[kSmallBatch];
#pragma unroll
        for (int k = 0; k < kSmallBatch; ++k) {
            const int i = base + k * 1024 + threadIdx.x;
            if (i < N) {
                px[k] = pos[3 * i + 0];
                py[k] = pos[3 * i + 1];
                pz[k] = pos[3 * i + 2];
                pq[k] = q[i];
                pr[k] = S.rank[i];
            }
        }
#pragma unroll
        for (int k = 0; k < kSmallBatch; ++k) {
            const int i = base + k * 1024 + threadIdx.x;
            if (i < N) {
                int c;
                const BinCoords<R> bc = small_bin_class<R>(S, px[k], py[k], pz[k], hp, lo, c);
                const int b = bc.bin;
                int p = binoff[b];
                if (deal) {
                    const int j = rbase[b] + pr[k];
                    p += rstart[j] + __popc(rmask[j] & ((1u << c) - 1u));
                } else {
                    p += cnt[b * 32 + c] + pr[k];
                }
                V v;
                v.x = bc.vx;
                v.y = bc.vy;
                v.z = bc.vz;
                v.w = pq[k];
                sorted[p] = v;
                S.perm[p] = i;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <typename K>
static hipError_t allow_lds(K kernel, int bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <typename R>
static hipError_t bin_small_t(const Launch& L) {
    if (L.n_small == 0) return hipSuccess;
    hipError_t e = allow_lds(k_bin_small<R>, L.small_lds);
    if (e != hipSuccess) return e;
    k_bin_small<R><<<L.n_small, 1024, L.small_lds, L.stream>>>(L.sys, L.bsys, L.bpart);
    return hipGetLastError();
}

hipError_t launch_bin_small(const Launch& L) {
    return L.prec == 64 ? bin_small_t<double>(L) : bin_small_t<float>(L);
}

template <typename R>
static hipError_t prepare_t(const Launch& L, int phase, bool with_small) {
    hipError_t e;
    switch (phase) {
        case 0:
            if (with_small && (e = bin_small_t<R>(L)) != hipSuccess) return e;
            if (L.n_large == 0) break;
            if ((e = allow_lds(k_hist<R>, L.hist_lds)) != hipSuccess) return e;
            k_hist<R><<<L.n_pitems, kChunkThreads, L.hist_lds, L.stream>>>(L.sys, L.pitems, L.bpart);
            break;
        case 1:
            if (L.n_large == 0) break;
            if (L.n_titems > 0 && !L.scan_rows_fused) {
                k_scan_rows<<<(L.n_titems + 3) / 4, 256, 0, L.stream>>>(L.sys, L.titems, L.n_titems);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
            k_scan<<<L.nsys, 1024, 0, L.stream>>>(L.sys, L.bpart, L.scan_rows_fused);
            break;
        case 2: {
            if (L.n_large == 0) break;
            k_scatter<R><<<L.n_pitems, kChunkThreads, 0, L.stream>>>(L.sys, L.pitems);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if (L.n_titems > 0) k_deal<R><<<L.n_titems, 256, 0, L.stream>>>(L.sys, L.titems);
            break;
        }
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prepare(const Launch& L, int phase, bool with_small) {
    return L.prec == 64 ? prepare_t<double>(L, phase, with_small) : prepare_t<float>(L, phase, with_small);
}

template <typename R, int P>
static hipError_t spread_p(const Launch& L, const Group& G) {
    hipError_t e = allow_lds(k_spread<R, P>, G.lds_spread);
    if (e != hipSuccess) return e;
    k_spread<R, P><<<G.count, kSpreadThreads, G.lds_spread, L.stream>>>(L.sys, L.xitems + G.off, G.count / kXcds);
    return hipGetLastError();
}

template <typename R, int P, int BT>
static hipError_t gather_bt(const Launch& L, const Group& G) {
    hipError_t e = allow_lds(k_gather<R, P, BT>, G.lds_gather);
    if (e != hipSuccess) return e;
    k_gather<R, P, BT><<<G.count, BT, G.lds_gather, L.stream>>>(L.sys, L.xitems + G.off, G.count / kXcds);
    return hipGetLastError();
}

template <typename R, int P>
static hipError_t gather_p(const Launch& L, const Group& G) {
    return G.count >= 4 * kComputeUnits ? gather_bt<R, P, kGatherThreadsMany>(L, G)
                                        : gather_bt<R, P, kGatherThreadsFew>(L, G);
}

#define ESP_P_SWITCH(FN, R, ...)                        \
    switch (G.P) {                                      \
        case 4: return FN<R, 4>(__VA_ARGS__);           \
        case 5: return FN<R, 5>(__VA_ARGS__);           \
        case 6: return FN<R, 6>(__VA_ARGS__);           \
        case 7: return FN<R, 7>(__VA_ARGS__);           \
        case 8: return FN<R, 8>(__VA_ARGS__);           \
        case 9: return FN<R, 9>(__VA_ARGS__);           \
        case 10: return FN<R, 10>(__VA_ARGS__);         \
        case 11: return FN<R, 11>(__VA_ARGS__);         \
        case 12: return FN<R, 12>(__VA_ARGS__);         \
        default: return hipErrorInvalidValue;           \
    }

hipError_t launch_spread(const Launch& L, const Group& G) {
    if (L.prec == 64) { ESP_P_SWITCH(spread_p, double, L, G) }
    ESP_P_SWITCH(spread_p, float, L, G)
}

hipError_t launch_gather(const Launch& L, const Group& G) {
    if (L.prec == 64) { ESP_P_SWITCH(gather_p, double, L, G) }
    ESP_P_SWITCH(gather_p, float, L, G)
}

hipError_t launch_fold(const Launch& L) {
    if (L.prec == 64)
        k_fold<double><<<L.n_planes, 256, 0, L.stream>>>(L.sys, L.planes);
    else
        k_fold<float><<<L.n_planes, 256, 0, L.stream>>>(L.sys, L.planes);
    return hipGetLastError();
}

hipError_t launch_drift(const Launch& L) {
    k_drift<<<L.n_pitems, kChunkThreads, 0, L.stream>>>(L.sys, L.pitems);
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch& L, double* E_dev) {
    if (!L.any_fin_kernel) return hipSuccess;  // every system was finalized by k_inv_yz
    k_finalize<<<L.nsys, 64, 0, L.stream>>>(L.sys, L.epart, L.bpart, L.lpart, E_dev);
    return hipGetLastError();
}

}  // namespace esp
