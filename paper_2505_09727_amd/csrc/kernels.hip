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

// Grid coordinate u in [0, n) of one position component.
template <typename R>
__device__ __forceinline__ R grid_coord(R x, R inv_L, int n) {
    R t = x * inv_L;
    t = t - floor(t);
    R u = t * R(n);
    if (u >= R(n)) u -= R(n);
    if (u < R(0)) u = R(0);
    return u;
}

// Bin of a particle: cells floor(u) grouped into T^3 blocks (T divides n).
template <typename R>
__device__ __forceinline__ int bin_of(R ux, R uy, R uz, const SysDesc& S) {
    const int nm1 = S.n - 1;
    const int cx = min((int)ux, nm1), cy = min((int)uy, nm1), cz = min((int)uz, nm1);
    return (cx / S.T * S.tiles1 + cy / S.T) * S.tiles1 + cz / S.T;
}

// ---------------------------------------------------------------------------
// Binning without global atomics.
//
// k_hist: one block per chunk of 256 particles of one system. Grid
// coordinates, bin id, and the rank of the particle among the chunk's
// particles of the same bin (LDS atomics); the chunk's bin counts go to column
// `item` of the system's bin-major count matrix (plain stores). Also the chunk
// sums of q, |q|, q^2 and max |q| (neutrality check, self energy, fixed-point
// range of the spread).
template <typename R>
__global__ void __launch_bounds__(256) k_hist(const SysDesc* __restrict__ sys, const int2* __restrict__ items,
                                              double* __restrict__ bpart) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int* cnt = reinterpret_cast<int*>(smem_raw);
    __shared__ double red[16];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int n = S.n, t1 = S.tiles1, nb = t1 * t1 * t1;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    const int il = wi.y + threadIdx.x;
    double sq = 0.0, sa = 0.0, s2 = 0.0;
    if (il < S.N) {
        const R* pos = reinterpret_cast<const R*>(S.pos);
        const R inv_L = R(S.inv_L);
        const R ux = grid_coord(pos[3 * il + 0], inv_L, n);
        const R uy = grid_coord(pos[3 * il + 1], inv_L, n);
        const R uz = grid_coord(pos[3 * il + 2], inv_L, n);
        S.rank[il] = atomicAdd(&cnt[bin_of(ux, uy, uz, S)], 1);
        const double qq = (double)reinterpret_cast<const R*>(S.q)[il];
        sq = qq;
        sa = fabs(qq);
        s2 = qq * qq;
    }
    __syncthreads();
    const int it = blockIdx.x - S.pitem_off;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) S.hist[b * S.npitem + it] = cnt[b];
    const double qm = block_max(sa, red);
    const double t0 = block_sum(sq, red);
    const double t1s = block_sum(sa, red);
    const double t2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        bpart[4 * blockIdx.x + 0] = t0;
        bpart[4 * blockIdx.x + 1] = t1s;
        bpart[4 * blockIdx.x + 2] = t2;
        bpart[4 * blockIdx.x + 3] = qm;
    }
}

// Exclusive scan of a system's bin-major count matrix (one block per system):
// the entry (bin, item) becomes the first sorted slot of that chunk's
// particles in that bin; bin_start[bin] is the first slot of the bin. Also
// the fixed-point scale of the FP32 spread: 2^F with every single
// contribution |q w_x w_y w_z| 2^F <= 2^30, so it is exact through int32.
__global__ void __launch_bounds__(1024) k_scan(const SysDesc* __restrict__ sys, const double* __restrict__ bpart) {
    __shared__ int warp_tot[16];
    __shared__ int carry_s;
    __shared__ double red[16];
    const SysDesc& S = sys[blockIdx.x];
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
    const int total = nb * S.npitem;
    int* hist = S.hist;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < total; base += blockDim.x) {
        const int l = base + threadIdx.x;
        const int v = l < total ? hist[l] : 0;
        int x = v;
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) warp_tot[wid] = x;
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wid; ++w) before += warp_tot[w];
        const int carry = carry_s;
        if (l < total) {
            const int off = carry + before + x - v;
            hist[l] = off;
            if (l % S.npitem == 0) S.bin_start[l / S.npitem] = off;
        }
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry_s = carry + before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) S.bin_start[nb] = S.N;
}

// Scatter particles into bin order as (u_x, u_y, u_z, q) and record the
// permutation back to the caller's order.
template <typename R>
__global__ void __launch_bounds__(256) k_scatter(const SysDesc* __restrict__ sys, const int2* __restrict__ items) {
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int il = wi.y + threadIdx.x;
    if (il >= S.N) return;
    const R* pos = reinterpret_cast<const R*>(S.pos);
    const R inv_L = R(S.inv_L);
    const int n = S.n;
    const R ux = grid_coord(pos[3 * il + 0], inv_L, n);
    const R uy = grid_coord(pos[3 * il + 1], inv_L, n);
    const R uz = grid_coord(pos[3 * il + 2], inv_L, n);
    const int b = bin_of(ux, uy, uz, S);
    const int dst = S.hist[b * S.npitem + (blockIdx.x - S.pitem_off)] + S.rank[il];
    typename Vec4<R>::type v;
    v.x = ux;
    v.y = uy;
    v.z = uz;
    v.w = reinterpret_cast<const R*>(S.q)[il];
    reinterpret_cast<typename Vec4<R>::type*>(S.sorted)[dst] = v;
    S.perm[dst] = il;
}

// ---------------------------------------------------------------------------
// Window weights of one axis by Horner in y in [-1/2, 1/2): the P polynomial
// pieces of psi^{c1}(2 (u - l)/P) for l = l0 .. l0+P-1, l0 = floor(u - P/2) + 1.
// Window polynomial coefficients of one system staged in LDS, transposed so
// the P coefficients of one power of y are contiguous: ct[m * P + j]. The
// global table holds coef[j * (deg + 1) + m] (window piece j, power m).
template <typename R, int P>
__device__ __forceinline__ void stage_coef(R* __restrict__ ct, const R* __restrict__ coef, int deg) {
    const int d1 = deg + 1;
    for (int i = threadIdx.x; i < P * d1; i += blockDim.x) {
        const int j = i / d1, m = i - j * d1;
        ct[m * P + j] = coef[i];
    }
}

// Window weights of the three axes of one particle (eq. spread): the P pieces
// of the polynomial window at y = frac(u - P/2) - 1/2, evaluated by Horner's
// rule for all three axes at once so each power's coefficients are read from
// LDS once. l0[a] is the first grid index of axis a's support.
template <typename R, int P>
__device__ __forceinline__ void windows3(R ux, R uy, R uz, const R* __restrict__ ct, int deg, R (&w)[3][P],
                                         int (&l0)[3]) {
    const R hp = R(0.5) * R(P);
    const R u[3] = {ux, uy, uz};
    R y[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R f = floor(u[a] - hp);
        y[a] = (u[a] - hp) - f - R(0.5);
        l0[a] = (int)f + 1;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const R c = ct[deg * P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a][j] = c;
    }
    for (int m = deg - 1; m >= 0; --m) {
        R c[P];
#pragma unroll
        for (int j = 0; j < P; ++j) c[j] = ct[m * P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int j = 0; j < P; ++j) w[a][j] = w[a][j] * y[a] + c[j];
    }
}

// As windows3, with the derivatives d w / d y (= d w / d u).
template <typename R, int P>
__device__ __forceinline__ void windows3_d(R ux, R uy, R uz, const R* __restrict__ ct, int deg, R (&w)[3][P],
                                           R (&dw)[3][P], int (&l0)[3]) {
    const R hp = R(0.5) * R(P);
    const R u[3] = {ux, uy, uz};
    R y[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R f = floor(u[a] - hp);
        y[a] = (u[a] - hp) - f - R(0.5);
        l0[a] = (int)f + 1;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const R c = ct[deg * P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            w[a][j] = c;
            dw[a][j] = R(0);
        }
    }
    for (int m = deg - 1; m >= 0; --m) {
        R c[P];
#pragma unroll
        for (int j = 0; j < P; ++j) c[j] = ct[m * P + j];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int j = 0; j < P; ++j) {
                dw[a][j] = dw[a][j] * y[a] + w[a][j];
                w[a][j] = w[a][j] * y[a] + c[j];
            }
    }
}

__device__ __forceinline__ int wrapi(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

// Spread (eq. spread): one block per bin of T^3 grid cells. The block
// accumulates its particles' P^3 windows into an LDS tile of E^3 points
// (E = T + P - 1 + (P odd)) and stores the whole tile, halo included, to the
// bin's slot of the tile buffer with plain stores. The halos of neighbouring
// bins are summed when the forward FFT loads its planes (fold_point), so no
// global atomics are needed.
//
// LDS accumulator: FP32 systems accumulate in 64-bit fixed point (ds_add_u64;
// LDS float atomics are ~20x slower than 64-bit integer ones on gfx950, and
// integer sums are order-independent, so the spread is deterministic). Each
// contribution q w_x w_y w_z is scaled by the system's 2^F and truncated to an
// int32 (an error of at most 2^-F per term); the tile is converted back to
// float when stored. FP64 systems
// accumulate with ds_add_f64.
template <typename R> struct SpreadAcc {
    using type = R;
};
template <> struct SpreadAcc<float> {
    using type = unsigned long long;
};

template <typename R, int P>
__global__ void __launch_bounds__(256) k_spread(const SysDesc* __restrict__ sys, const int2* __restrict__ items) {
    using A = typename SpreadAcc<R>::type;
    constexpr bool kFixed = !std::is_floating_point<A>::value;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A* lds = reinterpret_cast<A*>(smem_raw);
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int t = wi.y, T = S.T, t1 = S.tiles1;
    const int tz = t % t1, ty = (t / t1) % t1, tx = t / (t1 * t1);
    const int lo = -((P - 1) / 2);
    const int E = S.E, E3 = E * E * E;
    const int ox = tx * T + lo, oy = ty * T + lo, oz = tz * T + lo;
    const int beg = S.bin_start[t], end = S.bin_start[t + 1];
    R* out = reinterpret_cast<R*>(S.tiles) + (long long)t * E3;
    if (beg == end) {  // uniform over the block
        for (int i = threadIdx.x; i < E3; i += blockDim.x) out[i] = R(0);
        return;
    }
    R* ct = reinterpret_cast<R*>(smem_raw + (size_t)E3 * sizeof(A));
    stage_coef<R, P>(ct, reinterpret_cast<const R*>(S.poly), S.degree);
    for (int i = threadIdx.x; i < E3; i += blockDim.x) lds[i] = A(0);
    __syncthreads();
    const int deg = S.degree;
    const R scale = kFixed ? R(S.out[4]) : R(1);
    const typename Vec4<R>::type* sorted = reinterpret_cast<const typename Vec4<R>::type*>(S.sorted);
    for (int k = beg + threadIdx.x; k < end; k += blockDim.x) {
        const typename Vec4<R>::type v = sorted[k];
        R w[3][P];
        int l0[3];
        windows3<R, P>(v.x, v.y, v.z, ct, deg, w, l0);
        const int bx = l0[0] - ox, by = l0[1] - oy, bz = l0[2] - oz;
        const R qs = v.w * scale;
#pragma unroll
        for (int a = 0; a < P; ++a) {
            const R qa = qs * w[0][a];
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const R qab = qa * w[1][b];
                A* row = lds + ((bx + a) * E + (by + b)) * E + bz;
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    if constexpr (kFixed)
                        atomicAdd(row + c, (A)(long long)__float2int_rz(qab * w[2][c]));
                    else
                        atomicAdd(row + c, qab * w[2][c]);
                }
            }
        }
    }
    __syncthreads();
    if constexpr (kFixed) {
        const R inv = R(1) / scale;
        for (int i = threadIdx.x; i < E3; i += blockDim.x) out[i] = R((long long)lds[i]) * inv;
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

// Gather (eq. interp) with analytic window derivatives (AD forces):
// phi_i = u~_i - q_i S(0), F_i = -q_i (n/L) grad_u u~_i, written in caller order.
template <typename R, int P>
__global__ void __launch_bounds__(256) k_gather(const SysDesc* __restrict__ sys, const int2* __restrict__ items) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* lds = reinterpret_cast<R*>(smem_raw);
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int t = wi.y, T = S.T, t1 = S.tiles1, n = S.n;
    const int tz = t % t1, ty = (t / t1) % t1, tx = t / (t1 * t1);
    const int lo = -((P - 1) / 2);
    const int E = S.E, E3 = E * E * E;
    const int ox = tx * T + lo, oy = ty * T + lo, oz = tz * T + lo;
    const int beg = S.bin_start[t], end = S.bin_start[t + 1];
    if (beg == end) return;
    const R* g = reinterpret_cast<const R*>(S.grid);
    const int rl = n + 2;
    R* ct = reinterpret_cast<R*>(smem_raw + (((size_t)E3 * sizeof(R) + 15) & ~size_t(15)));
    stage_coef<R, P>(ct, reinterpret_cast<const R*>(S.poly), S.degree);
    for (int i = threadIdx.x; i < E3; i += blockDim.x) {
        const int a = i / (E * E), rem = i - a * E * E, b = rem / E, c = rem - b * E;
        const int gx = wrapi(ox + a, n), gy = wrapi(oy + b, n), gz = wrapi(oz + c, n);
        lds[i] = g[((long long)gx * n + gy) * rl + gz];
    }
    __syncthreads();
    const int deg = S.degree;
    const R sc = R(S.n) * R(S.inv_L);
    const R s0 = R(S.s0);
    const typename Vec4<R>::type* sorted = reinterpret_cast<const typename Vec4<R>::type*>(S.sorted);
    R* phi = reinterpret_cast<R*>(S.phi);
    R* F = reinterpret_cast<R*>(S.F);
    for (int k = beg + threadIdx.x; k < end; k += blockDim.x) {
        const typename Vec4<R>::type v = sorted[k];
        R w[3][P], dw[3][P];
        int l0[3];
        windows3_d<R, P>(v.x, v.y, v.z, ct, deg, w, dw, l0);
        const int bx = l0[0] - ox, by = l0[1] - oy, bz = l0[2] - oz;
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
        const int o = S.perm[k];
        if (phi) phi[o] = u - v.w * s0;
        if (F) {
            const R f = -v.w * sc;
            F[3LL * o + 0] = f * gxs;
            F[3LL * o + 1] = f * gys;
            F[3LL * o + 2] = f * gzs;
        }
    }
}

// Energy per system: E = E_k - S(0)/2 sum q^2, plus the charge sums.
__global__ void __launch_bounds__(256) k_finalize(const SysDesc* __restrict__ sys, const double* __restrict__ epart,
                                                  const double* __restrict__ bpart, double* __restrict__ E_dev) {
    __shared__ double red[16];
    const SysDesc& S = sys[blockIdx.x];
    double ek = 0.0, sq = 0.0, sa = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < S.ncol; i += blockDim.x) ek += epart[S.col_off + i];
    for (int i = threadIdx.x; i < S.npitem; i += blockDim.x) {
        sq += bpart[4 * (S.pitem_off + i) + 0];
        sa += bpart[4 * (S.pitem_off + i) + 1];
        s2 += bpart[4 * (S.pitem_off + i) + 2];
    }
    ek = block_sum(ek, red);
    sq = block_sum(sq, red);
    sa = block_sum(sa, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        const double E = ek - 0.5 * S.s0 * s2;
        S.out[0] = E;
        S.out[1] = sq;
        S.out[2] = sa;
        S.out[3] = s2;
        if (E_dev) E_dev[blockIdx.x] = E;
    }
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

__global__ void __launch_bounds__(256) k_drift(const SysDesc* __restrict__ sys, const int2* __restrict__ items) {
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int il = wi.y + threadIdx.x;
    if (S.step <= 0 || il >= S.N) return;
    float* pos = reinterpret_cast<float*>(const_cast<void*>(S.pos));
    const float L = (float)(1.0 / S.inv_L);
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
static hipError_t prepare_t(const Launch& L, int phase) {
    hipError_t e;
    switch (phase) {
        case 0:
            if ((e = allow_lds(k_hist<R>, L.hist_lds)) != hipSuccess) return e;
            k_hist<R><<<L.n_pitems, 256, L.hist_lds, L.stream>>>(L.sys, L.pitems, L.bpart);
            break;
        case 1:
            k_scan<<<L.nsys, 1024, 0, L.stream>>>(L.sys, L.bpart);
            break;
        case 2:
            k_scatter<R><<<L.n_pitems, 256, 0, L.stream>>>(L.sys, L.pitems);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prepare(const Launch& L, int phase) {
    return L.prec == 64 ? prepare_t<double>(L, phase) : prepare_t<float>(L, phase);
}

template <typename R, int P>
static hipError_t spread_p(const Launch& L, const Group& G) {
    hipError_t e = allow_lds(k_spread<R, P>, G.lds_spread);
    if (e != hipSuccess) return e;
    k_spread<R, P><<<G.count, 256, G.lds_spread, L.stream>>>(L.sys, L.titems + G.off);
    return hipGetLastError();
}

template <typename R, int P>
static hipError_t gather_p(const Launch& L, const Group& G) {
    hipError_t e = allow_lds(k_gather<R, P>, G.lds_gather);
    if (e != hipSuccess) return e;
    k_gather<R, P><<<G.count, 256, G.lds_gather, L.stream>>>(L.sys, L.titems + G.off);
    return hipGetLastError();
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
    k_drift<<<L.n_pitems, 256, 0, L.stream>>>(L.sys, L.pitems);
    return hipGetLastError();
}

hipError_t launch_finalize(const Launch& L, double* E_dev) {
    k_finalize<<<L.nsys, 256, 0, L.stream>>>(L.sys, L.epart, L.bpart, E_dev);
    return hipGetLastError();
}

}  // namespace esp
