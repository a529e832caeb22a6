// Local part of the split on the device (Methods, eq. localpart with the
// kernel L(r) of eq. kernelsplitting):
//   u^l_i = sum_{j != i, |r_ij| < rc} q_j L(|r_ij|)   over nearest images,
//   F^l_i = -q_i grad_i u^l_i.
// Added to the long-range outputs, phi, F and E become the full Coulomb values
// of the problem statement (eq. task).
//
// Cells. Each long-range bin (T^3 grid cells) is split into lcs^3 sub-cells of
// edge e = T/lcs >= rho/2 (rho = rc/h), so every pair within rc lies within lR
// sub-cells along each axis. k_cellsort reorders each bin's particles by
// sub-cell, and inside a sub-cell by caller index: the pair sums then run in an
// order fixed by the positions and the caller's numbering alone, whatever the
// binning path or the order its LDS atomics left inside a bin. k_local gives
// every particle of a bin one thread, which walks the (2 lR + 1)^3 sub-cells
// around its own; a periodic image is a shift by n grid units, and with
// rc <= L/2 at most one image of a particle lies within rc.
//
// Kernel. Inside rc, L(r) = 1/(4 pi r) - s(r) with s(r) = G(r/rc)/(4 pi r)
// smooth. In grid units s and s'(r)/r are piecewise polynomials A, B in
// x = r^2/rho^2 (fitted on the host), so a pair costs one reciprocal square
// root and two Horner evaluations:
//   u^l_i = (1/h)     sum_j q_j (1/(4 pi r) - A(x)),
//   F^l_i = (q_i/h^2) sum_j q_j (1/(4 pi r^3) + B(x)) (u_i - u_j),
// with r and u in grid units. The results go to a per-particle buffer in bin
// order, which the gather adds to phi and F; the energy partial of every bin,
// sum_i q_i u^l_i, goes to the launch's per-bin slots for k_finalize.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace esp {

namespace {

__device__ __forceinline__ void bin_coords_l(int t, const SysDesc& S, int& tx, int& ty, int& tz) {
    const int t1 = S.tiles1;
    tz = t % t1;
    const int r = t / t1;
    ty = r % t1;
    tx = r / t1;
}

// Sub-cell coordinate (0 .. lcs-1) of grid coordinate u inside bin row tb.
template <typename R>
__device__ __forceinline__ int sub_cell(R u, int tb, int lcs, R lsT) {
    const int c = (int)floor(u * lsT) - tb * lcs;
    return min(max(c, 0), lcs - 1);
}

// Grid coordinate of position x relative to the origin o = tb T of its bin
// row, in FP64 and taken at the image nearest the bin's centre: values lie in
// [0, T) up to the rounding that placed the particle in this bin, so the
// stored coordinate keeps ~T/n times the precision of u itself.
template <typename R>
__device__ __forceinline__ R bin_local(R x, double inv_L, int n, int o, int T) {
    double t = (double)x * inv_L;
    t -= floor(t);
    double u = t * n - o;
    const double c = u - 0.5 * T;
    if (c >= 0.5 * n) u -= n;
    if (c < -0.5 * n) u += n;
    return R(u);
}

template <typename R>
__device__ __forceinline__ R rsqrt_r(R x);
template <>
__device__ __forceinline__ float rsqrt_r<float>(float x) {
    return rsqrtf(x);
}
template <>
__device__ __forceinline__ double rsqrt_r<double>(double x) {
    return 1.0 / sqrt(x);
}

}  // namespace

constexpr int kMaxSubCells = 512;  // lcs <= 8

template <typename R>
__global__ void __launch_bounds__(kLocalThreads) k_cellsort(const SysDesc* __restrict__ sys,
                                                            const int2* __restrict__ items) {
    using V = typename Vec4<R>::type;
    __shared__ int cnt[kMaxSubCells];
    __shared__ int first[kMaxSubCells];
    __shared__ int cur[kMaxSubCells];
    __shared__ int key_s[kCellSortCap];
    __shared__ int perm_s[kCellSortCap];
    __shared__ int src_s[kCellSortCap];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (!S.local) return;  // uniform over the block
    const int t = wi.y, s = S.lcs, nc = s * s * s;
    const int beg = S.bin_start[t], count = S.bin_start[t + 1] - beg;
    int tx, ty, tz;
    bin_coords_l(t, S, tx, ty, tz);
    const R lsT = R(S.lsT);
    const V* src = reinterpret_cast<const V*>(S.sorted) + beg;
    const int* perm = S.perm + beg;
    // the copy the pair sums read: coordinates relative to the bin's origin,
    // from the caller's positions; the sub-cell key comes from the same
    // coordinates, so a particle's sub-cell and stored position always agree
    const R* pos = reinterpret_cast<const R*>(S.pos);
    const int n = S.n, T = S.T;
    auto local_coords = [&](int p, R qv) {
        V o;
        o.x = bin_local<R>(pos[3LL * p + 0], S.inv_L, n, tx * T, T);
        o.y = bin_local<R>(pos[3LL * p + 1], S.inv_L, n, ty * T, T);
        o.z = bin_local<R>(pos[3LL * p + 2], S.inv_L, n, tz * T, T);
        o.w = qv;
        return o;
    };
    auto keyof = [&](int i) {
        const V v = local_coords(perm[i], R(0));
        return (sub_cell<R>(v.x, 0, s, lsT) * s + sub_cell<R>(v.y, 0, s, lsT)) * s + sub_cell<R>(v.z, 0, s, lsT);
    };
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        cnt[c] = 0;
        cur[c] = 0;
    }
    __syncthreads();
    const bool staged = count <= kCellSortCap;
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const int k = keyof(i);
        if (staged) key_s[i] = k;
        atomicAdd(&cnt[k], 1);
    }
    __syncthreads();
    // exclusive scan of the sub-cell counts by the first wave, 8 per lane
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int v[8], sum = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = lane * 8 + j;
            v[j] = c < nc ? cnt[c] : 0;
            sum += v[j];
        }
        int inc = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const int u = __shfl_up(inc, off, 64);
            if (lane >= off) inc += u;
        }
        int run = inc - sum;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = lane * 8 + j;
            if (c < nc) first[c] = run;
            run += v[j];
        }
    }
    __syncthreads();
    int* cstart = S.cstart + (long long)t * nc;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) cstart[c] = beg + first[c];
    const int nbins = S.tiles1 * S.tiles1 * S.tiles1;
    if (t == nbins - 1 && threadIdx.x == 0) S.cstart[(long long)nbins * nc] = S.N;
    V* dst = reinterpret_cast<V*>(S.cpos) + beg;
    int* didx = S.cidx + beg;
    if (staged) {
        // place (order inside a sub-cell left open), then rank inside the
        // sub-cell by caller index
        for (int i = threadIdx.x; i < count; i += blockDim.x) {
            const int k = key_s[i];
            const int slot = first[k] + atomicAdd(&cur[k], 1);
            perm_s[slot] = perm[i];
            src_s[slot] = i;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < count; j += blockDim.x) {
            const int i = src_s[j];
            const int k = key_s[i];
            const int p = perm_s[j];
            const int a = first[k], b = a + cnt[k];
            int r = 0;
            for (int m = a; m < b; ++m) r += perm_s[m] < p;
            dst[a + r] = local_coords(p, src[i].w);
            didx[a + r] = beg + i;
        }
    } else {
        // a bin beyond the LDS staging: rank against the whole bin
        for (int i = threadIdx.x; i < count; i += blockDim.x) {
            const int k = keyof(i), p = perm[i];
            int r = 0;
            for (int m = 0; m < count; ++m) r += (perm[m] < p) && (keyof(m) == k);
            dst[first[k] + r] = local_coords(p, src[i].w);
            didx[first[k] + r] = beg + i;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kLocalThreads) k_local(const SysDesc* __restrict__ sys,
                                                         const int2* __restrict__ items, double* __restrict__ lpart) {
    using V = typename Vec4<R>::type;
    __shared__ R coef[kLocalCoefMax];
    __shared__ double red[16];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (!S.local) return;  // uniform over the block
    const int t = wi.y, s = S.lcs, nc = s * s * s, LR = S.lR, K = S.lpieces, d1 = S.ldeg + 1;
    const int t1 = S.tiles1, T = S.T, G = t1 * s;
    const int beg = S.bin_start[t], count = S.bin_start[t + 1] - beg;
    const R* gc = reinterpret_cast<const R*>(S.lcoef);
    for (int i = threadIdx.x; i < 2 * K * d1; i += blockDim.x) coef[i] = gc[i];
    __syncthreads();
    const R* cA = coef;
    const R* cB = coef + K * d1;
    int tx, ty, tz;
    bin_coords_l(t, S, tx, ty, tz);
    const R rho2 = R(S.lrho2), inv_rho2 = R(1.0 / S.lrho2), Kf = R(K);
    const R c4 = R(0.079577471545947667884);  // 1/(4 pi)
    const R lsT = R(S.lsT);
    const R sc = R(S.n * S.inv_L);  // 1/h
    // separable sub-cell index: cell(gx, gy, gz) = X(gx) + Y(gy) + Z(gz) with
    // Z(g) = (g/s)(nc - s) + g, Y(g) = (g/s)(t1 nc - s^2) + s g,
    // X(g) = (g/s)(t1^2 nc - s^3) + s^2 g
    const int zq = nc - s, yq = t1 * nc - s * s, xq = t1 * t1 * nc - nc;
    const V* cpos = reinterpret_cast<const V*>(S.cpos);
    const int* cst = S.cstart;
    V* loc = reinterpret_cast<V*>(S.loc);
    double e = 0.0;
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        const V vi = cpos[beg + k];
        const int cx = tx * s + sub_cell<R>(vi.x, 0, s, lsT);
        const int cy = ty * s + sub_cell<R>(vi.y, 0, s, lsT);
        const int cz = tz * s + sub_cell<R>(vi.z, 0, s, lsT);
        R up = 0, fx = 0, fy = 0, fz = 0;
        // i's coordinates in the frame of the neighbour's bin: each stored
        // coordinate is relative to its own bin's origin, so the frames differ
        // by whole bins (exact), periodic images included
        for (int dx = -LR; dx <= LR; ++dx) {
            int gx = cx + dx, wx = 0;
            if (gx < 0) {
                gx += G;
                wx = -t1;
            } else if (gx >= G) {
                gx -= G;
                wx = t1;
            }
            const int bx = gx / s;
            const R xs = vi.x + R((tx - bx - wx) * T);
            const int X = bx * xq + s * s * gx;
            for (int dy = -LR; dy <= LR; ++dy) {
                int gy = cy + dy, wy = 0;
                if (gy < 0) {
                    gy += G;
                    wy = -t1;
                } else if (gy >= G) {
                    gy -= G;
                    wy = t1;
                }
                const int by = gy / s;
                const R ys = vi.y + R((ty - by - wy) * T);
                const int XY = X + by * yq + s * gy;
                for (int dz = -LR; dz <= LR; ++dz) {
                    int gz = cz + dz, wz = 0;
                    if (gz < 0) {
                        gz += G;
                        wz = -t1;
                    } else if (gz >= G) {
                        gz -= G;
                        wz = t1;
                    }
                    const int bz = gz / s;
                    const R zs = vi.z + R((tz - bz - wz) * T);
                    const int cell = XY + bz * zq + gz;
                    const int ja = cst[cell], jb = cst[cell + 1];
                    for (int j = ja; j < jb; ++j) {
                        const V vj = cpos[j];
                        const R ddx = xs - vj.x, ddy = ys - vj.y, ddz = zs - vj.z;
                        const R r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        if (r2 < rho2 && r2 > R(0)) {
                            const R x = r2 * inv_rho2;
                            const int pc = min((int)(x * Kf), K - 1);
                            const R y = x * Kf - R(pc) - R(0.5);
                            const R* a = cA + pc * d1;
                            const R* b = cB + pc * d1;
                            R A = a[d1 - 1], B = b[d1 - 1];
                            for (int m = d1 - 2; m >= 0; --m) {
                                A = A * y + a[m];
                                B = B * y + b[m];
                            }
                            const R ri = rsqrt_r<R>(r2);
                            const R rc4 = c4 * ri;
                            up += vj.w * (rc4 - A);
                            const R g = vj.w * (rc4 * ri * ri + B);
                            fx += g * ddx;
                            fy += g * ddy;
                            fz += g * ddz;
                        }
                    }
                }
            }
        }
        const R pot = up * sc;
        const R fq = vi.w * sc * sc;
        V o;
        o.x = pot;
        o.y = fq * fx;
        o.z = fq * fy;
        o.w = fq * fz;
        loc[S.cidx[beg + k]] = o;
        e += (double)vi.w * (double)pot;
    }
    e = block_sum(e, red);
    if (threadIdx.x == 0) lpart[blockIdx.x] = e;
}

hipError_t launch_local(const Launch& L) {
    if (!L.any_local || L.n_titems == 0) return hipSuccess;
    if (L.prec == 64) {
        k_cellsort<double><<<L.n_titems, kLocalThreads, 0, L.stream>>>(L.sys, L.titems);
        k_local<double><<<L.n_titems, kLocalThreads, 0, L.stream>>>(L.sys, L.titems, L.lpart);
    } else {
        k_cellsort<float><<<L.n_titems, kLocalThreads, 0, L.stream>>>(L.sys, L.titems);
        k_local<float><<<L.n_titems, kLocalThreads, 0, L.stream>>>(L.sys, L.titems, L.lpart);
    }
    return hipGetLastError();
}

}  // namespace esp
