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
// rc <= L/2 at most one image of a particle lies within rc. In a triclinic
// cell the bins and sub-cells are parallelepipeds of the fractional grid
// u = n H^-1 r; a sub-cell's edge is then measured between its faces
// (plane spacing), and displacements are mapped to Cartesian units by H/L
// before the distance test.
//
// Kernel. Inside rc, L(r) = 1/(4 pi r) - s(r) with s(r) = G(r/rc)/(4 pi r)
// smooth. In grid units s and s'(r)/r are polynomials A, B in x = r^2/rho^2
// (fitted on the host; the same coefficients for every lane), so a pair costs
// one reciprocal square root and two Horner evaluations:
//   u^l_i = (1/h)     sum_j q_j (1/(4 pi r) - A(x)),
//   F^l_i = (q_i/h^2) sum_j q_j (1/(4 pi r^3) + B(x)) (u_i - u_j),
// with r and u in grid units. The results go to a per-particle buffer in bin
// order, which the gather adds to phi and F; the energy partial of every bin,
// sum_i q_i u^l_i, goes to the launch's per-bin slots for k_finalize.
//
// Close pairs. The staged coordinates carry the rounding of values up to ~2T
// grid units (a few 1e-6), a large relative error of a displacement of a few
// hundredths of a grid unit, whose pair force is large. A pair closer than
// kClosePair grid units (h_x) therefore takes its displacement again, in
// FP64, from the caller's positions (minimum image), as the definition
// does; the sweep pays for that only on the rare wave steps where a lane
// meets such a pair.
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

// Grid coordinate of fractional coordinate t (FP64) relative to the origin
// o = tb T of its bin row, taken at the image nearest the bin's centre: values
// lie in [0, T) up to the rounding that placed the particle in this bin, so the
// stored coordinate keeps ~T/n times the precision of u itself.
template <typename R>
__device__ __forceinline__ R bin_local(double t, int n, int o, int T) {
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
constexpr double kClosePair = 0.5;  // grid units (h_x): pairs closer than this take an FP64 displacement

// Minimum-image displacement r_i - r_j in units of h_x (Cartesian), in FP64
// from the caller's positions.
__device__ __forceinline__ void exact_disp(const SysDesc& S, const double (&ri)[3], const double (&rj)[3],
                                           double& cx, double& cy, double& cz) {
    const double dx = ri[0] - rj[0], dy = ri[1] - rj[1], dz = ri[2] - rj[2];
    const double n = (double)S.n;
    if (S.tilt) {
        double sx = dx * S.inv_L + dy * S.ixy + dz * S.ixz;
        double sy = dy * S.inv_Ly + dz * S.iyz;
        double sz = dz * S.inv_Lz;
        sx = (sx - rint(sx)) * n;
        sy = (sy - rint(sy)) * n;
        sz = (sz - rint(sz)) * n;
        cx = sx + S.mxy * sy + S.mxz * sz;
        cy = S.lay * sy + S.myz * sz;
        cz = S.laz * sz;
    } else {
        const double sc = S.nside[0];  // 1/h_x
        cx = (dx - S.side[0] * rint(dx * S.inv_L)) * sc;
        cy = (dy - S.side[1] * rint(dy * S.inv_Ly)) * sc;
        cz = (dz - S.side[2] * rint(dz * S.inv_Lz)) * sc;
    }
}

template <typename R>
__device__ __forceinline__ void caller_pos(const SysDesc& S, int gi, double (&r)[3]) {
    const R* pos = reinterpret_cast<const R*>(S.pos);
    const long long p = S.perm[S.cidx[gi]];
    r[0] = (double)pos[3 * p + 0];
    r[1] = (double)pos[3 * p + 1];
    r[2] = (double)pos[3 * p + 2];
}

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
        const double x = pos[3LL * p + 0], y = pos[3LL * p + 1], z = pos[3LL * p + 2];
        V o;
        o.x = bin_local<R>(x * S.inv_L + (y * S.ixy + z * S.ixz), n, tx * T, T);
        o.y = bin_local<R>(y * S.inv_Ly + z * S.iyz, n, ty * T, T);
        o.z = bin_local<R>(z * S.inv_Lz, n, tz * T, T);
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

// One pair's contribution to i's sums; d = u_i - u_j in grid units. The
// polynomials A, B of degree D in y = x - 1/2 (x = r^2/rho^2) have the same
// coefficients for every lane (scalar registers).
template <typename R, int D>
__device__ __forceinline__ void pair_term(R dx, R dy, R dz, R qj, R rho2, R inv_rho2, const R (&cA)[D + 1],
                                          const R (&cB)[D + 1], R& up, R& fx, R& fy, R& fz) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rho2 && r2 > R(0)) {
        const R y = r2 * inv_rho2 - R(0.5);
        R A = cA[D], B = cB[D];
#pragma unroll
        for (int m = D - 1; m >= 0; --m) {
            A = A * y + cA[m];
            B = B * y + cB[m];
        }
        const R ri = rsqrt_r<R>(r2);
        const R rc4 = R(0.079577471545947667884) * ri;  // 1/(4 pi r)
        up += qj * (rc4 - A);
        const R g = qj * (rc4 * ri * ri + B);
        fx += g * dx;
        fy += g * dy;
        fz += g * dz;
    }
}

// Exclusive scan of a[0..n) in LDS by the whole block; a[n] gets the total.
__device__ void block_exclusive_scan(int* a, int n, int* wsum) {
    const int BD = blockDim.x, per = (n + BD - 1) / BD;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    int sum = 0;
    for (int i = lo; i < hi; ++i) sum += a[i];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wid; ++w) base += wsum[w];
    int run = base + inc - sum;
    for (int i = lo; i < hi; ++i) {
        const int c = a[i];
        a[i] = run;
        run += c;
    }
    if (threadIdx.x == BD - 1) a[n] = run;
    __syncthreads();
}

// The pair sums of one block of lsa^3 sub-cells of a bin (a local work
// item). The particles of the (lsa + 2 lR)^3 sub-cells around the block (its
// halo) are staged in LDS, shifted into the bin's frame, in halo sub-cell order
// (z fastest): for every (dx, dy) of the stencil the 2 lR + 1 sub-cells along z
// form one contiguous run. A block whose halo exceeds the LDS staging walks
// the sub-cells in global memory instead. The block's own particles are lsa^2
// runs of consecutive sub-cells along z in the bin's sub-cell order.
template <typename R, int D>
__global__ void __launch_bounds__(kLocalThreads) k_local(const SysDesc* __restrict__ sys,
                                                         const int2* __restrict__ items, double* __restrict__ lpart,
                                                         int cap) {
    using V = typename Vec4<R>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    __shared__ int wsum[kLocalThreads / 64];
    __shared__ int roff[65], rglob[64];  // own runs (lsa^2 <= 64): first index in the block, in cpos
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    if (!S.local) return;  // uniform over the block
    const int s = S.lcs, nc = s * s * s, LR = S.lR, a = S.lsa, nsb = s / a, nsb3 = nsb * nsb * nsb;
    const int t = wi.y / nsb3, sub = wi.y - t * nsb3;
    const int ox = (sub / (nsb * nsb)) * a, oy = ((sub / nsb) % nsb) * a, oz = (sub % nsb) * a;
    const int t1 = S.tiles1, T = S.T, G = t1 * s;
    // degree <= D: the table is zero-padded beyond the system's degree
    const R* gc = reinterpret_cast<const R*>(S.lcoef);
    R cA[D + 1], cB[D + 1];
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        cA[m] = gc[m];
        cB[m] = gc[kLocalCoefStride + m];
    }
    int tx, ty, tz;
    bin_coords_l(t, S, tx, ty, tz);
    const R rho2 = R(S.lrho2), inv_rho2 = R(1.0 / S.lrho2);
    const R close2 = R(kClosePair * kClosePair);
    const R lsT = R(S.lsT);
    const R sc = R(S.n * S.inv_L);  // 1/h_x
    // pair geometry in units of h_x: a grid-unit displacement d maps to
    // (H/L) d, upper triangular with diagonal (1, h_y/h_x, h_z/h_x) and
    // off-diagonal entries only in a triclinic cell
    const R ay = R(S.lay), az = R(S.laz), mxy = R(S.mxy), mxz = R(S.mxz), myz = R(S.myz);
    // explicit fused operations: a particle's own staged copy maps to exactly
    // its own coordinates, so the self pair keeps r = 0
    auto to_cart = [&](R gx, R gy, R gz, R& cx, R& cy, R& cz) {
        cx = fma(mxz, gz, fma(mxy, gy, gx));
        cy = fma(myz, gz, gy * ay);
        cz = gz * az;
    };
    // separable sub-cell index: cell(gx, gy, gz) = X(gx) + Y(gy) + Z(gz) with
    // Z(g) = (g/s)(nc - s) + g, Y(g) = (g/s)(t1 nc - s^2) + s g,
    // X(g) = (g/s)(t1^2 nc - s^3) + s^2 g
    const int zq = nc - s, yq = t1 * nc - s * s, xq = t1 * t1 * nc - nc;
    const V* cpos = reinterpret_cast<const V*>(S.cpos);
    const int* cst = S.cstart;
    V* loc = reinterpret_cast<V*>(S.loc);
    const int W = a + 2 * LR, W3 = W * W * W;
    V* hp = reinterpret_cast<V*>(smem_raw);
    int* hs = reinterpret_cast<int*>(smem_raw + (size_t)cap * sizeof(V));
    // halo row h along one axis of a block starting at sub-cell o of bin row
    // b: its global sub-cell and the shift into the bin's frame (grid units)
    auto halo_axis = [&](int h, int b, int o, int& g, int& shift) {
        g = b * s + o - LR + h;
        int w = 0;
        if (g < 0) {
            g += G;
            w = -t1;
        } else if (g >= G) {
            g -= G;
            w = t1;
        }
        shift = (g / s + w - b) * T;
    };
    auto halo_cell = [&](int c, int& cell, R& sx, R& sy, R& sz) {
        const int hz = c % W, hy = (c / W) % W, hx = c / (W * W);
        int gx, gy, gz, ix, iy, iz;
        halo_axis(hx, tx, ox, gx, ix);
        halo_axis(hy, ty, oy, gy, iy);
        halo_axis(hz, tz, oz, gz, iz);
        cell = (gx / s) * xq + s * s * gx + (gy / s) * yq + s * gy + (gz / s) * zq + gz;
        sx = R(ix);
        sy = R(iy);
        sz = R(iz);
    };
    for (int c = threadIdx.x; c < W3; c += blockDim.x) {
        int cell;
        R sx, sy, sz;
        halo_cell(c, cell, sx, sy, sz);
        hs[c] = cst[cell + 1] - cst[cell];
    }
    // own runs: sub-cells (ox + i, oy + j, oz .. oz + a - 1) of this bin
    if (threadIdx.x < a * a) {
        const int r = threadIdx.x;
        const int c0 = t * nc + ((ox + r / a) * s + (oy + r % a)) * s + oz;
        rglob[r] = cst[c0];
        roff[r] = cst[c0 + a] - cst[c0];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int r = 0; r < a * a; ++r) {
            const int c = roff[r];
            roff[r] = run;
            run += c;
        }
        roff[a * a] = run;
    }
    block_exclusive_scan(hs, W3, wsum);  // synchronises, so roff is complete too
    const bool staged = hs[W3] <= cap;  // uniform over the block
    if (staged) {
        for (int c = threadIdx.x; c < W3; c += blockDim.x) {
            int cell;
            R sx, sy, sz;
            halo_cell(c, cell, sx, sy, sz);
            const int j0 = cst[cell], nj = cst[cell + 1] - j0;
            V* dst = hp + hs[c];
            for (int j = 0; j < nj; ++j) {
                V v = cpos[j0 + j];
                to_cart(v.x + sx, v.y + sy, v.z + sz, v.x, v.y, v.z);
                dst[j] = v;
            }
        }
        __syncthreads();
    }
    const int nown = roff[a * a];
    const int span = 2 * LR + 1, nrun = span * span;
    // lanes per own particle: a block with few own particles (coarse sub-cells,
    // as in strongly tilted cells) splits each particle's stencil rows over NL
    // adjacent lanes and adds their partial sums in a fixed butterfly order
    int NL = 1;
    if (staged)
        while (NL < 16 && 2 * NL <= nrun && 2 * NL * nown <= (int)blockDim.x) NL *= 2;
    const int gl = threadIdx.x & (NL - 1);
    double e = 0.0;
    for (int k = threadIdx.x / NL; k < nown; k += blockDim.x / NL) {
        int lo = 0, hi = a * a;  // run r with roff[r] <= k < roff[r + 1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (roff[mid] <= k)
                lo = mid;
            else
                hi = mid;
        }
        const int gi = rglob[lo] + (k - roff[lo]);
        const V vi = cpos[gi];
        const int lx = sub_cell<R>(vi.x, 0, s, lsT);
        const int ly = sub_cell<R>(vi.y, 0, s, lsT);
        const int lz = sub_cell<R>(vi.z, 0, s, lsT);
        R up = 0, fx = 0, fy = 0, fz = 0;
        double ri[3];  // i's caller position, for close pairs
        caller_pos<R>(S, gi, ri);
        // a pair closer than kClosePair: its displacement from the caller's
        // positions (j: index into cpos)
        auto refine = [&](int gj, R& dx, R& dy, R& dz) {
            const R r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < close2 && r2 > R(0)) {
                double rj[3], cx, cy, cz;
                caller_pos<R>(S, gj, rj);
                exact_disp(S, ri, rj, cx, cy, cz);
                dx = R(cx);
                dy = R(cy);
                dz = R(cz);
            }
        };
        if (staged) {
            R vix, viy, viz;
            to_cart(vi.x, vi.y, vi.z, vix, viy, viz);
            // index into cpos of the staged particle in slot j of the z-run
            // of halo cells row .. row + 2 lR
            auto global_of = [&](int row, int j) {
                int c = row;
                while (c < row + 2 * LR && hs[c + 1] <= j) ++c;
                int cell;
                R sx, sy, sz;
                halo_cell(c, cell, sx, sy, sz);
                return cst[cell] + (j - hs[c]);
            };
            auto staged_pair = [&](int row, int j, const V& vj) {
                R dx = vix - vj.x, dy = viy - vj.y, dz = viz - vj.z;
                const R r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < close2 && r2 > R(0)) refine(global_of(row, j), dx, dy, dz);
                pair_term<R, D>(dx, dy, dz, vj.w, rho2, inv_rho2, cA, cB, up, fx, fy, fz);
            };
            // halo rows hx .. hx + 2 lR around halo row hx + lR of the particle
            const int hx = min(max(lx - ox, 0), a - 1), hy = min(max(ly - oy, 0), a - 1),
                      hz = min(max(lz - oz, 0), a - 1);
            for (int rr = gl; rr < nrun; rr += NL) {
                const int u = rr / span, v = rr - u * span;
                const int row = ((hx + u) * W + (hy + v)) * W + hz;
                const int ja = hs[row], jb = hs[row + 2 * LR + 1];
                // four candidates loaded before any is used: the LDS
                // latency overlaps instead of stalling every pair
                int j = ja;
                for (; j + 3 < jb; j += 4) {
                    const V v0 = hp[j], v1 = hp[j + 1], v2 = hp[j + 2], v3 = hp[j + 3];
                    staged_pair(row, j, v0);
                    staged_pair(row, j + 1, v1);
                    staged_pair(row, j + 2, v2);
                    staged_pair(row, j + 3, v3);
                }
                for (; j < jb; ++j) staged_pair(row, j, hp[j]);
            }
        } else {
            const int cx = tx * s + lx, cy = ty * s + ly, cz = tz * s + lz;
            // i's coordinates in the frame of the neighbour's bin: each stored
            // coordinate is relative to its own bin's origin, so the frames
            // differ by whole bins (exact), periodic images included
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
                            R dx, dy, dz;
                            to_cart(xs - vj.x, ys - vj.y, zs - vj.z, dx, dy, dz);
                            if (j != gi) refine(j, dx, dy, dz);
                            pair_term<R, D>(dx, dy, dz, vj.w, rho2, inv_rho2, cA, cB, up, fx, fy, fz);
                        }
                    }
                }
            }
        }
        for (int off = NL >> 1; off > 0; off >>= 1) {  // the lanes of a group are all active
            up += __shfl_xor(up, off, 64);
            fx += __shfl_xor(fx, off, 64);
            fy += __shfl_xor(fy, off, 64);
            fz += __shfl_xor(fz, off, 64);
        }
        if (gl == 0) {
            const R pot = up * sc;
            const R fq = vi.w * sc * sc;
            V o;
            o.x = pot;
            o.y = fq * fx;
            o.z = fq * fy;
            o.w = fq * fz;
            loc[S.cidx[gi]] = o;
            e += (double)vi.w * (double)pot;
        }
    }
    e = block_sum(e, red);
    if (threadIdx.x == 0) lpart[blockIdx.x] = e;
}

template <typename R, int D>
static hipError_t local_d(const Launch& L) {
    const int lds = L.local_cap * (int)sizeof(typename Vec4<R>::type) + (L.local_cells + 1) * 4;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_local<R, D>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    k_cellsort<R><<<L.n_titems, kLocalThreads, 0, L.stream>>>(L.sys, L.titems);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_local<R, D><<<L.n_litems, kLocalThreads, lds, L.stream>>>(L.sys, L.litems, L.lpart, L.local_cap);
    return hipGetLastError();
}

// the launch's largest degree, rounded up to an even kernel instance
template <typename R>
static hipError_t local_t(const Launch& L) {
    if (L.local_deg <= 8) return local_d<R, 8>(L);
    if (L.local_deg <= 10) return local_d<R, 10>(L);
    if (L.local_deg <= 12) return local_d<R, 12>(L);
    if (L.local_deg <= 14) return local_d<R, 14>(L);
    if (L.local_deg <= kLocalCoefStride - 1) return local_d<R, 16>(L);
    return hipErrorInvalidValue;
}

hipError_t launch_local(const Launch& L) {
    if (!L.any_local || L.n_titems == 0 || L.n_litems == 0) return hipSuccess;
    return L.prec == 64 ? local_t<double>(L) : local_t<float>(L);
}

}  // namespace esp
