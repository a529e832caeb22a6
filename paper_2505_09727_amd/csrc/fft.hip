// 3D FFT, influence scaling and k-space energy of the ESP long-range
// pipeline (Methods, "Fast algorithm for the spectral part": the forward
// transform of the spread grid, the diagonal scaling by p_k of eq. pk, the
// inverse transform), for gfx950.
//
// Real grids are stored n x n x (n+2): the half spectrum n x n x (n/2+1) of an
// x-plane overwrites that plane in place. The transform runs as three passes:
//   fwd_zy  one block per x-plane: real-to-complex along z, complex along y;
//           with from_tiles the plane is first assembled from the spread's
//           bin tiles (halo fold);
//   x       one block per chunk of consecutive (ky, kz) columns: forward
//           along x, scaling by p_k with the energy partial, inverse along x;
//   inv_yz  one block per x-plane: inverse along y, complex-to-real along z.
//
// Every kernel is instantiated per grid size N (even, 2^a 3^b, 8..144), so the
// Stockham stages are fully resolved at compile time: radix 4 while 4 divides
// the remaining length, then 2, then 3. A system's result depends only on its
// own N (not on the other systems of a launch), and the arithmetic is not
// contracted into FMAs, so results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "device_util.hpp"
#include "kernels.hpp"

namespace esp {

#pragma clang fp contract(off)

// One Stockham autosort stage of radix RAD after NS points have been combined,
// on NL lines of length N held in LDS; element (line, idx) is at
// buf[base(line) + idx * ES], base(line) = (line / L1) S1 + (line % L1) S2
// (lines grouped L1 to a plane). Every thread loads and transforms its butterflies
// into registers, the block synchronises, then every thread stores, so the
// stage runs in place. LF maps consecutive threads to consecutive lines.
template <typename R, int N, int RAD, int NS, int NL, int L1, int S1, int S2, int ES, int BD, bool LF, int DIR>
__device__ __forceinline__ void st_stage(cplx<R>* __restrict__ buf, const cplx<R>* __restrict__ tw) {
    constexpr int NB = N / RAD;
    constexpr int TOTAL = NL * NB;
    constexpr int SPAN = N / (NS * RAD);
    constexpr int IT = (TOTAL + BD - 1) / BD;
    cplx<R> v[IT][RAD];
    int dst[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int item = threadIdx.x + it * BD;
        dst[it] = -1;
        if (TOTAL % BD == 0 || item < TOTAL) {
            int line, j;
            if constexpr (LF) {
                j = item / NL;
                line = item - j * NL;
            } else {
                line = item / NB;
                j = item - line * NB;
            }
            const int lb = (line / L1) * S1 + (line % L1) * S2;
            const cplx<R>* src = buf + lb + j * ES;
            const int jm = j % NS;
#pragma unroll
            for (int k = 0; k < RAD; ++k) {
                cplx<R> a = src[k * NB * ES];
                if constexpr (NS > 1) {
                    if (k > 0) {
                        cplx<R> w = tw[k * jm * SPAN];
                        if constexpr (DIR < 0) w.y = -w.y;
                        a = cmul(a, w);
                    }
                }
                v[it][k] = a;
            }
            Bfly<R, RAD>::run(v[it], DIR);
            dst[it] = lb + ((j - jm) * RAD + jm) * ES;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        if (dst[it] >= 0) {
#pragma unroll
            for (int k = 0; k < RAD; ++k) buf[dst[it] + k * NS * ES] = v[it][k];
        }
    }
    __syncthreads();
}

// Unnormalised DFT y_k = sum_l exp(DIR 2 pi i k l / N) x_l of NL lines in LDS,
// natural order in and out; tw[t] = exp(2 pi i t / N).
template <typename R, int N, int NS, int NL, int L1, int S1, int S2, int ES, int BD, bool LF, int DIR>
__device__ __forceinline__ void fft_ct2(cplx<R>* __restrict__ buf, const cplx<R>* __restrict__ tw) {
    if constexpr (NS < N) {
        constexpr int M = N / NS;
        constexpr int RAD = M % 4 == 0 ? 4 : (M % 2 == 0 ? 2 : 3);
        st_stage<R, N, RAD, NS, NL, L1, S1, S2, ES, BD, LF, DIR>(buf, tw);
        fft_ct2<R, N, NS * RAD, NL, L1, S1, S2, ES, BD, LF, DIR>(buf, tw);
    }
}

// Lines at buf[line * LS + idx * ES].
template <typename R, int N, int NS, int NL, int LS, int ES, int BD, bool LF, int DIR>
__device__ __forceinline__ void fft_ct(cplx<R>* __restrict__ buf, const cplx<R>* __restrict__ tw) {
    fft_ct2<R, N, NS, NL, NL, 0, LS, ES, BD, LF, DIR>(buf, tw);
}

// Launch shapes, functions of N and the real type only.
template <int N> constexpr int plane_threads() {
    constexpr int items = (N / 2 + 1) * (N / 4 > 0 ? N / 4 : 1);
    return items <= 64 ? 64 : items <= 128 ? 128 : items <= 256 ? 256 : 512;
}
template <typename R> constexpr int x_columns() { return 256 / (int)sizeof(cplx<R>); }  // 256-byte row chunks
template <typename R, int N> constexpr int x_threads() {
    constexpr int items = x_columns<R>() * (N / 4 > 0 ? N / 4 : 1);
    return items <= 64 ? 64 : items <= 128 ? 128 : items <= 256 ? 256 : 512;
}

// Assemble grid plane x from the spread's bin tiles (the halo fold): every
// point sums the tile entries that cover it, at most 3 per axis (a tile spans
// E = T + P - 1 + (P odd) <= T + 12 points and T >= 8), over x, then y, then z
// entries. The first floor(BD / N) N threads each own one column z, whose
// entries they look up once, and walk the rows y = tid / N, + floor(BD / N),
// ...; a row's y entries are common to the lanes on that row. The result goes
// to LDS in pair-row order: rows 2r and 2r+1 are the real and imaginary parts
// of complex row r, rows N + 1 complex values apart (conflict-free z stages).
template <typename R, int N, int BD>
__device__ __forceinline__ void fold_plane(R* __restrict__ bufr, const R* __restrict__ tiles, const SysDesc& S,
                                           const CoverTab* __restrict__ tab, const CoverTab& cx) {
    static_assert(BD >= N, "one thread per column at least");
    constexpr int RS = BD / N;
    const int t1 = S.tiles1, E = S.E, EE = E * E, E3 = EE * E;
    const int r0 = (int)threadIdx.x / N, z = (int)threadIdx.x - r0 * N;
    if (r0 >= RS) return;
    const auto tg = gptr(tiles);
    const CoverTab cz = tab[z];
    int zo[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) zo[c] = c < cz.cnt ? cz.bin[c] * E3 + cz.off[c] : 0;
    // two rows per step, the loads of both issued before any is summed
    for (int y0 = r0; y0 < N; y0 += 2 * RS) {
        int yo[2][3], ycnt[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int y = y0 + u * RS;
            const CoverTab cy = tab[y < N ? y : 0];
            ycnt[u] = y < N ? cy.cnt : 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) yo[u][b] = b < cy.cnt ? cy.bin[b] * t1 * E3 + cy.off[b] * E : 0;
        }
        R acc[2] = {R(0), R(0)};
        for (int a = 0; a < cx.cnt; ++a) {
            const int xo = cx.bin[a] * t1 * t1 * E3 + cx.off[a] * EE;
            R v[2][3][3];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        v[u][b][c] = (b < ycnt[u] && c < cz.cnt) ? tg[(unsigned)(xo + yo[u][b] + zo[c])] : R(0);
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[u] += v[u][b][c];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int y = y0 + u * RS;
            if (y < N) bufr[2 * ((y >> 1) * (N + 1) + z) + (y & 1)] = acc[u];
        }
    }
}

// Forward pass along z (two real rows transformed as one complex row, then
// separated) and y, for one x-plane.
template <typename R, int N>
__global__ void __launch_bounds__(plane_threads<N>()) k_fwd_zy(const SysDesc* __restrict__ sys,
                                                              const int2* __restrict__ items, int from_tiles) {
    constexpr int HS = N / 2 + 1, RL = N + 2, HALF = N / 2, BD = plane_threads<N>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* buf = tw + N;
    const cplx<R>* tw_g = reinterpret_cast<const cplx<R>*>(S.tw);
    for (int i = threadIdx.x; i < N; i += BD) tw[i] = tw_g[i];
    R* plane = reinterpret_cast<R*>(S.grid) + (long long)wi.y * N * RL;
    if (from_tiles) {
        CoverTab* tab = reinterpret_cast<CoverTab*>(buf + N * HS);
        build_cover(tab, S, -((S.P - 1) / 2));
        __syncthreads();
        fold_plane<R, N, BD>(reinterpret_cast<R*>(buf), reinterpret_cast<const R*>(S.tiles), S, tab, tab[wi.y]);
    } else {
        for (int idx = threadIdx.x; idx < HALF * N; idx += BD) {
            const int r = idx / N, z = idx - r * N;
            buf[r * (N + 1) + z] = {gptr(plane)[(2 * r) * RL + z], gptr(plane)[(2 * r + 1) * RL + z]};
        }
    }
    __syncthreads();
    // z: pair rows N + 1 apart, consecutive threads on consecutive rows
    fft_ct<R, N, 1, HALF, N + 1, 1, BD, true, +1>(buf, tw);
    {
        constexpr int TOTAL = HALF * HS, IT = (TOTAL + BD - 1) / BD;
        cplx<R> A[IT], B[IT];
        int o[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int item = threadIdx.x + it * BD;
            o[it] = -1;
            if (item < TOTAL) {
                const int r = item / HS, k = item - r * HS;
                const cplx<R> zk = buf[r * (N + 1) + k];
                const cplx<R> zn = buf[r * (N + 1) + (k == 0 ? 0 : N - k)];
                A[it] = {R(0.5) * (zk.x + zn.x), R(0.5) * (zk.y - zn.y)};
                B[it] = {R(0.5) * (zk.y + zn.y), -R(0.5) * (zk.x - zn.x)};
                o[it] = (2 * r) * HS + k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; ++it)
            if (o[it] >= 0) {
                buf[o[it]] = A[it];
                buf[o[it] + HS] = B[it];
            }
        __syncthreads();
    }
    fft_ct<R, N, 1, HS, 1, HS, BD, true, +1>(buf, tw);
    cplx<R>* gp = reinterpret_cast<cplx<R>*>(plane);
    for (int idx = threadIdx.x; idx < N * HS; idx += BD) gstore_c(gp, idx, buf[idx]);
}

// Spectral derivative factor of one axis for index k of an n-point
// transform: the derivative of exp(-2 pi i m x/L) is -2 pi i m/L times it
// (m = k or k - n); 0 at the Nyquist index n/2. Returned without the i.
template <typename R, int N>
__device__ __forceinline__ R ik_factor(int k, R inv_L) {
    const int m = k <= N / 2 ? k : k - N;
    return k == N / 2 ? R(0) : R(-2.0 * 3.14159265358979323846) * R(m) * inv_L;
}

// Inverse y then complex-to-real z of one x-plane: src holds the plane's
// half spectrum (complex, [ky][kz]), dst receives the real plane (rows of
// N + 2). deriv 2 / 3 first multiplies by the y / z derivative factor (ik).
template <typename R, int N, int BD>
__device__ __forceinline__ void inv_yz_plane(cplx<R>* __restrict__ buf, const cplx<R>* __restrict__ tw,
                                             const R* src, R* dst, int deriv, R inv_L) {
    constexpr int HS = N / 2 + 1, RL = N + 2, HALF = N / 2;
    const cplx<R>* gp = reinterpret_cast<const cplx<R>*>(src);
    for (int idx = threadIdx.x; idx < N * HS; idx += BD) {
        cplx<R> v = gload_c(gp, idx);
        if (deriv >= 2) {
            const int ky = idx / HS, kz = idx - ky * HS;
            const R d = deriv == 2 ? ik_factor<R, N>(ky, inv_L) : ik_factor<R, N>(kz, inv_L);
            v = {-v.y * d, v.x * d};
        }
        buf[idx] = v;
    }
    __syncthreads();
    fft_ct<R, N, 1, HS, 1, HS, BD, true, -1>(buf, tw);
    {
        // rows 2r and 2r+1 (half spectra A, B of two real rows) -> Z = A + iB
        constexpr int TOTAL = HALF * HS, IT = (TOTAL + BD - 1) / BD;
        cplx<R> Z[IT], Zc[IT];
        int o[IT], k_[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int item = threadIdx.x + it * BD;
            o[it] = -1;
            if (item < TOTAL) {
                const int r = item / HS, k = item - r * HS;
                const cplx<R> a = buf[(2 * r) * HS + k], b = buf[(2 * r + 1) * HS + k];
                Z[it] = {a.x - b.y, a.y + b.x};
                Zc[it] = {a.x + b.y, b.x - a.y};
                o[it] = r * (N + 1);
                k_[it] = k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < IT; ++it)
            if (o[it] >= 0) {
                const int k = k_[it];
                buf[o[it] + k] = Z[it];
                if (k > 0 && k < HALF) buf[o[it] + N - k] = Zc[it];
            }
        __syncthreads();
    }
    // z: pair rows N + 1 apart, consecutive threads on consecutive rows
    fft_ct<R, N, 1, HALF, N + 1, 1, BD, true, -1>(buf, tw);
    for (int idx = threadIdx.x; idx < HALF * N; idx += BD) {
        const int r = idx / N, z = idx - r * N;
        const cplx<R> v = buf[r * (N + 1) + z];
        gptr(dst)[(2 * r) * RL + z] = v.x;
        gptr(dst)[(2 * r + 1) * RL + z] = v.y;
    }
}

// Inverse pass along y, then complex-to-real along z, for one x-plane. With
// ik forces the block also makes the plane of each gradient grid: d/dy and
// d/dz from the potential's spectrum (read before the potential overwrites
// it in place), d/dx from the x-derivative spectrum the x pass left in the
// first gradient grid (in place).
template <typename R, int N>
__global__ void __launch_bounds__(plane_threads<N>()) k_inv_yz(const SysDesc* __restrict__ sys,
                                                              const int2* __restrict__ items,
                                                              const double* __restrict__ epart,
                                                              const double* __restrict__ bpart,
                                                              const double* __restrict__ lpart,
                                                              double* __restrict__ E_dev) {
    constexpr int RL = N + 2, BD = plane_threads<N>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* buf = tw + N;
    const cplx<R>* tw_g = reinterpret_cast<const cplx<R>*>(S.tw);
    for (int i = threadIdx.x; i < N; i += BD) tw[i] = tw_g[i];
    const long long off = (long long)wi.y * N * RL;
    R* plane = reinterpret_cast<R*>(S.grid) + off;
    if (S.ik) {  // uniform over the block
        R* g = reinterpret_cast<R*>(S.grad);
        const long long G = (long long)N * N * RL;
        inv_yz_plane<R, N, BD>(buf, tw, plane, g + G + off, 2, R(S.iky));
        __syncthreads();
        inv_yz_plane<R, N, BD>(buf, tw, plane, g + 2 * G + off, 3, R(S.ikz));
        __syncthreads();
        inv_yz_plane<R, N, BD>(buf, tw, plane, plane, 0, R(0));
        __syncthreads();
        inv_yz_plane<R, N, BD>(buf, tw, g + off, g + off, 0, R(0));
    } else {
        inv_yz_plane<R, N, BD>(buf, tw, plane, plane, 0, R(0));
    }
    // the system's energy, by the first wave of its plane-0 block: the
    // partials it sums were complete before this pass started
    if (S.fin_fft && wi.y == 0 && threadIdx.x < 64) finalize_system(S, epart, bpart, lpart, E_dev, wi.x);
}

// Pass along x for C consecutive columns c0 .. c0+cnt-1 of the flattened
// (ky, kz) index ky * (N/2+1) + kz: forward DFT, scaling by
// p_k = TS[|m|^2] Tphi[|mx|] Tphi[|my|] Tphi[|mz|] (n/L) (eq. pk) with the
// k-space energy partial
//   E_k = 1/2 sum_k p_k |b^_k|^2   (half spectrum: weight 2 off the kz = 0, N/2 planes),
// then the inverse DFT. mode 1 stops after the forward DFT, mode 2 after the
// scaling (diagnostics). Each x-row of the chunk is one contiguous run.
template <typename R, int N>
__global__ void __launch_bounds__((x_threads<R, N>())) k_fft_x(const SysDesc* __restrict__ sys,
                                                            const int4* __restrict__ items,
                                                            double* __restrict__ epart, int mode) {
    constexpr int HS = N / 2 + 1, HALF = N / 2, C = x_columns<R>(), BD = x_threads<R, N>();
    constexpr int ROW = N * HS;  // complex values per x-plane
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    const int4 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int c0 = wi.y, cnt = wi.z;
    cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* buf = tw + N;
    cplx<R>* bufx = buf + N * C;  // ik: the x-derivative of the scaled spectrum
    const bool ik = S.ik && mode == 0;
    const cplx<R>* tw_g = reinterpret_cast<const cplx<R>*>(S.tw);
    for (int i = threadIdx.x; i < N; i += BD) tw[i] = tw_g[i];
    cplx<R>* gp = reinterpret_cast<cplx<R>*>(S.grid) + c0;
    for (int idx = threadIdx.x; idx < N * C; idx += BD) {
        const int x = idx / C, l = idx - x * C;
        buf[idx] = l < cnt ? gload_c(gp, (long long)x * ROW + l) : cplx<R>{R(0), R(0)};
    }
    __syncthreads();
    fft_ct<R, N, 1, C, 1, C, BD, true, +1>(buf, tw);
    double e = 0.0;
    if (mode != 1) {
        const auto TS = gptr(reinterpret_cast<const R*>(S.TS));
        const auto Tp = gptr(reinterpret_cast<const R*>(S.Tphi));
        const auto p3 = gptr(reinterpret_cast<const R*>(S.p3));  // non-cubic box: the whole table
        const R ps = R(S.pscale);
        for (int idx = threadIdx.x; idx < N * C; idx += BD) {
            const int x = idx / C, l = idx - x * C;
            if (l >= cnt) continue;
            const int col = c0 + l;
            const int ky = col / HS, kz = col - ky * HS;
            const int mx = x <= HALF ? x : N - x;
            const int my = ky <= HALF ? ky : N - ky;
            const R p = p3 ? p3[(long long)x * ROW + col]
                           : TS[mx * mx + my * my + kz * kz] * Tp[mx] * (Tp[my] * ps) * Tp[kz];
            const cplx<R> b = buf[idx];
            const double wgt = (kz == 0 || kz == HALF) ? 1.0 : 2.0;
            e += wgt * (double)p * ((double)b.x * (double)b.x + (double)b.y * (double)b.y);
            const cplx<R> cb = {b.x * p, b.y * p};
            buf[idx] = cb;
            if (ik) {
                const R d = ik_factor<R, N>(x, R(S.ikx));
                bufx[idx] = {-cb.y * d, cb.x * d};
            }
        }
        __syncthreads();
        if (mode == 0) fft_ct<R, N, 1, C, 1, C, BD, true, -1>(buf, tw);
        if (ik) fft_ct<R, N, 1, C, 1, C, BD, true, -1>(bufx, tw);
    }
    for (int idx = threadIdx.x; idx < N * C; idx += BD) {
        const int x = idx / C, l = idx - x * C;
        if (l < cnt) gstore_c(gp, (long long)x * ROW + l, buf[idx]);
    }
    if (ik) {
        cplx<R>* gx = reinterpret_cast<cplx<R>*>(S.grad) + c0;
        for (int idx = threadIdx.x; idx < N * C; idx += BD) {
            const int x = idx / C, l = idx - x * C;
            if (l < cnt) gstore_c(gx, (long long)x * ROW + l, bufx[idx]);
        }
    }
    const double tot = block_sum(e, red);
    if (threadIdx.x == 0) epart[blockIdx.x] = 0.5 * tot;
}

// The same Stockham stages on one line held in a thread's registers: element
// idx of the line is a[idx], and every butterfly, twiddle and store index is
// that of st_stage with one line of element stride 1, so the results are
// those of the LDS stages bit for bit.
template <typename R, int N, int NS, int DIR>
__device__ __forceinline__ void reg_fft(cplx<R> (&a)[N], const cplx<R>* __restrict__ tw) {
    if constexpr (NS < N) {
        constexpr int M = N / NS;
        constexpr int RAD = M % 4 == 0 ? 4 : (M % 2 == 0 ? 2 : 3);
        constexpr int NB = N / RAD;
        constexpr int SPAN = N / (NS * RAD);
        cplx<R> b[N];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int jm = j % NS;
            cplx<R> v[RAD];
#pragma unroll
            for (int k = 0; k < RAD; ++k) {
                cplx<R> x = a[j + k * NB];
                if constexpr (NS > 1) {
                    if (k > 0) {
                        cplx<R> w = tw[k * jm * SPAN];
                        if constexpr (DIR < 0) w.y = -w.y;
                        x = cmul(x, w);
                    }
                }
                v[k] = x;
            }
            Bfly<R, RAD>::run(v, DIR);
#pragma unroll
            for (int k = 0; k < RAD; ++k) b[(j - jm) * RAD + jm + k * NS] = v[k];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) a[i] = b[i];
        reg_fft<R, N, NS * RAD, DIR>(a, tw);
    }
}

// x pass with one column per thread, its N values in registers (no LDS
// stages, no barriers): forward DFT along x, scaling by p_k with the energy
// partial, inverse DFT, as k_fft_x and with its arithmetic. One wave per
// chunk of up to kXRegColumns consecutive flattened (ky, kz) columns; each
// x-row of the chunk is one contiguous run. Systems with AD forces, FP32
// grids of 40 to 64 points (fft_x_in_registers).
template <typename R, int N>
__global__ void __launch_bounds__(kXRegColumns) k_fft_x_reg(const SysDesc* __restrict__ sys,
                                                           const int4* __restrict__ items,
                                                           double* __restrict__ epart, int mode) {
    constexpr int HS = N / 2 + 1, HALF = N / 2, ROW = N * HS;
    __shared__ cplx<R> tw[N];
    __shared__ double red[1];
    const int4 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    const int c0 = wi.y, cnt = wi.z, l = threadIdx.x;
    const cplx<R>* tw_g = reinterpret_cast<const cplx<R>*>(S.tw);
    for (int i = threadIdx.x; i < N; i += kXRegColumns) tw[i] = tw_g[i];
    __syncthreads();
    double e = 0.0;
    if (l < cnt) {
        cplx<R>* gp = reinterpret_cast<cplx<R>*>(S.grid) + c0 + l;
        cplx<R> a[N];
#pragma unroll
        for (int x = 0; x < N; ++x) a[x] = gload_c(gp, (long long)x * ROW);
        reg_fft<R, N, 1, +1>(a, tw);
        if (mode != 1) {
            const auto TS = gptr(reinterpret_cast<const R*>(S.TS));
            const auto Tp = gptr(reinterpret_cast<const R*>(S.Tphi));
            const auto p3 = gptr(reinterpret_cast<const R*>(S.p3));  // non-cubic box: the whole table
            const R ps = R(S.pscale);
            const int col = c0 + l;
            const int ky = col / HS, kz = col - ky * HS;
            const int my = ky <= HALF ? ky : N - ky;
            const double wgt = (kz == 0 || kz == HALF) ? 1.0 : 2.0;
            const R typs = Tp[my] * ps, tkz = Tp[kz];
#pragma unroll
            for (int x = 0; x < N; ++x) {
                const int mx = x <= HALF ? x : N - x;
                // k_fft_x's product, in its order
                const R p = p3 ? p3[(long long)x * ROW + col] : TS[mx * mx + my * my + kz * kz] * Tp[mx] * typs * tkz;
                const cplx<R> b = a[x];
                e += wgt * (double)p * ((double)b.x * (double)b.x + (double)b.y * (double)b.y);
                a[x] = {b.x * p, b.y * p};
            }
            if (mode == 0) reg_fft<R, N, 1, -1>(a, tw);
        }
#pragma unroll
        for (int x = 0; x < N; ++x) gstore_c(gp, (long long)x * ROW, a[x]);
    }
    const double tot = block_sum(e, red);
    if (threadIdx.x == 0) epart[blockIdx.x] = 0.5 * tot;
}

// ---------------------------------------------------------------------------
// Whole 3D transform of one system in one block, for grids whose half
// spectrum fits in LDS (FP32 n <= 32, FP64 n <= 24): halo fold, forward z, y
// and x, scaling with the energy, inverse x, y and z, one write of the real
// grid. The passes and their arithmetic are those of the three-kernel path;
// planes sit at buf[x * N (N/2+1)] in the same layouts.

template <int N, typename R> constexpr bool fused_fits() {
    return (N + N * N * (N / 2 + 1)) * 2 * (int)sizeof(R) + (N + 1) * (int)sizeof(CoverTab) <= 160 * 1024;
}
constexpr int kFusedThreads = 1024;

template <typename R, int N, int BD>
__device__ __forceinline__ void fold_volume(R* __restrict__ bufr, const R* __restrict__ tiles, const SysDesc& S,
                                            const CoverTab* __restrict__ tab) {
    constexpr int NV = N * N * N, PG = 2, PL2 = 2 * N * (N / 2 + 1);
    const int t1 = S.tiles1, E = S.E, EE = E * E, E3 = EE * E;
    for (int p0 = 0; p0 < NV; p0 += PG * BD) {
        R acc[PG];
        int xs[PG], ys[PG], zs[PG];
#pragma unroll
        for (int q = 0; q < PG; ++q) {
            const int idx = p0 + q * BD + (int)threadIdx.x;
            const int i = idx < NV ? idx : 0;
            xs[q] = i / (N * N);
            ys[q] = (i / N) % N;
            zs[q] = i % N;
            acc[q] = R(0);
        }
#pragma unroll 1
        for (int a = 0; a < 3; ++a) {
            R v[PG][3][3];
#pragma unroll
            for (int q = 0; q < PG; ++q) {
                const int idx = p0 + q * BD + (int)threadIdx.x;
                const CoverTab cx = tab[xs[q]], cy = tab[ys[q]], cz = tab[zs[q]];
                const bool okx = ((NV % (PG * BD) == 0) || idx < NV) && a < cx.cnt;
                const R* ta = tiles + (okx ? cx.bin[a] * t1 * t1 * E3 + cx.off[a] * EE : 0);
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        v[q][b][c] = (okx && b < cy.cnt && c < cz.cnt)
                                         ? ta[(cy.bin[b] * t1 + cz.bin[c]) * E3 + cy.off[b] * E + cz.off[c]]
                                         : R(0);
            }
#pragma unroll
            for (int q = 0; q < PG; ++q)
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[q] += v[q][b][c];
        }
#pragma unroll
        for (int q = 0; q < PG; ++q) {
            const int idx = p0 + q * BD + (int)threadIdx.x;
            if ((NV % (PG * BD) == 0) || idx < NV) {
                const int y = ys[q], z = zs[q];
                bufr[xs[q] * PL2 + 2 * ((y >> 1) * N + z) + (y & 1)] = acc[q];
            }
        }
    }
}

// The same fold streamed tile by tile: the block adds each bin tile's E^3
// entries (contiguous in HBM, loaded row by row by 32-lane groups) into the
// zeroed LDS grid, one tile after another. A tile covers distinct grid points
// when E <= N, so the adds of one tile never collide; the caller uses
// fold_volume otherwise.
template <typename R, int N, int BD>
__device__ __forceinline__ void fold_stream(R* __restrict__ bufr, const R* __restrict__ tiles, const SysDesc& S) {
    constexpr int PL2 = 2 * N * (N / 2 + 1);
    const int T = S.T, t1 = S.tiles1, E = S.E, EE = E * E, E3 = EE * E;
    const int lo = -((S.P - 1) / 2);
    for (int i = threadIdx.x; i < N * PL2; i += BD) bufr[i] = R(0);
    const int c = threadIdx.x & 31;
    constexpr int rstep = BD >> 5;
    const int nb = t1 * t1 * t1;
    for (int t = 0; t < nb; ++t) {
        __syncthreads();
        const int tz = t % t1, ty = (t / t1) % t1, tx = t / (t1 * t1);
        const int ox = tx * T + lo, oy = ty * T + lo, oz = tz * T + lo;
        const R* tp = tiles + (size_t)t * E3;
        int z = oz + c;
        z += z < 0 ? N : 0;
        z -= z >= N ? N : 0;
        int r = threadIdx.x >> 5, a = r / E, b = r - a * E;
        for (; r < EE; r += rstep) {
            if (c < E) {
                int x = ox + a, y = oy + b;
                x += x < 0 ? N : 0;
                x -= x >= N ? N : 0;
                y += y < 0 ? N : 0;
                y -= y >= N ? N : 0;
                bufr[x * PL2 + 2 * ((y >> 1) * N + z) + (y & 1)] += tp[r * E + c];
            }
            b += rstep;
            while (b >= E) {
                b -= E;
                ++a;
            }
        }
    }
}

// Pair rows (2r, 2r+1) transformed as complex row r -> half spectra of the two
// real rows, in every plane (forward), or back (inverse).
template <typename R, int N, int BD, bool FWD>
__device__ __forceinline__ void untangle_all(cplx<R>* __restrict__ buf) {
    constexpr int HS = N / 2 + 1, HALF = N / 2, PL = N * HS;
    constexpr int TOTAL = N * HALF * HS, IT = (TOTAL + BD - 1) / BD;
    cplx<R> A[IT], B[IT];
    int o[IT], k_[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int item = threadIdx.x + it * BD;
        o[it] = -1;
        if (item < TOTAL) {
            const int x = item / (HALF * HS), rem = item - x * (HALF * HS);
            const int r = rem / HS, k = rem - r * HS;
            cplx<R>* pl = buf + x * PL;
            if constexpr (FWD) {
                const cplx<R> zk = pl[r * N + k];
                const cplx<R> zn = pl[r * N + (k == 0 ? 0 : N - k)];
                A[it] = {R(0.5) * (zk.x + zn.x), R(0.5) * (zk.y - zn.y)};
                B[it] = {R(0.5) * (zk.y + zn.y), -R(0.5) * (zk.x - zn.x)};
                o[it] = x * PL + (2 * r) * HS + k;
            } else {
                const cplx<R> a = pl[(2 * r) * HS + k], b = pl[(2 * r + 1) * HS + k];
                A[it] = {a.x - b.y, a.y + b.x};
                B[it] = {a.x + b.y, b.x - a.y};
                o[it] = x * PL + r * N;
                k_[it] = k;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it)
        if (o[it] >= 0) {
            if constexpr (FWD) {
                buf[o[it]] = A[it];
                buf[o[it] + HS] = B[it];
            } else {
                const int k = k_[it];
                buf[o[it] + k] = A[it];
                if (k > 0 && k < HALF) buf[o[it] + N - k] = B[it];
            }
        }
    __syncthreads();
}

template <typename R, int N>
__global__ void __launch_bounds__(kFusedThreads) k_fft3d(const SysDesc* __restrict__ sys, const int2* __restrict__ items,
                                                         double* __restrict__ epart, int from_tiles, int mode) {
    constexpr int HS = N / 2 + 1, RL = N + 2, HALF = N / 2, PL = N * HS, BD = kFusedThreads;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[16];
    const int2 wi = items[blockIdx.x];
    const SysDesc& S = sys[wi.x];
    cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
    cplx<R>* buf = tw + N;
    const cplx<R>* tw_g = reinterpret_cast<const cplx<R>*>(S.tw);
    for (int i = threadIdx.x; i < N; i += BD) tw[i] = tw_g[i];
    R* grid = reinterpret_cast<R*>(S.grid);
    if (from_tiles && S.E <= N) {
        fold_stream<R, N, BD>(reinterpret_cast<R*>(buf), reinterpret_cast<const R*>(S.tiles), S);
    } else if (from_tiles) {
        CoverTab* tab = reinterpret_cast<CoverTab*>(buf + N * PL);
        build_cover(tab, S, -((S.P - 1) / 2));
        __syncthreads();
        fold_volume<R, N, BD>(reinterpret_cast<R*>(buf), reinterpret_cast<const R*>(S.tiles), S, tab);
    } else {
        for (int idx = threadIdx.x; idx < N * HALF * N; idx += BD) {
            const int x = idx / (HALF * N), rem = idx - x * (HALF * N), r = rem / N, z = rem - r * N;
            buf[x * PL + r * N + z] = {grid[(x * N + 2 * r) * RL + z], grid[(x * N + 2 * r + 1) * RL + z]};
        }
    }
    __syncthreads();
    fft_ct2<R, N, 1, N * HALF, HALF, PL, N, 1, BD, false, +1>(buf, tw);   // z, pair rows
    untangle_all<R, N, BD, true>(buf);
    fft_ct2<R, N, 1, N * HS, HS, PL, 1, HS, BD, true, +1>(buf, tw);       // y
    fft_ct2<R, N, 1, PL, PL, 0, 1, PL, BD, true, +1>(buf, tw);            // x
    double e = 0.0;
    if (mode != 1) {
        const R* TS = reinterpret_cast<const R*>(S.TS);
        const R* Tp = reinterpret_cast<const R*>(S.Tphi);
        const R ps = R(S.pscale);
        for (int idx = threadIdx.x; idx < N * PL; idx += BD) {
            const int x = idx / PL, col = idx - x * PL;
            const int ky = col / HS, kz = col - ky * HS;
            const int mx = x <= HALF ? x : N - x;
            const int my = ky <= HALF ? ky : N - ky;
            const R p = TS[mx * mx + my * my + kz * kz] * Tp[mx] * (Tp[my] * ps) * Tp[kz];
            const cplx<R> b = buf[idx];
            const double wgt = (kz == 0 || kz == HALF) ? 1.0 : 2.0;
            e += wgt * (double)p * ((double)b.x * (double)b.x + (double)b.y * (double)b.y);
            buf[idx] = {b.x * p, b.y * p};
        }
        __syncthreads();
    }
    if (mode == 0) {
        fft_ct2<R, N, 1, PL, PL, 0, 1, PL, BD, true, -1>(buf, tw);        // x
        fft_ct2<R, N, 1, N * HS, HS, PL, 1, HS, BD, true, -1>(buf, tw);   // y
        untangle_all<R, N, BD, false>(buf);
        fft_ct2<R, N, 1, N * HALF, HALF, PL, N, 1, BD, false, -1>(buf, tw);  // z
        for (int idx = threadIdx.x; idx < N * HALF * N; idx += BD) {
            const int x = idx / (HALF * N), rem = idx - x * (HALF * N), r = rem / N, z = rem - r * N;
            const cplx<R> v = buf[x * PL + r * N + z];
            grid[(x * N + 2 * r) * RL + z] = v.x;
            grid[(x * N + 2 * r + 1) * RL + z] = v.y;
        }
    } else {
        // diagnostics: the (scaled) half spectrum in the grid's complex layout
        cplx<R>* gp = reinterpret_cast<cplx<R>*>(grid);
        for (int idx = threadIdx.x; idx < N * PL; idx += BD) gp[idx] = buf[idx];
    }
    const double tot = block_sum(e, red);
    if (threadIdx.x == 0) epart[S.col_off] = 0.5 * tot;
}

#pragma clang fp contract(fast)

// ---------------------------------------------------------------------------
// Launchers

template <typename K>
static hipError_t allow_lds(K kernel, int bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               bytes);
}

template <typename R, int N>
static hipError_t fft_n(const Launch& L, const FftGroup& G, int which, int mode, double* E_dev) {
    hipError_t e;
    if constexpr (fused_fits<N, R>()) {
        if (G.fused) {
            // one kernel for the whole transform: launched at the first pass;
            // mode packs (source 3 = real grid) x 4 + (x-pass mode)
            if (which != 0) return hipSuccess;
            const int lds = fft_fused_lds(N, L.prec);
            if ((e = allow_lds(k_fft3d<R, N>, lds)) != hipSuccess) return e;
            k_fft3d<R, N><<<G.sys_count, kFusedThreads, lds, L.stream>>>(L.sys, L.fsys + G.sys_off, L.epart,
                                                                          (mode & 3) == 3 ? 0 : 1, mode >> 2);
            return hipGetLastError();
        }
    }
    const int lds_plane = fft_plane_lds(N, L.prec);
    if (which == 0) {
        if ((e = allow_lds(k_fwd_zy<R, N>, lds_plane)) != hipSuccess) return e;
        k_fwd_zy<R, N><<<G.plane_count, plane_threads<N>(), lds_plane, L.stream>>>(L.sys, L.planes + G.plane_off,
                                                                                   (mode & 3) == 3 ? 0 : 1);
    } else if (which == 1) {
        if constexpr (sizeof(R) == 4 && N >= 40 && N <= 64) {
            if (G.xreg) {
                k_fft_x_reg<R, N><<<G.col_count, kXRegColumns, 0, L.stream>>>(L.sys, L.cols + G.col_off,
                                                                             L.epart + G.col_off, mode);
                return hipGetLastError();
            }
        }
        const int lds = fft_x_lds(N, L.prec, L.any_ik);
        if ((e = allow_lds(k_fft_x<R, N>, lds)) != hipSuccess) return e;
        k_fft_x<R, N><<<G.col_count, x_threads<R, N>(), lds, L.stream>>>(L.sys, L.cols + G.col_off,
                                                                         L.epart + G.col_off, mode);
    } else {
        if ((e = allow_lds(k_inv_yz<R, N>, lds_plane)) != hipSuccess) return e;
        k_inv_yz<R, N><<<G.plane_count, plane_threads<N>(), lds_plane, L.stream>>>(
            L.sys, L.planes + G.plane_off, L.epart, L.bpart, L.lpart, E_dev);
    }
    return hipGetLastError();
}

template <typename R>
static hipError_t fft_r(const Launch& L, const FftGroup& G, int which, int mode, double* E_dev) {
    switch (G.n) {
        case 8: return fft_n<R, 8>(L, G, which, mode, E_dev);
        case 12: return fft_n<R, 12>(L, G, which, mode, E_dev);
        case 16: return fft_n<R, 16>(L, G, which, mode, E_dev);
        case 18: return fft_n<R, 18>(L, G, which, mode, E_dev);
        case 24: return fft_n<R, 24>(L, G, which, mode, E_dev);
        case 32: return fft_n<R, 32>(L, G, which, mode, E_dev);
        case 36: return fft_n<R, 36>(L, G, which, mode, E_dev);
        case 48: return fft_n<R, 48>(L, G, which, mode, E_dev);
        case 54: return fft_n<R, 54>(L, G, which, mode, E_dev);
        case 64: return fft_n<R, 64>(L, G, which, mode, E_dev);
        case 72: return fft_n<R, 72>(L, G, which, mode, E_dev);
        case 96: return fft_n<R, 96>(L, G, which, mode, E_dev);
        case 108: return fft_n<R, 108>(L, G, which, mode, E_dev);
        case 128: return fft_n<R, 128>(L, G, which, mode, E_dev);
        case 144: return fft_n<R, 144>(L, G, which, mode, E_dev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fft(const Launch& L, const FftGroup& G, int which, int mode, double* E_dev) {
    return L.prec == 64 ? fft_r<double>(L, G, which, mode, E_dev) : fft_r<float>(L, G, which, mode, E_dev);
}

}  // namespace esp
