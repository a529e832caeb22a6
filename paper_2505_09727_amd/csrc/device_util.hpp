// Device helpers shared by the pipeline kernels (kernels.hip) and the 3D FFT
// kernels (fft.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace esp {

template <typename R> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

template <typename R> struct cplx { R x, y; };

// Global-memory views of the descriptors' pointers (which are generic):
// accesses through them compile to global_* instructions, which count only on
// the vector-memory counter, where flat_* accesses count on the LDS counter
// too, so that every wait for an LDS result would also wait for them.
template <typename T> __device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T> __device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
// Element k of a global array of complex values, loaded / stored.
template <typename R>
__device__ __forceinline__ cplx<R> gload_c(const cplx<R>* p, long long k) {
    typedef R e2 __attribute__((ext_vector_type(2)));
    const e2 v = gptr(reinterpret_cast<const e2*>(p))[k];
    return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void gstore_c(cplx<R>* p, long long k, cplx<R> v) {
    typedef R e2 __attribute__((ext_vector_type(2)));
    e2 w;
    w.x = v.x;
    w.y = v.y;
    gptr(reinterpret_cast<e2*>(p))[k] = w;
}
// Element k of a global array of 4-vectors.
template <typename R>
__device__ __forceinline__ typename Vec4<R>::type gload4(const void* p, long long k) {
    typedef R e4 __attribute__((ext_vector_type(4)));
    const e4 x = gptr(static_cast<const e4*>(p))[k];
    typename Vec4<R>::type v;
    v.x = x.x;
    v.y = x.y;
    v.z = x.z;
    v.w = x.w;
    return v;
}

// FFT arithmetic is kept free of fused multiply-adds, so every butterfly
// rounds the same way whatever code the compiler schedules around it.
#pragma clang fp contract(off)

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---------------------------------------------------------------------------
// Small DFT butterflies, sign s: y_k = sum_m v_m exp(s 2 pi i m k / RAD)
template <typename R, int RAD> struct Bfly;

template <typename R> struct Bfly<R, 2> {
    __device__ __forceinline__ static void run(cplx<R>* v, int) {
        const cplx<R> a = v[0], b = v[1];
        v[0] = {a.x + b.x, a.y + b.y};
        v[1] = {a.x - b.x, a.y - b.y};
    }
};

template <typename R> struct Bfly<R, 3> {
    __device__ __forceinline__ static void run(cplx<R>* v, int s) {
        const R h = R(0.86602540378443864676) * R(s);
        const cplx<R> a = v[0], b = v[1], c = v[2];
        const cplx<R> t1 = {b.x + c.x, b.y + c.y};
        const cplx<R> t2 = {a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y};
        const cplx<R> t3 = {h * (b.x - c.x), h * (b.y - c.y)};
        v[0] = {a.x + t1.x, a.y + t1.y};
        v[1] = {t2.x - t3.y, t2.y + t3.x};
        v[2] = {t2.x + t3.y, t2.y - t3.x};
    }
};

template <typename R> struct Bfly<R, 4> {
    __device__ __forceinline__ static void run(cplx<R>* v, int s) {
        const cplx<R> a = v[0], b = v[1], c = v[2], d = v[3];
        const cplx<R> t0 = {a.x + c.x, a.y + c.y}, t1 = {a.x - c.x, a.y - c.y};
        const cplx<R> t2 = {b.x + d.x, b.y + d.y}, t3 = {b.x - d.x, b.y - d.y};
        const cplx<R> it3 = s > 0 ? cplx<R>{-t3.y, t3.x} : cplx<R>{t3.y, -t3.x};
        v[0] = {t0.x + t2.x, t0.y + t2.y};
        v[2] = {t0.x - t2.x, t0.y - t2.y};
        v[1] = {t1.x + it3.x, t1.y + it3.y};
        v[3] = {t1.x - it3.x, t1.y - it3.y};
    }
};

#pragma clang fp contract(fast)

// ---------------------------------------------------------------------------
// Deterministic block sum of a double (fixed tree; blockDim a power of two).
// Energy of one system, E = E_k - S(0)/2 sum q^2 (plus (1/2) sum q u^l with
// the local part), and the charge sums, by the 64 lanes of one wave (all
// active) in a fixed order, so the result does not depend on the kernel or
// block that runs it. Written to S.out[0..3] and E_dev[sys] (if non-null).
__device__ inline void finalize_system(const SysDesc& S, const double* __restrict__ epart,
                                       const double* __restrict__ bpart, const double* __restrict__ lpart,
                                       double* __restrict__ E_dev, int sys) {
    const int lane = threadIdx.x & 63;
    double ek = 0.0, sq = 0.0, sa = 0.0, s2 = 0.0;
    for (int i = lane; i < S.ncol; i += 64) ek += epart[S.col_off + i];
    if (S.local)
        for (int i = lane; i < S.nlitem; i += 64) ek += 0.5 * lpart[S.litem_off + i];
    for (int i = lane; i < S.npitem; i += 64) {
        sq += bpart[4 * (S.pitem_off + i) + 0];
        sa += bpart[4 * (S.pitem_off + i) + 1];
        s2 += bpart[4 * (S.pitem_off + i) + 2];
    }
    for (int off = 32; off > 0; off >>= 1) {
        ek += __shfl_down(ek, off, 64);
        sq += __shfl_down(sq, off, 64);
        sa += __shfl_down(sa, off, 64);
        s2 += __shfl_down(s2, off, 64);
    }
    if (lane == 0) {
        const double E = ek - 0.5 * S.s0 * s2;
        S.out[0] = E;
        S.out[1] = sq;
        S.out[2] = sa;
        S.out[3] = s2;
        if (E_dev) E_dev[sys] = E;
    }
}

__device__ inline double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t += red[w];
    return t;  // valid in thread 0
}

__device__ inline double block_max(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) t = fmax(t, red[w]);
    return t;  // valid in thread 0
}

// Block reduction of three sums and one maximum (fixed tree, so the result
// does not depend on timing; blockDim a multiple of 64, at most 1024).
// red holds 64 doubles. Results valid in thread 0.
__device__ inline void block_sum3_max(double& a, double& b, double& c, double& m, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
        m = fmax(m, __shfl_down(m, off, 64));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[4 * wid + 0] = a;
        red[4 * wid + 1] = b;
        red[4 * wid + 2] = c;
        red[4 * wid + 3] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        a = b = c = m = 0.0;
        for (int w = 0; w < nw; ++w) {
            a += red[4 * w + 0];
            b += red[4 * w + 1];
            c += red[4 * w + 2];
            m = fmax(m, red[4 * w + 3]);
        }
    }
}

// The (bin, offset) pairs of one axis whose tiles cover grid index g: bin t's
// tile starts at t*T + lo (mod n) and spans E points, so g lies at offset
// o = (g - lo - t*T) mod n (and o + n, o + 2n, ... while below E).
__device__ __forceinline__ int covering(int g, int lo, int T, int t1, int n, int E, int* tb, int* off) {
    int gm = (g - lo) % n;
    if (gm < 0) gm += n;
    const int tf = gm / T;
    const int o1 = gm - tf * T;
    int c = 0;
    for (int k = 0; o1 + k * T < E && c < 4; ++k) {
        int tt = (tf - k) % t1;
        if (tt < 0) tt += t1;
        tb[c] = tt;
        off[c] = o1 + k * T;
        ++c;
    }
    return c;
}

// Covering lists of all n indices of an axis, built once per block in LDS.
struct CoverTab {
    int cnt;
    int bin[4];
    int off[4];
};

__device__ __forceinline__ void build_cover(CoverTab* tab, const SysDesc& S, int lo) {
    // written in place (a private CoverTab indexed at run time would live in
    // scratch memory)
    for (int g = threadIdx.x; g < S.n; g += blockDim.x)
        tab[g].cnt = covering(g, lo, S.T, S.tiles1, S.n, S.E, tab[g].bin, tab[g].off);
}

// b_l for one grid point, summed over every bin tile that covers it.
template <typename R>
__device__ __forceinline__ R fold_point(const R* __restrict__ tiles, const SysDesc& S, const CoverTab& cx,
                                        const CoverTab& cy, const CoverTab& cz) {
    const int t1 = S.tiles1, E = S.E;
    const long long E3 = (long long)E * E * E;
    R acc = R(0);
    for (int a = 0; a < cx.cnt; ++a)
        for (int b = 0; b < cy.cnt; ++b) {
            const long long base = ((long long)cx.bin[a] * t1 + cy.bin[b]) * t1 * E3 +
                                   ((long long)cx.off[a] * E + cy.off[b]) * E;
            for (int c = 0; c < cz.cnt; ++c) acc += tiles[base + (long long)cz.bin[c] * E3 + cz.off[c]];
        }
    return acc;
}

}  // namespace esp
