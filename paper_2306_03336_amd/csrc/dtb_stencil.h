// dtb_stencil.h -- the j2d5pt update of one cell, shared by the kernels.
//
// Listing 1 of Zhang et al., GPGPU '23: w*W + e*E + s*S + c*C + n*N with
// W = (i, j-1), E = (i, j+1), S = (i-1, j), N = (i+1, j).  FMA = false rounds
// every product and sums left to right in the printed order W, E, S, C, N;
// FMA = true runs the same chain as one multiply and four fused
// multiply-adds.  Everything is built with -ffp-contract=off, so nothing is
// fused unless written here.
#pragma once
#include <hip/hip_runtime.h>

namespace dtb {

// Fused multiply-add in the precision of the operands (v_fma_f32 for float,
// v_fma_f64 for double; never a float promoted to double).
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
struct Coef {
    T c, n, s, e, w;
};

template <typename T>
__device__ __forceinline__ Coef<T> load_coef(const double* k)
{
    return Coef<T>{(T)k[0], (T)k[1], (T)k[2], (T)k[3], (T)k[4]};
}

template <bool FMA, typename T>
__device__ __forceinline__ T j2d5pt(T W, T E, T S, T C, T N, const Coef<T>& k)
{
    if constexpr (FMA) {
        T acc = k.w * W;
        acc = fma_t(k.e, E, acc);
        acc = fma_t(k.s, S, acc);
        acc = fma_t(k.c, C, acc);
        acc = fma_t(k.n, N, acc);
        return acc;
    } else {
        T acc = k.w * W;
        acc = acc + k.e * E;
        acc = acc + k.s * S;
        acc = acc + k.c * C;
        acc = acc + k.n * N;
        return acc;
    }
}

// ---- j2d9pt: the 3 x 3 box.  Nine weights in row-major order of the block
// -- rows i-1, i, i+1 (S to N), each west to east: (sw, s, se, w, c, e, nw, n,
// ne) -- and the products summed in that order.  The paper presents j2d5pt as
// a case study of the method; the box is the next shape in the same
// framework, and this order is the library's reading.
template <typename T>
struct Coef9 {
    T k[9];
};

template <typename T>
__device__ __forceinline__ Coef9<T> load_coef9(const double* k)
{
    Coef9<T> c;
#pragma unroll
    for (int q = 0; q < 9; ++q) c.k[q] = (T)k[q];
    return c;
}

// a[] holds the nine neighbours in the weights' order.
template <bool FMA, typename T>
__device__ __forceinline__ T j2d9pt(const T (&a)[9], const Coef9<T>& w)
{
    T acc = w.k[0] * a[0];
#pragma unroll
    for (int q = 1; q < 9; ++q) {
        if constexpr (FMA) acc = fma_t(w.k[q], a[q], acc);
        else acc = acc + w.k[q] * a[q];
    }
    return acc;
}

}  // namespace dtb
