// Device-side building blocks shared by the single-system kernels
// (pb_kernels.hip) and the batched kernels (pb_batch.hip): packed source
// entries, precision-specific primitives, deterministic reductions and the
// per-tile pair loops.  Internal; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

#include "pb_kernels.h"

namespace pbk {
namespace dev {

constexpr double INV_4PI = 0.079577471545947667884441881686257181;
constexpr double FAR_SRC = 2.0e6;   // padded sources, weight 0
constexpr double FAR_TGT = -2.0e6;  // padded targets, never written back

template <typename T>
struct alignas(8 * sizeof(T)) Src8 {
    T x, y, z, w, mx, my, mz, pad;
};

// ---- precision-specific primitives ---------------------------------------

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt(x); }

// exp(-t) for t >= 0
__device__ __forceinline__ float exp_neg(float t)
{
    return __builtin_amdgcn_exp2f(t * -1.44269504088896340736f);
}
__device__ __forceinline__ double exp_neg(double t) { return exp(-t); }

template <typename T>
struct Coef {
    T eps, epsm1, ieps, iepsm1, kappa, k2;
    __device__ explicit Coef(const PairParams &p)
        : eps(T(p.eps)), epsm1(T(p.eps - 1.0)), ieps(T(1.0 / p.eps)),
          iepsm1(T(1.0 / p.eps - 1.0)), kappa(T(p.kappa)), k2(T(p.kappa * p.kappa)) {}
};

// Sum of per-tile partials.  FP64: plain.  FP32: compensated (Knuth's
// TwoSum), so the error of the long sum stays at the size of one tile.
template <typename T>
struct Acc;
template <>
struct Acc<double> {
    double s = 0.0;
    __device__ void add(double v) { s += v; }
    __device__ double value() const { return s; }
};
template <>
struct Acc<float> {
    float hi = 0.f, lo = 0.f;
    __device__ void add(float v)
    {
        float s = hi + v;
        float bb = s - hi;
        float err = (hi - (s - bb)) + (v - bb);
        hi = s;
        lo += err;
    }
    __device__ double value() const { return double(hi) + double(lo); }
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block; valid in thread 0.  sh holds blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k)
            r += sh[k];
    }
    return r;
}

template <typename T, bool TRANS, bool DIAG>
__device__ __forceinline__ void sweep_tile(const Src8<T> *sh, int self, T xi, T yi, T zi,
                                           T nxi, T nyi, T nzi, const Coef<T> &cf, T &accP,
                                           T &accQ)
{
#pragma unroll 2
    for (int jj = 0; jj < TILE; ++jj) {
        const Src8<T> s = sh[jj];
        const T dx = xi - s.x, dy = yi - s.y, dz = zi - s.z;
        const T r2 = dx * dx + dy * dy + dz * dz;
        T ir = rsqrt_t(r2);
        if (DIAG)
            ir = (jj == self) ? T(0) : ir;   // j = i omitted (eqs. eqbim_5/6)
        const T ir2 = ir * ir;
        const T u = ir2 * ir;
        const T kr = cf.kappa * (r2 * ir);
        const T e = exp_neg(kr);
        const T em1 = e - T(1);
        const T tm1 = fma(kr, e, em1);
        const T cxd = nxi * dx + nyi * dy + nzi * dz;
        const T md = s.mx * dx + s.my * dy + s.mz * dz;
        const T nm = nxi * s.mx + nyi * s.my + nzi * s.mz;
        const T g2 = fma(cf.eps, tm1, cf.epsm1);
        const T g3 = fma(cf.ieps, tm1, cf.iepsm1);
        const T h = fma(tm1, T(3) * ir2, cf.k2 * e);
        const T cP = TRANS ? -g3 : g2;
        const T cQ = TRANS ? g2 : -g3;
        accP = fma(-em1, ir * s.w, accP);
        accP = fma(cP * md, u, accP);
        const T inner = fma(md, h, cQ * s.w);
        accQ = fma(u, fma(-cxd, inner, tm1 * nm), accQ);
    }
}

// FP32 forward sweep in reduced form.  Lengths are in units of 1/kappa
// (SCALED, kappa > 0) or plain (kappa = 0).  Stream entries (mode 2):
//   (x, y, z, w1 = (1 - 1/eps) a psi, m = -3 a phi n, w2n = -a psi / eps),
// targets keep n_i and -n_i/3 in registers, and the separation is taken as
// d = x_j - x_i.  With md3 = m.d (= 3 a phi n_j.(x_i - x_j)),
// b = (tm1 + 1 - 1/eps)/3 and h3 = tm1/r^2 + kappa^2 e/3:
//   row 1 / eps: sum_j [(e-1) w2n / r + b md3 u]
//   row 2:       sum_j u [tm1 (-n_i/3).m + (n_i.d) (md3 h3 + w1 + tm1 w2n)]
// which is the generic kernel's algebra with two multiplies folded into the
// stream.  Scaling lengths by kappa multiplies row 1 by kappa^2 and row 2 by
// kappa^3 (applied by the caller) and makes kappa r the distance itself.
// The signs are placed so that every fused multiply-add accumulates into a
// dead register with no operand negated.  35 VALU operations per pair (36
// unscaled); TPT targets per thread share every LDS read.
struct CoefF32 {
    float kappa, kexp, c13, k23;
};

template <int TPT, int DSLOT, bool SCALED>
__device__ __forceinline__ void sweep_f32(const Src8<float> *sh, const float (&tg)[TPT][9],
                                          const CoefF32 &cf, float (&P)[TPT], float (&Q)[TPT])
{
#pragma unroll 2
    for (int jj = 0; jj < TILE; ++jj) {
        const Src8<float> s = sh[jj];
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            const float dx = s.x - tg[t][0], dy = s.y - tg[t][1], dz = s.z - tg[t][2];
            const float r2 = dx * dx + dy * dy + dz * dz;
            float ir = __builtin_amdgcn_rsqf(r2);
            if (DSLOT == t)
                ir = (jj == (int)threadIdx.x) ? 0.f : ir;   // j = i omitted
            const float ir2 = ir * ir;
            const float u = ir2 * ir;
            const float r = r2 * ir;
            const float kr = SCALED ? r : cf.kappa * r;
            const float e = __builtin_amdgcn_exp2f(cf.kexp * r);
            const float em1 = e - 1.f;
            P[t] = fmaf(em1, ir * s.pad, P[t]);
            const float tm1 = fmaf(kr, e, em1);
            const float cxd = tg[t][3] * dx + tg[t][4] * dy + tg[t][5] * dz;
            const float md3 = s.mx * dx + s.my * dy + s.mz * dz;
            const float nm = tg[t][6] * s.mx + tg[t][7] * s.my + tg[t][8] * s.mz;
            const float b = fmaf(tm1, 0.333333343f, cf.c13);
            P[t] = fmaf(b * md3, u, P[t]);
            const float h3 = fmaf(tm1, ir2, cf.k23 * e);
            const float cqw = fmaf(tm1, s.pad, s.w);
            const float inner = fmaf(md3, h3, cqw);
            Q[t] = fmaf(u, fmaf(cxd, inner, tm1 * nm), Q[t]);
        }
    }
}


}  // namespace dev
}  // namespace pbk
