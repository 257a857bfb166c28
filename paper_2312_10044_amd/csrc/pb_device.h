// Device-side building blocks shared by the single-system kernels
// (pb_kernels.hip) and the batched kernels (pb_batch.hip): packed source
// entries, precision-specific primitives, deterministic reductions and the
// per-tile pair loops.  Internal; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

#include "pb_fp64math.h"
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

// 1/sqrt(x), x > 0 (FP64: the hardware estimate refined by fm::rsqrt_refine,
// within 1 ulp)
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x)
{
    return fm::rsqrt_refine(x, __builtin_amdgcn_rsq(x));
}

// exp(-t) for t >= 0.  FP64 keeps the library exp here: the table lookup of
// fm::exp_neg_pair is a memory access, which the pairwise sweep hides behind
// eight pairs in flight per lane but the one-pair-per-step charge and
// per-target loops do not (measured no faster).
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

// Targets per thread of the pairwise FP32 sweep (blocks of TILE / SYM_TT),
// and the waves per SIMD its launch bounds ask for: 4 (the compiler then
// keeps both targets' pair heads in registers; forcing 5, at most 96 VGPRs,
// measured 0.4 % slower, and 6 waves 4 % slower).
constexpr int SYM_TT = 2;
constexpr int SYM_NT = TILE / SYM_TT;
constexpr int SYM_MIN_WAVES = 4;

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


// ---- pairwise FP32 sweep: each unordered pair evaluated once ----------------
//
// For a pair (i, j) the distance, exp(-kappa r), tm1, b and h3 are symmetric,
// so one evaluation yields both the contribution of source j to row i and of
// source i to row j.  Every collocation point is a target and a source; the
// packed entry carries both roles (reduced form, lengths in units of 1/kappa
// when kappa > 0): position, w1 = (1 - 1/eps) a psi / sigma, w2n = -a psi /
// (eps sigma), sn = -n and nu = 3 a phi.  The moment m = -3 a phi n of the
// reduced form is parallel to the normal, so every product with m is a
// product with the normal times nu: m_j.d = nu_j (sn_j.d), n_i.m_j =
// nu_j (n_i.sn_j), and the three dot products of a pair (n_i.d, sn_j.d,
// n_i.sn_j) serve both directions.
struct alignas(16) Src12 {
    float x, y, z, w1;
    float w2n, nx, ny, nz;
    float nu, res0, res1, res2;
};

// The thread's own point: position, n_i (the stream holds -n) and its
// source weights w1, w2n and nu.
struct OwnF32 {
    float x, y, z;
    float nx, ny, nz;
    float w1, w2n, nu;
    float mx, my, mz;   // -n / 3: n_i.sn_j / -3 in one dot product
};

__device__ __forceinline__ OwnF32 own_point(const Src12 &e)
{
    OwnF32 o;
    o.x = e.x;
    o.y = e.y;
    o.z = e.z;
    o.nx = -e.nx;
    o.ny = -e.ny;
    o.nz = -e.nz;
    o.w1 = e.w1;
    o.w2n = e.w2n;
    o.nu = e.nu;
    o.mx = e.nx * 0.333333343f;
    o.my = e.ny * 0.333333343f;
    o.mz = e.nz * 0.333333343f;
    return o;
}

// A source tile in LDS, 36 bytes per entry in three aligned arrays (the
// entry's 9 used values), read back as two 16-byte and one 4-byte broadcast.
struct SrcTileF32 {
    float4 a[TILE];   // x, y, z, w1
    float4 b[TILE];   // w2n, sn
    float c[TILE];    // nu
    __device__ __forceinline__ void put(int t, const Src12 &e)
    {
        a[t] = make_float4(e.x, e.y, e.z, e.w1);
        b[t] = make_float4(e.w2n, e.nx, e.ny, e.nz);
        c[t] = e.nu;
    }
    __device__ __forceinline__ Src12 get(int j) const
    {
        const float4 u = a[j], v = b[j];
        Src12 e;
        e.x = u.x;
        e.y = u.y;
        e.z = u.z;
        e.w1 = u.w;
        e.w2n = v.x;
        e.nx = v.y;
        e.ny = v.z;
        e.nz = v.w;
        e.nu = c[j];
        e.res0 = e.res1 = e.res2 = 0.f;
        return e;
    }
};

// Lane exchanges by DPP.  CTRL is one of the in-row permutations (row mirror
// 0x140, half-row mirror 0x141, quad permutations 0x1B and 0xB1) with every
// row and bank enabled, so each lane reads a valid lane and no lane keeps its
// old value.  FP32: the old value 0 lets the compiler fold the exchange into
// the add that consumes it (one DPP add).  FP64 adds take no DPP operand, so
// the two halves of a double move by mov_dpp, whose undefined old value
// spares the register initialisation an explicit one costs.
template <int CTRL>
__device__ __forceinline__ void dpp_ctrl_check()
{
    static_assert(CTRL == 0x140 || CTRL == 0x141 || CTRL == 0x1B || CTRL == 0xB1,
                  "only full in-row permutations");
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    dpp_ctrl_check<CTRL>();
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    dpp_ctrl_check<CTRL>();
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) { return dpp_f<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) { return dpp_d<CTRL>(v); }

// Reduce-scatter over the 16 lanes of each row, in two calls: the values
// v0..v3 of sources k and k+2 of a group of four first meet at stage 1
// (row mirror, lane xor 15: lanes with bit 3 set keep the second half), so
// that stage is done as soon as both sources are evaluated.  The finishing
// stages pair lanes by the half-row mirror (xor 7) and the quad permutations
// xor 3 and xor 1; the masks 15, 7, 3, 1 span all 16 lane offsets.  On
// return lane l holds the sum over its row of value (l >> 1) & 7, where value
// 2k + c is component c of source k.
template <typename T>
__device__ __forceinline__ void rs_stage1(T a0, T a1, T b0, T b1, int lane, T &s0, T &s1)
{
    const bool b3 = lane & 8;
    s0 = (b3 ? b0 : a0) + dpp_t<0x140>(b3 ? a0 : b0);
    s1 = (b3 ? b1 : a1) + dpp_t<0x140>(b3 ? a1 : b1);
}

template <typename T>
__device__ __forceinline__ T rs_finish(const T (&a)[4], int lane)
{
    const bool b2 = lane & 4, b1 = lane & 2;
    T b[2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
        b[k] = (b2 ? a[k + 2] : a[k]) + dpp_t<0x141>(b2 ? a[k] : a[k + 2]);
    const T c = (b1 ? b[1] : b[0]) + dpp_t<0x1B>(b1 ? b[0] : b[1]);
    return c + dpp_t<0xB1>(c);
}

// One pair, forward direction only (source s on the own point o); with DIAG the
// pair is dropped when `skip` (ir = 0 zeroes every term).  With d = x_j - x_i,
// A = n_i.d, B = sn_j.d, C = n_i.sn_j, t3n = -tm1/3 and
// b = (tm1 + 1 - 1/eps)/3 = c13 - t3n (the own point carries m = -n_i/3, so
// t3n C = tm1 (m.sn_j) and t3n itself is never formed):
//   row 1 / eps += (e-1) w2n_j / r + b nu_j B u
//   row 2       += u [A (nu_j B h3 + tm1 w2n_j + w1_j) + t3n C nu_j]
template <bool SCALED, bool DIAG>
__device__ __forceinline__ void pair_fwd(const Src12 &s, const OwnF32 &o, const CoefF32 &cf,
                                         bool skip, float &P, float &Q)
{
    const float dx = s.x - o.x, dy = s.y - o.y, dz = s.z - o.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    float ir = __builtin_amdgcn_rsqf(r2);
    if (DIAG)
        ir = skip ? 0.f : ir;
    const float ir2 = ir * ir;
    const float u = ir2 * ir;
    const float r = r2 * ir;
    const float kr = SCALED ? r : cf.kappa * r;
    const float e = __builtin_amdgcn_exp2f(cf.kexp * r);
    const float em1 = e - 1.f;
    P = fmaf(em1 * ir, s.w2n, P);
    const float tm1 = fmaf(kr, e, em1);
    const float b = fmaf(tm1, 0.333333343f, cf.c13);   // c13 - t3n
    const float A = o.nx * dx + o.ny * dy + o.nz * dz;
    const float B = s.nx * dx + s.ny * dy + s.nz * dz;
    const float C3 = o.mx * s.nx + o.my * s.ny + o.mz * s.nz;   // -C / 3
    const float md = s.nu * B;
    P = fmaf(b * u, md, P);
    const float h3 = fmaf(tm1, ir2, cf.k23 * e);
    const float inner = fmaf(md, h3, fmaf(tm1, s.w2n, s.w1));
    Q = fmaf(u, fmaf(A, inner, (tm1 * C3) * s.nu), Q);
}

// One pair, both directions: P, Q accumulate row i; cp, cq receive the
// contribution of point i to row j.  The reverse direction is the forward
// formula with i and j exchanged and d negated; in the notation of pair_fwd:
//   row j, 1 / eps: (e-1) w2n_i / r + b nu_i A u
//   row j, 2:       u [B (nu_i A h3 + tm1 w2n_i + w1_i) + t3n C nu_i]
// so the pair costs 43 VALU operations and two transcendentals.  It is split
// in two: pair_head (d, 1/r, r and e, the two transcendentals) and pair_tail
// (the rest), so that a lane can issue the heads of both its targets before
// either tail and hide the transcendentals' latency behind the other
// target's work.
struct PairHead {
    float dx, dy, dz, ir, r, e;
};

template <bool SCALED>
__device__ __forceinline__ PairHead pair_head(const Src12 &s, const OwnF32 &o, const CoefF32 &cf)
{
    PairHead h;
    h.dx = s.x - o.x;
    h.dy = s.y - o.y;
    h.dz = s.z - o.z;
    const float r2 = h.dx * h.dx + h.dy * h.dy + h.dz * h.dz;
    h.ir = __builtin_amdgcn_rsqf(r2);
    h.r = r2 * h.ir;
    h.e = __builtin_amdgcn_exp2f(cf.kexp * h.r);
    return h;
}

// FIRST starts cp, cq; otherwise the pair's contributions are added to them
// (the thread's further targets on the same source).
template <bool SCALED, bool FIRST>
__device__ __forceinline__ void pair_tail(const Src12 &s, const OwnF32 &o, const CoefF32 &cf,
                                          const PairHead &h, float &P, float &Q, float &cp,
                                          float &cq)
{
    const float dx = h.dx, dy = h.dy, dz = h.dz, ir = h.ir, r = h.r, e = h.e;
    const float ir2 = ir * ir;
    const float u = ir2 * ir;
    const float kr = SCALED ? r : cf.kappa * r;
    const float em1 = e - 1.f;
    const float em1ir = em1 * ir;
    P = fmaf(em1ir, s.w2n, P);
    const float p2 = FIRST ? em1ir * o.w2n : fmaf(em1ir, o.w2n, cp);
    const float tm1 = fmaf(kr, e, em1);
    const float bu = fmaf(tm1, 0.333333343f, cf.c13) * u;   // (c13 - t3n) u
    const float h3 = fmaf(tm1, ir2, cf.k23 * e);
    const float A = o.nx * dx + o.ny * dy + o.nz * dz;
    const float B = s.nx * dx + s.ny * dy + s.nz * dz;
    const float C3 = o.mx * s.nx + o.my * s.ny + o.mz * s.nz;   // -C / 3
    const float tc = tm1 * C3;   // t3n C
    // source j on row i
    const float md = s.nu * B;
    P = fmaf(bu, md, P);
    const float inner = fmaf(md, h3, fmaf(tm1, s.w2n, s.w1));
    Q = fmaf(u, fmaf(A, inner, tc * s.nu), Q);
    // source i on row j
    const float pm = o.nu * A;
    cp = fmaf(bu, pm, p2);
    const float innerr = fmaf(pm, h3, fmaf(tm1, o.w2n, o.w1));
    const float yr = fmaf(B, innerr, tc * o.nu);
    cq = FIRST ? u * yr : fmaf(u, yr, cq);
}

// Diagonal tile (sources = the thread's own tile): forward direction, j = i
// dropped.  The thread owns TT targets, k * (TILE / TT) + self of the tile.
template <bool SCALED, int TT>
__device__ __forceinline__ void sweep_diag(const SrcTileF32 &sh, const OwnF32 (&o)[TT],
                                           const CoefF32 &cf, float (&P)[TT], float (&Q)[TT],
                                           int self)
{
#pragma unroll 2
    for (int jj = 0; jj < TILE; ++jj) {
        const Src12 s = sh.get(jj);
#pragma unroll
        for (int k = 0; k < TT; ++k)
            pair_fwd<SCALED, true>(s, o[k], cf, jj == k * (TILE / TT) + self, P[k], Q[k]);
    }
}

// One source against the thread's TT targets; (cp, cq) is its contribution to
// the source's rows summed over those targets.
template <bool SCALED, int TT>
__device__ __forceinline__ void pair_both_tt(const Src12 &s, const OwnF32 (&o)[TT],
                                             const CoefF32 &cf, float (&P)[TT], float (&Q)[TT],
                                             float &cp, float &cq)
{
    PairHead h[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k)
        h[k] = pair_head<SCALED>(s, o[k], cf);
    __builtin_amdgcn_sched_barrier(0);
    pair_tail<SCALED, true>(s, o[0], cf, h[0], P[0], Q[0], cp, cq);
#pragma unroll
    for (int k = 1; k < TT; ++k) {
        __builtin_amdgcn_sched_barrier(0);
        pair_tail<SCALED, false>(s, o[k], cf, h[k], P[k], Q[k], cp, cq);
    }
}

// Off-diagonal tile: both directions.  The contributions to the tile's source
// rows are summed over the wave's targets in groups of 4 sources (8 values
// per lane: reduce-scatter within rows, then across the 4 rows) and stored
// in colw[comp * TILE + j] (comp 0: row 1, 1: row 2); colw holds 2 * TILE
// floats.
template <bool SCALED, int TT>
__device__ __forceinline__ void sweep_pairwise(const SrcTileF32 &sh, const OwnF32 (&o)[TT],
                                               const CoefF32 &cf, float (&P)[TT],
                                               float (&Q)[TT], float *colw, int lane)
{
    for (int g = 0; g < TILE; g += 4) {
        float a[4];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            float p0, q0, p2, q2;
            pair_both_tt<SCALED, TT>(sh.get(g + k), o, cf, P, Q, p0, q0);
            __builtin_amdgcn_sched_barrier(0);
            pair_both_tt<SCALED, TT>(sh.get(g + k + 2), o, cf, P, Q, p2, q2);
            rs_stage1(p0, q0, p2, q2, lane, a[2 * k], a[2 * k + 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        float t = rs_finish(a, lane);
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        // value index q: source g + q/2, row q%2.  Every lane with the same q
        // holds the same sum, bit for bit (each addition above adds the same
        // two operands in both lanes of a pair), so all 64 lanes store it:
        // eight lanes write one word with one value, and the loop stays free
        // of branches.
        const int q = (lane >> 1) & 7;
        colw[(q & 1) * TILE + g + (q >> 1)] = t;
    }
}


using fm::exp_neg_pair;

// 1/sqrt(x) for finite x > 0: the hardware estimate (relative error below
// 2^-22) refined by fm::rsqrt_refine to about one ulp.  x = 0 gives NaN;
// callers that can meet it replace the result.
__device__ __forceinline__ double rsqrt_pos(double x)
{
    return fm::rsqrt_refine(x, __builtin_amdgcn_rsq(x));
}

// ---- pairwise FP64 sweep ------------------------------------------------------
//
// The generic (FP64) pair algebra, with d = x_i - x_j, evaluated once per
// unordered pair.  Forward stream: w = a psi, f = a phi; transpose stream:
// w = l1, f = l2; the moment is m = f n.  With A = n_i.d, B = n_j.d and
// C = n_i.n_j, every product with a moment is a product with a normal times
// f (m_j.d = f_j B, n_i.m_j = f_j C, m_i.d = f_i A, n_j.m_i = f_i C), so the
// three dot products serve both directions.  For source j on row i (cP = g2,
// cQ = -g3 forward; cP = -g3, cQ = g2 transposed):
//   P_i += -(e-1) w_j / r + cP f_j B / r^3
//   Q_i += [-A (f_j B h + cQ w_j) + tm1 f_j C] / r^3
// and for source i on row j the same with i and j exchanged, d -> -d:
//   P_j += -(e-1) w_i / r - cP f_i A / r^3
//   Q_j += [B (-f_i A h + cQ w_i) + tm1 f_i C] / r^3.
// Transposed, P and Q are rows 2 and 1 of the output (swapped by the caller).
struct alignas(64) Src8d {
    double x, y, z, w, nx, ny, nz, f;
};

struct OwnF64 {
    double x, y, z, nx, ny, nz, w, f;
};

__device__ __forceinline__ OwnF64 own_point64(const Src8d &e)
{
    return OwnF64{e.x, e.y, e.z, e.nx, e.ny, e.nz, e.w, e.f};
}

// With BOTH, FIRST starts cp, cq; otherwise the pair's contributions to the
// source's rows are added to them (the thread's further targets).
template <bool TRANS, bool BOTH, bool DIAG, bool FIRST = true>
__device__ __forceinline__ void pair64(const Src8d &s, const OwnF64 &o, const Coef<double> &cf,
                                       bool skip, double &P, double &Q, double &cp, double &cq)
{
    const double dx = o.x - s.x, dy = o.y - s.y, dz = o.z - s.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    double ir = rsqrt_pos(r2);
    if (DIAG)
        ir = skip ? 0.0 : ir;
    const double ir2 = ir * ir;
    const double u = ir2 * ir;
    const double kr = cf.kappa * (r2 * ir);
    const double e = exp_neg_pair(kr);
    const double em1 = e - 1.0;
    const double tm1 = fma(kr, e, em1);
    const double g2 = fma(cf.eps, tm1, cf.epsm1);
    const double g3 = fma(cf.ieps, tm1, cf.iepsm1);
    const double h = fma(tm1, 3.0 * ir2, cf.k2 * e);
    const double cPu = (TRANS ? -g3 : g2) * u;
    const double cQ = TRANS ? g2 : -g3;
    const double a = -em1 * ir;
    const double A = o.nx * dx + o.ny * dy + o.nz * dz;
    const double B = s.nx * dx + s.ny * dy + s.nz * dz;
    const double C = o.nx * s.nx + o.ny * s.ny + o.nz * s.nz;
    const double tc = tm1 * C;
    const double md = s.f * B;
    P = fma(a, s.w, P);
    P = fma(cPu, md, P);
    Q = fma(u, fma(-A, fma(md, h, cQ * s.w), tc * s.f), Q);
    if (BOTH) {
        const double pm = o.f * A;
        const double yq = fma(B, fma(-pm, h, cQ * o.w), tc * o.f);
        if (FIRST) {
            cp = fma(-cPu, pm, a * o.w);
            cq = u * yq;
        } else {
            cp = fma(-cPu, pm, fma(a, o.w, cp));
            cq = fma(u, yq, cq);
        }
    }
}

// Sources per LDS stage and targets per thread of the pairwise FP64 sweep:
// blocks of TILE / SYM64_TT threads (one wave), each owning SYM64_TT targets,
// so that every column reduction serves four pairs per lane; the source tile
// is staged in quarters, 5 KB of LDS per block.  The kernels' launch bounds
// ask for SYM64_MIN_WAVES waves per SIMD (at most 168 VGPRs; left free, the
// compiler takes 185 and 2 waves).
constexpr int SYM64_TT = 4;
constexpr int SYM64_MIN_WAVES = 3;
constexpr int SYM64_NT = TILE / SYM64_TT;
constexpr int SYM64_NS = SYM64_NT;

// Diagonal tile: forward direction, j = i dropped; sh holds sources
// base .. base + SYM64_NS - 1 of the tile.
template <bool TRANS>
__device__ __forceinline__ void sweep_diag64(const Src8d *sh, int base, const OwnF64 (&o)[SYM64_TT],
                                             const Coef<double> &cf, double (&P)[SYM64_TT],
                                             double (&Q)[SYM64_TT])
{
    double dummy0 = 0.0, dummy1 = 0.0;
#pragma unroll 2
    for (int jj = 0; jj < SYM64_NS; ++jj) {
        const Src8d s = sh[jj];
#pragma unroll
        for (int k = 0; k < SYM64_TT; ++k)
            pair64<TRANS, false, true>(s, o[k], cf,
                                       base + jj == k * SYM64_NT + (int)threadIdx.x, P[k], Q[k],
                                       dummy0, dummy1);
    }
}

template <bool TRANS>
__device__ __forceinline__ void pair64_tt(const Src8d &s, const OwnF64 (&o)[SYM64_TT],
                                          const Coef<double> &cf, double (&P)[SYM64_TT],
                                          double (&Q)[SYM64_TT], double &cp, double &cq)
{
    pair64<TRANS, true, false, true>(s, o[0], cf, false, P[0], Q[0], cp, cq);
#pragma unroll
    for (int k = 1; k < SYM64_TT; ++k) {
        __builtin_amdgcn_sched_barrier(0);
        pair64<TRANS, true, false, false>(s, o[k], cf, false, P[k], Q[k], cp, cq);
    }
}

// Off-diagonal tile, both directions; column sums as in sweep_pairwise, over
// the SYM64_NS staged sources, stored in colw[comp * SYM64_NS + j]
// (2 * SYM64_NS doubles).
template <bool TRANS>
__device__ __forceinline__ void sweep_pairwise64(const Src8d *sh, const OwnF64 (&o)[SYM64_TT],
                                                 const Coef<double> &cf,
                                                 double (&P)[SYM64_TT], double (&Q)[SYM64_TT],
                                                 double *colw, int lane)
{
    for (int g = 0; g < SYM64_NS; g += 4) {
        double a[4];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            double p0, q0, p2, q2;
            pair64_tt<TRANS>(sh[g + k], o, cf, P, Q, p0, q0);
            __builtin_amdgcn_sched_barrier(0);
            pair64_tt<TRANS>(sh[g + k + 2], o, cf, P, Q, p2, q2);
            rs_stage1(p0, q0, p2, q2, lane, a[2 * k], a[2 * k + 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        double t = rs_finish(a, lane);
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        const int q = (lane >> 1) & 7;   // as in sweep_pairwise
        colw[(q & 1) * SYM64_NS + g + (q >> 1)] = t;
    }
}


// ---- one work item of the pairwise sweeps ----------------------------------
//
// Target tile I of a system whose points start at `src` (T tiles), against its
// source tiles J0..J1-1 (J0 >= I; the tile J = I runs forward only).  Row sums
// go to rp[0..TILE) and rp[TILE..2 TILE), the contributions of tile pair
// (I, J) to the rows of tile J to cp_base + pair_index(I, J) * 2 TILE.  Blocks
// of SYM_NT (FP32) or SYM64_NT (FP64) threads; sh and colw are the block's LDS.

// FP32: blocks of TILE / SYM_TT threads, each thread owning SYM_TT targets
// (k * TILE / SYM_TT + threadIdx.x), so that every column reduction serves
// SYM_TT pairs per lane.
template <bool SCALED>
__device__ __forceinline__ void sym_item_f32(const Src12 *__restrict__ src, int I, int J0, int J1,
                                             int T, const CoefF32 &cf, double *__restrict__ rp,
                                             float *__restrict__ cp_base, SrcTileF32 &sh,
                                             float (*colw)[2 * TILE])
{
    constexpr int TT = SYM_TT, NT = TILE / SYM_TT, NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    OwnF32 o[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k)
        o[k] = own_point(src[(int64_t)I * TILE + k * NT + threadIdx.x]);
    Acc<float> aP[TT], aQ[TT];
    for (int J = J0; J < J1; ++J) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TT; ++k)
            sh.put(k * NT + threadIdx.x, src[(int64_t)J * TILE + k * NT + threadIdx.x]);
        __syncthreads();
        float P[TT], Q[TT];
#pragma unroll
        for (int k = 0; k < TT; ++k)
            P[k] = Q[k] = 0.f;
        if (J == I) {
            sweep_diag<SCALED, TT>(sh, o, cf, P, Q, (int)threadIdx.x);
        } else {
            sweep_pairwise<SCALED, TT>(sh, o, cf, P, Q, colw[wid], lane);
            __syncthreads();
            float *cp = cp_base + sym_pair_index(I, J, T) * (2 * TILE);
            for (int t = threadIdx.x; t < 2 * TILE; t += NT) {
                float v = colw[0][t];
#pragma unroll
                for (int w = 1; w < NW; ++w)
                    v += colw[w][t];
                cp[t] = v;
            }
        }
#pragma unroll
        for (int k = 0; k < TT; ++k) {
            aP[k].add(P[k]);
            aQ[k].add(Q[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < TT; ++k) {
        rp[k * NT + threadIdx.x] = aP[k].value();
        rp[TILE + k * NT + threadIdx.x] = aQ[k].value();
    }
}

// FP64: blocks of SYM64_NT threads (SYM64_TT targets each); every source tile
// is staged and swept in parts of SYM64_NS sources.
template <bool TRANS>
__device__ __forceinline__ void sym_item_f64(const Src8d *__restrict__ src, int I, int J0,
                                             int J1, int T, const Coef<double> &cf,
                                             double *__restrict__ rp,
                                             double *__restrict__ cp_base, Src8d *sh,
                                             double (*colw)[2 * SYM64_NS],
                                             double (*acc)[SYM64_NT])
{
    constexpr int TT = SYM64_TT, NT = SYM64_NT, NS = SYM64_NS;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, t = threadIdx.x;
    OwnF64 o[TT];
#pragma unroll
    for (int k = 0; k < TT; ++k)
        o[k] = own_point64(src[(int64_t)I * TILE + k * NT + t]);
    // The row sums over the item's source tiles live in LDS (acc[k][t] and
    // acc[TT + k][t], private to the thread): in registers they would be
    // spilled at this occupancy, at every source tile.
#pragma unroll
    for (int k = 0; k < TT; ++k)
        acc[k][t] = acc[TT + k][t] = 0.0;
    for (int J = J0; J < J1; ++J) {
        double P[TT], Q[TT];
#pragma unroll
        for (int k = 0; k < TT; ++k)
            P[k] = Q[k] = 0.0;
        for (int base = 0; base < TILE; base += NS) {
            __syncthreads();
            sh[t] = src[(int64_t)J * TILE + base + t];
            __syncthreads();
            if (J == I) {
                sweep_diag64<TRANS>(sh, base, o, cf, P, Q);
            } else {
                sweep_pairwise64<TRANS>(sh, o, cf, P, Q, colw[wid], lane);
                __syncthreads();
                double *cp = cp_base + sym_pair_index(I, J, T) * (2 * TILE);
                double c0 = colw[0][t], c1 = colw[0][NS + t];
#pragma unroll
                for (int w = 1; w < NT / 64; ++w) {   // the block's waves in order
                    c0 += colw[w][t];
                    c1 += colw[w][NS + t];
                }
                cp[base + t] = c0;
                cp[TILE + base + t] = c1;
            }
        }
#pragma unroll
        for (int k = 0; k < TT; ++k) {
            acc[k][t] += P[k];
            acc[TT + k][t] += Q[k];
        }
    }
#pragma unroll
    for (int k = 0; k < TT; ++k) {
        rp[k * NT + t] = acc[k][t];
        rp[TILE + k * NT + t] = acc[TT + k][t];
    }
}

// ---- banded pairwise FP32 sweep ----------------------------------------------
//
// A block of BAND_WAVES waves holds BAND_MT target tiles at once (two waves per
// tile, two targets per lane, as in sym_item_f32), a macro tile.  A work item
// is a band of consecutive macro tiles [m0, m1) against a run of source tiles
// [j0, j1) (j0 at or after the band's first tile): for each macro tile the
// block streams the run's tiles through LDS once; each wave evaluates its tile
// against the source tile (both directions when J > I, forward only with j = i
// dropped when J = I, nothing when J < I), keeps its row sums in registers
// across the run, and leaves its column sums for the source tile in colw; the
// block adds the waves' column sums, in wave order, to an LDS accumulator per
// source tile of the run, which thus collects every target tile of the band.
// Records (2 x TILE floats: row 1 then row 2) go to recs: one per (item, target
// tile I) at rslot + I - first tile of the band, when the run reaches J >= I,
// and one per (item, source tile J) at cslot + J - j0.  Every unordered tile
// pair is evaluated by exactly one item.
struct BandSmem {
    SrcTileF32 sh;
    float colw[BAND_WAVES][2 * TILE];
    float colacc[BAND_RUN_MAX][2 * TILE];
    int flags[BAND_WAVES];
};

template <bool SCALED>
__device__ __forceinline__ void band_item_f32(const Src12 *__restrict__ src, const BandItem &it,
                                              int T, const CoefF32 &cf, float *__restrict__ recs,
                                              BandSmem &sm)
{
    constexpr int TT = SYM_TT, NT = TILE / SYM_TT, NB = BAND_WAVES * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tw = w >> 1, tt = (w & 1) * 64 + lane;   // tile of the macro, thread within it
    const int run = it.j1 - it.j0, i0 = it.m0 * BAND_MT;
    for (int e = threadIdx.x; e < run * 2 * TILE; e += NB)
        sm.colacc[e / (2 * TILE)][e % (2 * TILE)] = 0.f;
    for (int M = it.m0; M < it.m1; ++M) {
        const int I = M * BAND_MT + tw;
        const bool mine = I < T;   // the last macro tile may reach past the mesh
        OwnF32 o[TT];
#pragma unroll
        for (int k = 0; k < TT; ++k)
            o[k] = own_point(src[(int64_t)(mine ? I : 0) * TILE + k * NT + tt]);
        Acc<float> aP[TT], aQ[TT];
        for (int J = it.j0; J < it.j1; ++J) {
            __syncthreads();
            if (threadIdx.x < TILE)
                sm.sh.put(threadIdx.x, src[(int64_t)J * TILE + threadIdx.x]);
            __syncthreads();
            const int mode = (!mine || J < I) ? 0 : (J == I ? 1 : 2);
            float P[TT], Q[TT];
#pragma unroll
            for (int k = 0; k < TT; ++k)
                P[k] = Q[k] = 0.f;
            if (mode == 2)
                sweep_pairwise<SCALED, TT>(sm.sh, o, cf, P, Q, sm.colw[w], lane);
            else if (mode == 1)
                sweep_diag<SCALED, TT>(sm.sh, o, cf, P, Q, tt);
            if (lane == 0)
                sm.flags[w] = mode == 2;
#pragma unroll
            for (int k = 0; k < TT; ++k) {
                aP[k].add(P[k]);
                aQ[k].add(Q[k]);
            }
            __syncthreads();
            float *acc = sm.colacc[J - it.j0];
            for (int e = threadIdx.x; e < 2 * TILE; e += NB) {
                float v = acc[e];
#pragma unroll
                for (int ww = 0; ww < BAND_WAVES; ++ww)
                    v += sm.flags[ww] ? sm.colw[ww][e] : 0.f;
                acc[e] = v;
            }
        }
        if (mine && it.j1 > I) {
            float *rr = recs + (int64_t)(it.rslot + I - i0) * (2 * TILE);
#pragma unroll
            for (int k = 0; k < TT; ++k) {
                rr[k * NT + tt] = (float)aP[k].value();
                rr[TILE + k * NT + tt] = (float)aQ[k].value();
            }
        }
    }
    __syncthreads();
    float *cr = recs + (int64_t)it.cslot * (2 * TILE);
    for (int e = threadIdx.x; e < run * 2 * TILE; e += NB)
        cr[e] = sm.colacc[e / (2 * TILE)][e % (2 * TILE)];
}

inline __device__ CoefF32 coef_f32(double eps, double kappa, bool scaled)
{
    const double kap = scaled ? 1.0 : kappa;   // kappa in the stream's length unit
    CoefF32 cf;
    cf.kappa = float(kap);
    cf.kexp = float(-kap * 1.4426950408889634074);
    cf.c13 = float((1.0 - 1.0 / eps) / 3.0);
    cf.k23 = float(kap * kap / 3.0);
    return cf;
}


}  // namespace dev
}  // namespace pbk
