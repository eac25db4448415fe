// hevi_device.h -- device helpers shared by the kernel files of the HEVI
// step (internal to the library): constants, storage types, the Koren face
// value, the column solve's reciprocal.
#pragma once

#include <type_traits>

#include "hevi_kernels.h"

namespace hv {
namespace {

constexpr double kGamma = 1.4;
constexpr double kGrav = 9.80665;

template <typename T, int L>
using vec_t = T __attribute__((ext_vector_type(L)));

// Pointer into device global memory.  Every array a kernel reaches through
// a member table is global, but the compiler cannot see that through the
// table and emits flat memory instructions; with the address space explicit
// it emits global ones, which take a scalar base and a 32-bit per-lane
// offset.  Which of the two schedules better differs per kernel (measured:
// the float64 slow flux gains 16% with global instructions, the float32 one
// loses 13%), so it is a property of the addressing below.
template <typename T>
using gptr = T __attribute__((address_space(1))) *;

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Field f of state buffer b.
__device__ __forceinline__ void *buf(const MemberDev *m, int b, int f) { return m->st[b][f]; }

template <typename T> __device__ __forceinline__ T xexpm1(T x) { return expm1(x); }
template <> __device__ __forceinline__ float xexpm1<float>(float x) { return expm1f(x); }
template <typename T> __device__ __forceinline__ T xlog1p(T x) { return log1p(x); }
template <> __device__ __forceinline__ float xlog1p<float>(float x) { return log1pf(x); }

// a * b + c with one rounding
__device__ __forceinline__ double xfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float xfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Half the Koren increment, psi(D+/D-) D- / 2, without the division:
// psi(r) = max(0, min(2r, (1 + 2r)/3, 2))  (Koren 1993, kappa = 1/3).
// Written sign-symmetrically: with s = sign(D-), a = |D-| and b = s D+,
//   psi D- / 2 = s max(0, min(b, (a + 2b)/6, a)),
// and D- = 0 gives 0.  Both signs share one min/max chain, and the halving
// is folded into exact power-of-two scalings (1/6 = (1/3)/2 exactly), so the
// value equals q1 + 0.5 * (the two-branch form) bit for bit.
template <typename T> struct SignBits;
template <> struct SignBits<float> {
    using U = unsigned;
    static constexpr U kSign = 0x80000000u;
};
template <> struct SignBits<double> {
    using U = unsigned long long;
    static constexpr U kSign = 0x8000000000000000ull;
};

template <typename T>
__device__ __forceinline__ T koren_half(T dm, T dp)
{
    using U = typename SignBits<T>::U;
    const U sgn = __builtin_bit_cast(U, dm) & SignBits<T>::kSign;
    const T a = fabs(dm);
    const T b = __builtin_bit_cast(T, __builtin_bit_cast(U, dp) ^ sgn);
    // a + 2b in one rounding (2b is exact), as a + (b + b) rounds it
    const T t = xfma(b, T(2), a) * T(1.0 / 6.0);
    const T v = fmax(T(0), fmin(fmin(b, t), a));
    return __builtin_bit_cast(T, __builtin_bit_cast(U, v) ^ sgn);
}

// x if on, else +0 (the value's bits masked, no select)
template <typename T>
__device__ __forceinline__ T keep_if(bool on, T x)
{
    using U = typename SignBits<T>::U;
    const U m = on ? ~U(0) : U(0);
    return __builtin_bit_cast(T, __builtin_bit_cast(U, x) & m);
}

// Limited face value between L and R for mass flux m (m >= 0: from L).  The
// downwind-side differences for m < 0 are the negated upwind ones
// (x - y = -(y - x) exactly).
template <typename T>
__device__ __forceinline__ T kface(T qLL, T qL, T qR, T qRR, T m)
{
    const bool up = m >= T(0);
    const T d1 = qR - qL;
    const T dm = up ? qL - qLL : -(qRR - qR);
    const T dp = up ? d1 : -d1;
    const T q1 = up ? qL : qR;
    return q1 + koren_half(dm, dp);
}

// Reciprocal for the column solve: the hardware estimate refined by Newton
// steps r <- r + r (1 - x r) (two in float64, one in float32), within an ulp
// of 1/x for the normal, nonzero pivots a diagonally dominant system has; a
// correctly rounded division costs about three times as many instructions.
__device__ __forceinline__ double solve_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float solve_rcp(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// Solve the segment's tridiagonal system A x_{r-1} + B x_r + C x_{r+1} = D
// (SG lanes, L >= 2 rows each),
// one row per level face, lane p holding rows p*L .. p*L+L-1.  A of the
// first row and C of the last row of the column must be 0.
}  // namespace
}  // namespace hv
