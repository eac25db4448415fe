// hevi_kernels.hip -- HIP kernels of the HEVI dynamical-core step for gfx950.
//
// Work mapping.  A column (i, j) of nz cells is owned by one 16-lane segment
// of a 64-lane wavefront (32 lanes for float64 storage with 64 levels); lane p
// of the segment owns the L = nz/16 (nz/32) consecutive levels
// k0 = p*L .. k0+L-1.  In the column-fastest layout those L values are
// contiguous, so each per-lane access is one vector load and a wavefront
// touches 4 (2) columns of contiguous memory.  Vertical neighbours live in the
// adjacent lane of the same segment (DPP row shifts or shuffles); horizontal
// neighbours are other columns and come through L1/L2.  A tile of 16 columns
// (16x1, 8x2 or 4x4, in launch or XCD-chunked order, as the autotuner chose;
// the results do not depend on it) runs as one block, or in the slow sweeps
// with 32-lane segments as two blocks of 8 columns.
//
// The per-column tridiagonal system of the vertically implicit part is solved
// without leaving the segment: every lane eliminates its interior rows in
// terms of the last unknown of the lane below and its own last unknown; the
// remaining 16-row (32-row) system of those interface unknowns is solved by
// parallel cyclic reduction over the segment (4 or 5 steps), and the interior
// values follow.
//
// Equations: the paper (Sect. 1.1) fixes finite volumes, an RK3 long step
// after Wicker & Skamarock (2002) and HEVI short steps; the discrete form
// implemented here is:
//  slow sweep, once per stage on the stage-input state
//    u = U / (mean of rho over the x-face), v likewise, w = W / (rho linearly
//    interpolated to the level face); theta = Theta / rho;
//    S_U = -div(m q) over the U control volume with mass fluxes m averaged
//    from U, V, W and q the Koren (kappa = 1/3) face value of u; S_V, S_W
//    likewise; R_Theta = -div(m (Koren face theta - centred face theta));
//    p'_s = p_ref expm1(gamma log1p(Theta'/Theta_ref)), C_s = gamma p/Theta,
//    P0_s = p'_s - C_s Theta'.
//  short step (length dtau), from state n to n+1
//    p' = P0_s + C_s Theta';  U+ = U + dtau (S_U - dx p'),  V+ likewise;
//    rho~ = rho' - dtau (dx U+ + dy V+);
//    Theta~ = Theta' + dtau (R_Theta - dx(theta_x U+) - dy(theta_y V+));
//    vertically, with X* = beta X+ + (1-beta) X and thf = theta_s on faces:
//    rho'+ = rho~ - dtau dz(W*),  Theta'+ = Theta~ - dtau dz(thf W*),
//    W+ = W + dtau (S_W - dz p* - g rho* on faces), which is tridiagonal in W+.
#include "hevi_kernels.h"
#include "hevi_device.h"

#include <cstdint>
#include <mutex>
#include <type_traits>

namespace hv {
namespace {

constexpr int SEG = kSeg;
constexpr int BLOCK = kBlock;

// Block -> (member, tile) -> this segment's column.  A tile is (1 << ti_log2)
// columns along x by 16 >> ti_log2 along y.
struct Where {
    const MemberDev *m;
    int i, j;
    bool active;
};
// Launch order of the blocks.  Workgroups go to the 8 XCDs (each with its own
// L2) in turn, so in launch order neighbouring tiles along x land on
// different L2s.  The XCD-chunked order deals the tiles in runs of
// kXcdChunk: within every group of 8 * kXcdChunk consecutive tiles, XCD x
// gets the kXcdChunk consecutive tiles x * kXcdChunk ..; blocks past the last
// whole group keep launch order.  Most x-neighbours then share an L2, while
// all XCDs still stream through neighbouring memory at any moment (giving
// each XCD one contiguous eighth of the domain instead was slower).  The
// autotuner decides whether it pays.  nblocks: blocks of the launch.
constexpr int kXcdChunk = 8;
__device__ __forceinline__ int block_order(const Group &gr, int nblocks)
{
    int b = (int)blockIdx.x;
    if (gr.xcd) {
        const int full = nblocks / (8 * kXcdChunk) * (8 * kXcdChunk);
        if (b < full) {
            const int n = b >> 3;
            b = (n / kXcdChunk) * (8 * kXcdChunk) + (b & 7) * kXcdChunk + n % kXcdChunk;
        }
    }
    return gr.rev ? nblocks - 1 - b : b;
}

// Blocks per tile (SP): in the slow sweeps a 32-lane segment's tile of 16
// columns runs as two blocks of 8 columns (256 threads each), so that
// resident blocks are not the occupancy limit (512-thread blocks fit only 4
// waves per SIMD where the registers allow 5; FP64 flux 1.67 -> 1.56 ms).
// The short step keeps one block per tile (measured 1.77 ms against
// 1.78-1.79 ms split).  Launches multiply the grid by it.
template <int SG>
constexpr int split_of() { return SG == 32 ? 2 : 1; }
template <int SG, int SP = split_of<SG>()>
constexpr int threads_of() { return kColsPerBlock / SP * SG; }

template <int SG = SEG, int SP = split_of<SG>()>
__device__ __forceinline__ Where locate(const Group &gr)
{
    Where w;
    constexpr int sp = SP;
    const int b0 = block_order(gr, gr.nblocks * sp);
    const int b = b0 / sp;
    int t = b, id = gr.first;
    if (gr.nm > 1) {
        const unsigned v = gr.blk[b];
        t = (int)(v & 0xFFFFFFu);
        id = (int)(v >> 24);
    }
    w.m = gr.mem + id;
    const int ti = 1 << gr.ti_log2, tj = kColsPerBlock >> gr.ti_log2;
    const int tiles_x = (w.m->nx + ti - 1) / ti;
    const int c = (int)threadIdx.x / SG + (b0 % sp) * (kColsPerBlock / sp);
    w.i = (t % tiles_x) * ti + (c & (ti - 1));
    w.j = (t / tiles_x) * tj + (c >> gr.ti_log2);
    w.active = w.i < w.m->nx && w.j < w.m->ny;
    return w;
}

// Storage orders of a 3D field with nz levels per column.
struct KIJ {
    static constexpr bool kContig = true;
    static constexpr bool kOff32 = false;
    static constexpr bool kGlobal = false;
    __device__ static size_t at(int i, int j, int k, int nx, int ny, int nz)
    {
        return ((size_t)j * nx + i) * nz + k;
    }
    __device__ static unsigned at32(int i, int j, int k, int nx, int ny, int nz)
    {
        return ((unsigned)j * nx + i) * nz + k;
    }
};
struct IJK {
    static constexpr bool kContig = false;
    static constexpr bool kOff32 = false;
    static constexpr bool kGlobal = false;
    __device__ static size_t at(int i, int j, int k, int nx, int ny, int nz)
    {
        return ((size_t)k * ny + j) * nx + i;
    }
    __device__ static unsigned at32(int i, int j, int k, int nx, int ny, int nz)
    {
        return ((unsigned)k * ny + j) * nx + i;
    }
};
// The same order addressed by 32-bit byte offsets from the array's base (one
// scalar base register per array, no per-lane 64-bit address arithmetic),
// with flat or (G) global memory instructions; valid while every array of
// the member is under 4 GiB, which the host checks before it picks these.
template <class Base, bool G>
struct Off32 : Base {
    static constexpr bool kOff32 = true;
    static constexpr bool kGlobal = G;
};


// One lane's share of a column: segments of SG lanes per column (16, or 32
// for the float64-solve short step), lane p owning levels p*L .. p*L+L-1.
template <class Lay, int L, int SG = SEG>
struct Lane {
    int i, j, p, k0, nx, ny, nz;
    size_t kstride;

    __device__ Lane(int nx_, int ny_, int nz_, int i_, int j_)
    {
        nx = nx_; ny = ny_; nz = nz_;
        i = i_;
        j = j_;
        p = threadIdx.x % SG;
        k0 = p * L;
        kstride = Lay::kContig ? 1 : (size_t)nx * ny;
    }
    __device__ size_t off(int di, int dj) const
    {
        return Lay::at(wrapc(i + di, nx), wrapc(j + dj, ny), k0, nx, ny, nz);
    }
    template <typename U>
    using ptr_t = std::conditional_t<Lay::kGlobal, gptr<U>, U *>;
    // element of the lane's column (i+di, j+dj) at level k0 + l
    template <typename T>
    __device__ ptr_t<T> elem(T *a, int di, int dj, int l = 0) const
    {
        if constexpr (Lay::kOff32) {
            const unsigned e = Lay::at32(wrapc(i + di, nx), wrapc(j + dj, ny), k0, nx, ny, nz) +
                               (unsigned)l * (unsigned)kstride;
            using B = std::conditional_t<std::is_const_v<T>, const char, char>;
            return (ptr_t<T>)((ptr_t<B>)a + (size_t)(e * (unsigned)sizeof(T)));
        } else {
            return (ptr_t<T>)a + off(di, dj) + (size_t)l * kstride;
        }
    }
    // Load the lane's L levels of column (i+di, j+dj).  NT = non-temporal:
    // for data no other column reads in this kernel.
    template <bool NT = false, typename T>
    __device__ void load(const T *__restrict__ a, int di, int dj, T (&x)[L]) const
    {
        if constexpr (Lay::kContig) {
            const auto vq = (ptr_t<const vec_t<T, L>>)elem(a, di, dj);
            vec_t<T, L> t;
            if constexpr (NT) t = __builtin_nontemporal_load(vq);
            else t = *vq;
#pragma unroll
            for (int l = 0; l < L; ++l) x[l] = t[l];
        } else {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const ptr_t<const T> q = elem(a, di, dj, l);
                if constexpr (NT) x[l] = __builtin_nontemporal_load(q);
                else x[l] = *q;
            }
        }
    }
    // Store the lane's L levels of the own column (non-temporal: results are
    // not read again by this kernel).
    template <typename T, typename S>
    __device__ void store(T *__restrict__ a, const S (&x)[L]) const
    {
        if constexpr (Lay::kContig) {
            vec_t<T, L> t;
#pragma unroll
            for (int l = 0; l < L; ++l) t[l] = (T)x[l];
            __builtin_nontemporal_store(t, (ptr_t<vec_t<T, L>>)elem(a, 0, 0));
        } else {
#pragma unroll
            for (int l = 0; l < L; ++l) __builtin_nontemporal_store((T)x[l], elem(a, 0, 0, l));
        }
    }
    // per-column geometry value f of column (i+di, j+dj)
    __device__ double geo(const double *__restrict__ g, int f, int di, int dj) const
    {
        return g[((size_t)wrapc(j + dj, ny) * nx + wrapc(i + di, nx)) * GEO_NFIELDS + f];
    }
    // per-level constant of the lane's levels (+ offset, clamped to the
    // column), as type S.  VEC: the lane's own L levels as one vector load,
    // from the table's float32 copy for float; otherwise one float64 load
    // per level.  Which schedules better differs per kernel (measured).
    template <typename S, bool VEC = true>
    __device__ void vmet(const double *__restrict__ vm, int f, S (&x)[L], int koff = 0) const
    {
        if constexpr (VEC && sizeof(S) == sizeof(float)) {
            const float *__restrict__ vf = (const float *)(vm + (size_t)VM_NFIELDS * nz) +
                                           (size_t)f * nz;
            if (koff == 0) {
                const vec_t<float, L> t = *(const vec_t<float, L> *)(vf + k0);
#pragma unroll
                for (int l = 0; l < L; ++l) x[l] = t[l];
                return;
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                int k = k0 + l + koff;
                k = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
                x[l] = vf[k];
            }
        } else if (VEC && koff == 0) {
            const vec_t<double, L> t = *(const vec_t<double, L> *)(vm + (size_t)f * nz + k0);
#pragma unroll
            for (int l = 0; l < L; ++l) x[l] = (S)t[l];
        } else {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                int k = k0 + l + koff;
                k = k < 0 ? 0 : (k >= nz ? nz - 1 : k);
                x[l] = (S)vm[(size_t)f * nz + k];
            }
        }
    }
};

// Moves within a segment: shift_up<N> gives lane p the value of lane p - N,
// shift_down<N> that of lane p + N; lanes whose source lies outside the
// segment keep their own value.  A 16-lane segment is one DPP row, so the
// move is a DPP row shift (row_shr / row_shl), a vector ALU operation; a
// general shuffle goes through the LDS crossbar (ds_bpermute), whose waits
// also wait for outstanding flat memory loads.  32-lane segments cross rows
// and keep the shuffle.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_row(unsigned x)
{
    return (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T x)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_row<CTRL>(__builtin_bit_cast(unsigned, x)));
    } else {
        static_assert(sizeof(T) == 8, "32- or 64-bit values");
        const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
        const unsigned lo = dpp_row<CTRL>((unsigned)u), hi = dpp_row<CTRL>((unsigned)(u >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}
template <int N, int SG = SEG, bool DPP = (SG == 16), typename T>
__device__ __forceinline__ T shift_up(T x)
{
    static_assert(N >= 1 && N < SG && (!DPP || SG == 16), "shift within the segment");
    if constexpr (DPP) return dpp_move<0x110 + N>(x);   // row_shr:N
    else return __shfl_up(x, (unsigned)N, SG);
}
template <int N, int SG = SEG, bool DPP = (SG == 16), typename T>
__device__ __forceinline__ T shift_down(T x)
{
    static_assert(N >= 1 && N < SG && (!DPP || SG == 16), "shift within the segment");
    if constexpr (DPP) return dpp_move<0x100 + N>(x);   // row_shl:N
    else return __shfl_down(x, (unsigned)N, SG);
}
// value of lane p-1 (lane 0 keeps its own) / of lane p+1 (the segment's last
// lane keeps its own)
template <int SG = SEG, bool DPP = (SG == 16), typename T>
__device__ __forceinline__ T from_below(T x) { return shift_up<1, SG, DPP>(x); }
template <int SG = SEG, bool DPP = (SG == 16), typename T>
__device__ __forceinline__ T from_above(T x) { return shift_down<1, SG, DPP>(x); }

// e[0..L+3] = levels k0-2 .. k0+L+1 of a per-lane array x.  Below the column
// the bottom value is repeated (zero-gradient ghost); above it, either the top
// value is repeated (cell quantities) or zero is used (level-face quantities,
// whose face nz is the rigid lid).
template <int SG = SEG, typename T, int L>
__device__ __forceinline__ void extend2(const T (&x)[L], T (&e)[L + 4], int p, bool zero_top)
{
    const T b2 = from_below<SG>(x[L - 2]);
    const T b1 = from_below<SG>(x[L - 1]);
    const T a0 = from_above<SG>(x[0]);
    const T a1 = from_above<SG>(x[1]);
    const bool bot = (p == 0), top = (p == SG - 1);
    e[0] = bot ? x[0] : b2;
    e[1] = bot ? x[0] : b1;
#pragma unroll
    for (int l = 0; l < L; ++l) e[2 + l] = x[l];
    const T topv = zero_top ? T(0) : x[L - 1];
    e[L + 2] = top ? topv : a0;
    e[L + 3] = top ? topv : a1;
}

// --------------------------------------------------------------------------
// slow sweep, part 1: specific velocities, theta and stage coefficients
// --------------------------------------------------------------------------
template <typename T, class Lay, int L, bool TR, int SG>
__device__ __forceinline__ void prep_body(
    const Lane<Lay, L, SG> &ln, const double *__restrict__ vm, const double *__restrict__ geo,
    const T *__restrict__ rref3, const T *__restrict__ rtref3, const T *__restrict__ pref3,
    const T *__restrict__ rp, const T *__restrict__ U, const T *__restrict__ V,
    const T *__restrict__ W, const T *__restrict__ tp, T *__restrict__ uo, T *__restrict__ vo,
    T *__restrict__ wo, T *__restrict__ tho, T *__restrict__ P0o, T *__restrict__ Cso,
    T *__restrict__ omo)
{
    T r0[L], rw[L], rs[L], Uc[L], Vc[L], Wc[L], tc[L];
    ln.load(rp, 0, 0, r0);
    ln.load(rp, -1, 0, rw);
    ln.load(rp, 0, -1, rs);
    // over terrain the neighbours read U and V too (for Omega)
    ln.template load<!TR>(U, 0, 0, Uc);
    ln.template load<!TR>(V, 0, 0, Vc);
    ln.template load<true>(W, 0, 0, Wc);
    ln.template load<true>(tp, 0, 0, tc);
    T rref[L], rtref[L], pref[L], a[L], b[L];
    ln.vmet(vm, VM_A, a);
    ln.vmet(vm, VM_B, b);
    if constexpr (TR) {
        T rrw[L], rrs[L];
        ln.load(rref3, 0, 0, rref);
        ln.load(rref3, -1, 0, rrw);
        ln.load(rref3, 0, -1, rrs);
        ln.template load<true>(rtref3, 0, 0, rtref);
        ln.template load<true>(pref3, 0, 0, pref);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            r0[l] = rref[l] + r0[l];
            rw[l] = rrw[l] + rw[l];
            rs[l] = rrs[l] + rs[l];
        }
    } else {
        ln.vmet(vm, VM_RHO, rref);
        ln.vmet(vm, VM_RT, rtref);
        ln.vmet(vm, VM_P, pref);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            r0[l] = rref[l] + r0[l];
            rw[l] = rref[l] + rw[l];
            rs[l] = rref[l] + rs[l];
        }
    }
    const T rbelow = from_below<SG>(r0[L - 1]);
    T u[L], v[L], w[L], th[L], P0[L], Cs[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int k = ln.k0 + l;
        u[l] = Uc[l] / (T(0.5) * (rw[l] + r0[l]));
        v[l] = Vc[l] / (T(0.5) * (rs[l] + r0[l]));
        const T rb = (l == 0) ? rbelow : r0[l - 1];
        w[l] = (k == 0) ? T(0) : Wc[l] / (a[l] * r0[l] + b[l] * rb);
        th[l] = (rtref[l] + tc[l]) / r0[l];
        const T pps = pref[l] * xexpm1(T(kGamma) * xlog1p(tc[l] / rtref[l]));
        const T cs = T(kGamma) * (pref[l] + pps) / (rtref[l] + tc[l]);
        Cs[l] = cs;
        P0[l] = pps - cs * tc[l];
    }
    ln.store(uo, u);
    ln.store(vo, v);
    ln.store(wo, w);
    ln.store(tho, th);
    ln.store(P0o, P0);
    ln.store(Cso, Cs);
    if constexpr (TR) {
        // flux through the zeta surfaces: Omega = W - (1 - zeta/H) * (slope-
        // weighted U and V averaged to the column centre, then linearly to
        // the level face); zero on the bottom lid
        T U1[L], V1[L], df[L];
        ln.load(U, 1, 0, U1);
        ln.load(V, 0, 1, V1);
        ln.vmet(vm, VM_DF, df);
        const T su0 = (T)ln.geo(geo, GEO_SU, 0, 0), su1 = (T)ln.geo(geo, GEO_SU, 1, 0);
        const T sv0 = (T)ln.geo(geo, GEO_SV, 0, 0), sv1 = (T)ln.geo(geo, GEO_SV, 0, 1);
        T mx[L], my[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            mx[l] = T(0.5) * (su0 * Uc[l] + su1 * U1[l]);
            my[l] = T(0.5) * (sv0 * Vc[l] + sv1 * V1[l]);
        }
        const T mxb = from_below<SG>(mx[L - 1]), myb = from_below<SG>(my[L - 1]);
        T om[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = ln.k0 + l;
            const T mxm = (l == 0) ? mxb : mx[l - 1];
            const T mym = (l == 0) ? myb : my[l - 1];
            const T e = df[l] * ((a[l] * mx[l] + b[l] * mxm) + (a[l] * my[l] + b[l] * mym));
            om[l] = (k == 0) ? T(0) : Wc[l] - e;
        }
        ln.store(omo, om);
    }
}

template <typename T, class Lay, int L, bool TR, int SG>
__global__ __launch_bounds__(threads_of<SG>()) void k_slow_prep(Group gr)
{
    const Where wh = locate<SG>(gr);
    if (!wh.active) return;
    const MemberDev *m = wh.m;
    const Lane<Lay, L, SG> ln(m->nx, m->ny, m->nz, wh.i, wh.j);
    prep_body<T, Lay, L, TR, SG>(ln, m->vm, m->geo, (const T *)m->ref[0], (const T *)m->ref[1],
                             (const T *)m->ref[2], (const T *)buf(m, gr.src, 0),
                             (const T *)buf(m, gr.src, 1), (const T *)buf(m, gr.src, 2),
                             (const T *)buf(m, gr.src, 3), (const T *)buf(m, gr.src, 4),
                             (T *)m->spec[0], (T *)m->spec[1], (T *)m->spec[2], (T *)m->slow[4],
                             (T *)m->slow[5], (T *)m->slow[6], (T *)m->spec[3]);
}

// --------------------------------------------------------------------------
// slow sweep, part 2: advective tendencies S_U, S_V, S_W and R_Theta
// --------------------------------------------------------------------------
// Over terrain (TR) every horizontal mass flux carries the face Jacobian,
// the momentum control volumes take means of the cell-face fluxes, the
// vertical mass flux is Omega (Wz = Omega, else Wz = W) and each tendency is
// divided by the Jacobian of its control volume.
template <typename T, class Lay, int L, bool TR, int SG>
__device__ __forceinline__ void slow_su(const Lane<Lay, L, SG> &ln, T rdx, T rdy, const T (&rdz)[L],
                                        const double *__restrict__ geo, const T *__restrict__ U,
                                        const T *__restrict__ V, const T *__restrict__ Wz,
                                        const T *__restrict__ uu, T *__restrict__ SU)
{
    T ux[5][L], uy[4][L];
#pragma unroll
    for (int d = 0; d < 5; ++d) ln.load(uu, d - 2, 0, ux[d]);
    ln.load(uu, 0, -2, uy[0]);
    ln.load(uu, 0, -1, uy[1]);
    ln.load(uu, 0, 1, uy[2]);
    ln.load(uu, 0, 2, uy[3]);
    T Um[L], U0[L], Up[L], Vw0[L], V00[L], Vw1[L], V01[L], Wm[L], W0[L];
    ln.load(U, -1, 0, Um);
    ln.load(U, 0, 0, U0);
    ln.load(U, 1, 0, Up);
    ln.load(V, -1, 0, Vw0);
    ln.load(V, 0, 0, V00);
    ln.load(V, -1, 1, Vw1);
    ln.load(V, 0, 1, V01);
    ln.load(Wz, -1, 0, Wm);
    ln.load(Wz, 0, 0, W0);
    T jum = T(1), ju0 = T(1), jup = T(1), jvw0 = T(1), jv00 = T(1), jvw1 = T(1), jv01 = T(1);
    if constexpr (TR) {
        jum = (T)ln.geo(geo, GEO_JU, -1, 0);
        ju0 = (T)ln.geo(geo, GEO_JU, 0, 0);
        jup = (T)ln.geo(geo, GEO_JU, 1, 0);
        jvw0 = (T)ln.geo(geo, GEO_JV, -1, 0);
        jv00 = (T)ln.geo(geo, GEO_JV, 0, 0);
        jvw1 = (T)ln.geo(geo, GEO_JV, -1, 1);
        jv01 = (T)ln.geo(geo, GEO_JV, 0, 1);
    }
    T ue[L + 4];
    extend2<SG>(ux[2], ue, ln.p, false);
    const bool top = (ln.p == SG - 1);
    // fluxes through the lane's level faces k0 .. k0+L-1; face k0+L is the
    // first face of the lane above (the rigid lid for the top lane)
    T fz[L + 1];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const T m = T(0.5) * (Wm[l] + W0[l]);
        const T q = kface(ue[l], ue[l + 1], ue[l + 2], ue[l + 3], m);
        fz[l] = (ln.k0 + l == 0) ? T(0) : m * q;
    }
    const T fz_a = from_above<SG>(fz[0]);
    fz[L] = top ? T(0) : fz_a;
    T out[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        T m0, m1, n0, n1;
        if constexpr (TR) {
            m0 = T(0.5) * (jum * Um[l] + ju0 * U0[l]);
            m1 = T(0.5) * (ju0 * U0[l] + jup * Up[l]);
            n0 = T(0.5) * (jvw0 * Vw0[l] + jv00 * V00[l]);
            n1 = T(0.5) * (jvw1 * Vw1[l] + jv01 * V01[l]);
        } else {
            m0 = T(0.5) * (Um[l] + U0[l]);
            m1 = T(0.5) * (U0[l] + Up[l]);
            n0 = T(0.5) * (Vw0[l] + V00[l]);
            n1 = T(0.5) * (Vw1[l] + V01[l]);
        }
        const T fx0 = m0 * kface(ux[0][l], ux[1][l], ux[2][l], ux[3][l], m0);
        const T fx1 = m1 * kface(ux[1][l], ux[2][l], ux[3][l], ux[4][l], m1);
        const T fy0 = n0 * kface(uy[0][l], uy[1][l], ux[2][l], uy[2][l], n0);
        const T fy1 = n1 * kface(uy[1][l], ux[2][l], uy[2][l], uy[3][l], n1);
        const T sum = (fx1 - fx0) * rdx + (fy1 - fy0) * rdy + (fz[l + 1] - fz[l]) * rdz[l];
        if constexpr (TR) out[l] = -sum / ju0;
        else out[l] = -sum;
    }
    ln.store(SU, out);
}

template <typename T, class Lay, int L, bool TR, int SG>
__device__ __forceinline__ void slow_sv(const Lane<Lay, L, SG> &ln, T rdx, T rdy, const T (&rdz)[L],
                                        const double *__restrict__ geo, const T *__restrict__ U,
                                        const T *__restrict__ V, const T *__restrict__ Wz,
                                        const T *__restrict__ vv, T *__restrict__ SV)
{
    T vy[5][L], vx[4][L];
#pragma unroll
    for (int d = 0; d < 5; ++d) ln.load(vv, 0, d - 2, vy[d]);
    ln.load(vv, -2, 0, vx[0]);
    ln.load(vv, -1, 0, vx[1]);
    ln.load(vv, 1, 0, vx[2]);
    ln.load(vv, 2, 0, vx[3]);
    T Vm[L], V0[L], Vp[L], Us0[L], U00[L], Us1[L], U10[L], Wm[L], W0[L];
    ln.load(V, 0, -1, Vm);
    ln.load(V, 0, 0, V0);
    ln.load(V, 0, 1, Vp);
    ln.load(U, 0, -1, Us0);
    ln.load(U, 0, 0, U00);
    ln.load(U, 1, -1, Us1);
    ln.load(U, 1, 0, U10);
    ln.load(Wz, 0, -1, Wm);
    ln.load(Wz, 0, 0, W0);
    T jvm = T(1), jv0 = T(1), jvp = T(1), jus0 = T(1), ju00 = T(1), jus1 = T(1), ju10 = T(1);
    if constexpr (TR) {
        jvm = (T)ln.geo(geo, GEO_JV, 0, -1);
        jv0 = (T)ln.geo(geo, GEO_JV, 0, 0);
        jvp = (T)ln.geo(geo, GEO_JV, 0, 1);
        jus0 = (T)ln.geo(geo, GEO_JU, 0, -1);
        ju00 = (T)ln.geo(geo, GEO_JU, 0, 0);
        jus1 = (T)ln.geo(geo, GEO_JU, 1, -1);
        ju10 = (T)ln.geo(geo, GEO_JU, 1, 0);
    }
    T ve[L + 4];
    extend2<SG>(vy[2], ve, ln.p, false);
    const bool top = (ln.p == SG - 1);
    // fluxes through the lane's level faces k0 .. k0+L-1; face k0+L is the
    // first face of the lane above (the rigid lid for the top lane)
    T fz[L + 1];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const T m = T(0.5) * (Wm[l] + W0[l]);
        const T q = kface(ve[l], ve[l + 1], ve[l + 2], ve[l + 3], m);
        fz[l] = (ln.k0 + l == 0) ? T(0) : m * q;
    }
    const T fz_a = from_above<SG>(fz[0]);
    fz[L] = top ? T(0) : fz_a;
    T out[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        T m0, m1, n0, n1;
        if constexpr (TR) {
            m0 = T(0.5) * (jus0 * Us0[l] + ju00 * U00[l]);
            m1 = T(0.5) * (jus1 * Us1[l] + ju10 * U10[l]);
            n0 = T(0.5) * (jvm * Vm[l] + jv0 * V0[l]);
            n1 = T(0.5) * (jv0 * V0[l] + jvp * Vp[l]);
        } else {
            m0 = T(0.5) * (Us0[l] + U00[l]);
            m1 = T(0.5) * (Us1[l] + U10[l]);
            n0 = T(0.5) * (Vm[l] + V0[l]);
            n1 = T(0.5) * (V0[l] + Vp[l]);
        }
        const T fx0 = m0 * kface(vx[0][l], vx[1][l], vy[2][l], vx[2][l], m0);
        const T fx1 = m1 * kface(vx[1][l], vy[2][l], vx[2][l], vx[3][l], m1);
        const T fy0 = n0 * kface(vy[0][l], vy[1][l], vy[2][l], vy[3][l], n0);
        const T fy1 = n1 * kface(vy[1][l], vy[2][l], vy[3][l], vy[4][l], n1);
        const T sum = (fx1 - fx0) * rdx + (fy1 - fy0) * rdy + (fz[l + 1] - fz[l]) * rdz[l];
        if constexpr (TR) out[l] = -sum / jv0;
        else out[l] = -sum;
    }
    ln.store(SV, out);
}

template <typename T, class Lay, int L, bool TR, int SG>
__device__ __forceinline__ void slow_sw(const Lane<Lay, L, SG> &ln, T rdx, T rdy,
                                        const double *__restrict__ vm, const double *__restrict__ geo,
                                        const T *__restrict__ U, const T *__restrict__ V,
                                        const T *__restrict__ Wz, const T *__restrict__ ww,
                                        T *__restrict__ SW)
{
    T wx[5][L], wy[4][L];
#pragma unroll
    for (int d = 0; d < 5; ++d) ln.load(ww, d - 2, 0, wx[d]);
    ln.load(ww, 0, -2, wy[0]);
    ln.load(ww, 0, -1, wy[1]);
    ln.load(ww, 0, 1, wy[2]);
    ln.load(ww, 0, 2, wy[3]);
    T U0[L], U1[L], V0[L], V1[L], W0[L];
    ln.load(U, 0, 0, U0);
    ln.load(U, 1, 0, U1);
    ln.load(V, 0, 0, V0);
    ln.load(V, 0, 1, V1);
    ln.load(Wz, 0, 0, W0);
    // level below the lane's first level (unused on the bottom level face)
    const T U0b = from_below<SG>(U0[L - 1]), U1b = from_below<SG>(U1[L - 1]);
    const T V0b = from_below<SG>(V0[L - 1]), V1b = from_below<SG>(V1[L - 1]);
    T we[L + 4], We[L + 4];
    extend2<SG>(wx[2], we, ln.p, true);
    extend2<SG>(W0, We, ln.p, true);
    T rdzf[L];
    ln.template vmet<T, TR>(vm, VM_RDZF, rdzf);
    T ju0 = T(1), ju1 = T(1), jv0 = T(1), jv1 = T(1), jc = T(1);
    if constexpr (TR) {
        ju0 = (T)ln.geo(geo, GEO_JU, 0, 0);
        ju1 = (T)ln.geo(geo, GEO_JU, 1, 0);
        jv0 = (T)ln.geo(geo, GEO_JV, 0, 0);
        jv1 = (T)ln.geo(geo, GEO_JV, 0, 1);
        jc = (T)ln.geo(geo, GEO_J, 0, 0);
    }
    // vertical fluxes at the cell centres cc = k0-1 .. k0+L-1; the first is
    // the last of the lane below (unused on the bottom lane, whose first
    // level face is the lower lid)
    T fz[L + 1];
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        const T m = T(0.5) * (We[l + 1] + We[l + 2]);
        fz[l] = m * kface(we[l], we[l + 1], we[l + 2], we[l + 3], m);
    }
    fz[0] = from_below<SG>(fz[L]);
    T out[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int k = ln.k0 + l;
        const T u0b = (l == 0) ? U0b : U0[l - 1];
        const T u1b = (l == 0) ? U1b : U1[l - 1];
        const T v0b = (l == 0) ? V0b : V0[l - 1];
        const T v1b = (l == 0) ? V1b : V1[l - 1];
        T m0, m1, n0, n1;
        if constexpr (TR) {
            m0 = T(0.5) * (ju0 * u0b + ju0 * U0[l]);
            m1 = T(0.5) * (ju1 * u1b + ju1 * U1[l]);
            n0 = T(0.5) * (jv0 * v0b + jv0 * V0[l]);
            n1 = T(0.5) * (jv1 * v1b + jv1 * V1[l]);
        } else {
            m0 = T(0.5) * (u0b + U0[l]);
            m1 = T(0.5) * (u1b + U1[l]);
            n0 = T(0.5) * (v0b + V0[l]);
            n1 = T(0.5) * (v1b + V1[l]);
        }
        const T fx0 = m0 * kface(wx[0][l], wx[1][l], wx[2][l], wx[3][l], m0);
        const T fx1 = m1 * kface(wx[1][l], wx[2][l], wx[3][l], wx[4][l], m1);
        const T fy0 = n0 * kface(wy[0][l], wy[1][l], wx[2][l], wy[2][l], n0);
        const T fy1 = n1 * kface(wy[1][l], wx[2][l], wy[2][l], wy[3][l], n1);
        const T sum = (fx1 - fx0) * rdx + (fy1 - fy0) * rdy + (fz[l + 1] - fz[l]) * rdzf[l];
        T s;
        if constexpr (TR) s = -sum / jc;
        else s = -sum;
        out[l] = (k == 0) ? T(0) : s;
    }
    ln.store(SW, out);
}

template <typename T, class Lay, int L, bool TR, int SG>
__device__ __forceinline__ void slow_rt(const Lane<Lay, L, SG> &ln, T rdx, T rdy, const T (&rdz)[L],
                                        const double *__restrict__ vm, const double *__restrict__ geo,
                                        const T *__restrict__ U, const T *__restrict__ V,
                                        const T *__restrict__ Wz, const T *__restrict__ th,
                                        T *__restrict__ RT)
{
    T tx[5][L], ty[4][L];
#pragma unroll
    for (int d = 0; d < 5; ++d) ln.load(th, d - 2, 0, tx[d]);
    ln.load(th, 0, -2, ty[0]);
    ln.load(th, 0, -1, ty[1]);
    ln.load(th, 0, 1, ty[2]);
    ln.load(th, 0, 2, ty[3]);
    T U0[L], U1[L], V0[L], V1[L], W0[L];
    ln.load(U, 0, 0, U0);
    ln.load(U, 1, 0, U1);
    ln.load(V, 0, 0, V0);
    ln.load(V, 0, 1, V1);
    ln.load(Wz, 0, 0, W0);
    T ju0 = T(1), ju1 = T(1), jv0 = T(1), jv1 = T(1), jc = T(1);
    if constexpr (TR) {
        ju0 = (T)ln.geo(geo, GEO_JU, 0, 0);
        ju1 = (T)ln.geo(geo, GEO_JU, 1, 0);
        jv0 = (T)ln.geo(geo, GEO_JV, 0, 0);
        jv1 = (T)ln.geo(geo, GEO_JV, 0, 1);
        jc = (T)ln.geo(geo, GEO_J, 0, 0);
    }
    T te[L + 4];
    extend2<SG>(tx[2], te, ln.p, false);
    const bool top = (ln.p == SG - 1);
    // the flat slow flux reads the float64 table (measured: the float32 copy
    // changes its schedule and costs 7% there, while it saves 8% over terrain)
    T a[L], b[L];
    if constexpr (TR) {
        ln.vmet(vm, VM_A, a);
        ln.vmet(vm, VM_B, b);
    } else {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            a[l] = (T)vm[(size_t)VM_A * ln.nz + ln.k0 + l];
            b[l] = (T)vm[(size_t)VM_B * ln.nz + ln.k0 + l];
        }
    }
    // fluxes through the lane's level faces k0 .. k0+L-1; face k0+L is the
    // first face of the lane above (the rigid lid for the top lane)
    T gz[L + 1];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const T m = W0[l];
        const T tl = kface(te[l], te[l + 1], te[l + 2], te[l + 3], m);
        const T tcen = a[l] * te[l + 2] + b[l] * te[l + 1];
        gz[l] = (ln.k0 + l == 0) ? T(0) : m * (tl - tcen);
    }
    const T gz_a = from_above<SG>(gz[0]);
    gz[L] = top ? T(0) : gz_a;
    T out[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        T m0 = U0[l], m1 = U1[l], n0 = V0[l], n1 = V1[l];
        if constexpr (TR) {
            m0 = ju0 * m0;
            m1 = ju1 * m1;
            n0 = jv0 * n0;
            n1 = jv1 * n1;
        }
        const T g0 = m0 * (kface(tx[0][l], tx[1][l], tx[2][l], tx[3][l], m0) -
                           T(0.5) * (tx[1][l] + tx[2][l]));
        const T g1 = m1 * (kface(tx[1][l], tx[2][l], tx[3][l], tx[4][l], m1) -
                           T(0.5) * (tx[2][l] + tx[3][l]));
        const T h0 = n0 * (kface(ty[0][l], ty[1][l], tx[2][l], ty[2][l], n0) -
                           T(0.5) * (ty[1][l] + tx[2][l]));
        const T h1 = n1 * (kface(ty[1][l], tx[2][l], ty[2][l], ty[3][l], n1) -
                           T(0.5) * (tx[2][l] + ty[2][l]));
        const T sum = (g1 - g0) * rdx + (h1 - h0) * rdy + (gz[l + 1] - gz[l]) * rdz[l];
        if constexpr (TR) out[l] = -sum / jc;
        else out[l] = -sum;
    }
    ln.store(RT, out);
}

template <typename T, class Lay, int L, bool TR, int SG>
__device__ __forceinline__ void flux_body(
    const Lane<Lay, L, SG> &ln, const double *__restrict__ vm, const double *__restrict__ geo, T rdx,
    T rdy, const T *__restrict__ U, const T *__restrict__ V, const T *__restrict__ Wz,
    const T *__restrict__ uu, const T *__restrict__ vv, const T *__restrict__ ww,
    const T *__restrict__ th, T *__restrict__ SU, T *__restrict__ SV, T *__restrict__ SW,
    T *__restrict__ RT)
{
    T rdz[L];
    ln.template vmet<T, TR>(vm, VM_RDZ, rdz);
    slow_su<T, Lay, L, TR, SG>(ln, rdx, rdy, rdz, geo, U, V, Wz, uu, SU);
    slow_sv<T, Lay, L, TR, SG>(ln, rdx, rdy, rdz, geo, U, V, Wz, vv, SV);
    slow_sw<T, Lay, L, TR, SG>(ln, rdx, rdy, vm, geo, U, V, Wz, ww, SW);
    slow_rt<T, Lay, L, TR, SG>(ln, rdx, rdy, rdz, vm, geo, U, V, Wz, th, RT);
}

// The flat float32 flux kernel with 4 contiguous levels per lane fits 4 waves
// per SIMD without spilling (measured 0.977 ms against 1.027 ms at its natural
// 3; the i-fastest form would spill there);
// the other variants keep the compiler's choice.
template <typename T, class Lay, int L, bool TR>
constexpr int flux_waves() { return (sizeof(T) == 4 && L == 4 && !TR && Lay::kContig) ? 4 : 1; }

template <typename T, class Lay, int L, bool TR, int SG>
__global__ __launch_bounds__(threads_of<SG>())
__attribute__((amdgpu_waves_per_eu(flux_waves<T, Lay, L, TR>())))
void k_slow_flux(Group gr)
{
    const Where wh = locate<SG>(gr);
    if (!wh.active) return;
    const MemberDev *m = wh.m;
    const Lane<Lay, L, SG> ln(m->nx, m->ny, m->nz, wh.i, wh.j);
    flux_body<T, Lay, L, TR, SG>(ln, m->vm, m->geo, (T)m->rdx, (T)m->rdy, (const T *)buf(m, gr.src, 1),
                             (const T *)buf(m, gr.src, 2),
                             TR ? (const T *)m->spec[3] : (const T *)buf(m, gr.src, 3),
                             (const T *)m->spec[0], (const T *)m->spec[1], (const T *)m->spec[2],
                             (const T *)m->slow[4], (T *)m->slow[0], (T *)m->slow[1],
                             (T *)m->slow[2], (T *)m->slow[3]);
}

// --------------------------------------------------------------------------
// slow sweep, part 2, in runs along x
// --------------------------------------------------------------------------
// Each x-face is shared by two columns: above, both evaluate it, so the Koren
// value and mass flux of every x-face (one of a cell's five faces, for each
// of the four tendencies) is computed twice, and every column loads its four
// x-neighbours of each advected quantity.  Here a segment walks a run of
// gr.run consecutive columns along x and carries over, in registers, the
// flux through the face it shares with the next column, the x-window of the
// four advected quantities and the mass-flux operands of that face: a column
// loads one new x-neighbour per quantity.  Every face flux takes the same
// operands in the same order as above, so the tendencies are bitwise equal.
// A block covers (1 << ti_log2) runs along x by 16 >> ti_log2 rows.
template <int SG>
__device__ __forceinline__ Where locate_run(const Group &gr)
{
    Where w;
    constexpr int sp = split_of<SG>();
    const int b0 = block_order(gr, gr.nblocks * sp);
    const int b = b0 / sp;
    int t = b, id = gr.first;
    if (gr.nm > 1) {
        const unsigned v = gr.blk[b];
        t = (int)(v & 0xFFFFFFu);
        id = (int)(v >> 24);
    }
    w.m = gr.mem + id;
    const int ti = 1 << gr.ti_log2, tj = kColsPerBlock >> gr.ti_log2;
    const int span = ti * gr.run;
    const int tiles_x = (w.m->nx + span - 1) / span;
    const int c = (int)threadIdx.x / SG + (b0 % sp) * (kColsPerBlock / sp);
    w.i = (t % tiles_x) * span + (c & (ti - 1)) * gr.run;
    w.j = (t / tiles_x) * tj + (c >> gr.ti_log2);
    w.active = w.i < w.m->nx && w.j < w.m->ny;
    return w;
}

template <typename T, class Lay, int L, bool TR, int SG>
__global__ __launch_bounds__(threads_of<SG>())
void k_slow_flux_run(Group gr)
{
    const Where wh = locate_run<SG>(gr);
    if (!wh.active) return;
    const MemberDev *m = wh.m;
    Lane<Lay, L, SG> ln(m->nx, m->ny, m->nz, wh.i, wh.j);
    const double *__restrict__ vm = m->vm;
    const double *__restrict__ geo = m->geo;
    const T rdx = (T)m->rdx, rdy = (T)m->rdy;
    const T *__restrict__ U = (const T *)buf(m, gr.src, 1);
    const T *__restrict__ V = (const T *)buf(m, gr.src, 2);
    const T *__restrict__ Wz = TR ? (const T *)m->spec[3] : (const T *)buf(m, gr.src, 3);
    const T *__restrict__ uu = (const T *)m->spec[0];
    const T *__restrict__ vv = (const T *)m->spec[1];
    const T *__restrict__ ww = (const T *)m->spec[2];
    const T *__restrict__ th = (const T *)m->slow[4];
    T *__restrict__ SU = (T *)m->slow[0];
    T *__restrict__ SV = (T *)m->slow[1];
    T *__restrict__ SW = (T *)m->slow[2];
    T *__restrict__ RT = (T *)m->slow[3];
    const int iend = min(wh.i + gr.run, m->nx);
    const bool top = (ln.p == SG - 1);

    // per-level constants of the lane's levels
    T rdz[L], rdzf[L], a[L], b[L];
    ln.template vmet<T, TR>(vm, VM_RDZ, rdz);
    ln.template vmet<T, TR>(vm, VM_RDZF, rdzf);
    ln.template vmet<T, TR>(vm, VM_A, a);
    ln.template vmet<T, TR>(vm, VM_B, b);

    // Carried from column i-1 to column i: the x-windows q(i-1), q(i),
    // q(i+1) of u, v, w, theta (slot 3 takes q(i+2)); the fluxes through the
    // face i-1/2; U(i, j), V(i-1, j), V(i-1, j+1), Wz(i-1, j) and over
    // terrain the face Jacobians of those points.
    T uw[4][L], vw[4][L], wq[4][L], tw[4][L];
    T fxU[L], fxV[L], fxW[L], fxT[L];
    T Uc[L], Vw0[L], Vw1[L], Wl[L];
    T ju_c = T(1), jvw0 = T(1), jvw1 = T(1);
    {
        // the face i0-1/2, as column i0 - 1 evaluates it as its east face
        T Ul[L], Usc[L], q0[L];
        T jus_c = T(1);
        ln.load(U, -1, 0, Ul);
        ln.load(U, 0, 0, Uc);
        ln.load(U, 0, -1, Usc);
        ln.load(V, -1, 0, Vw0);
        ln.load(V, -1, 1, Vw1);
        ln.load(Wz, -1, 0, Wl);
        T jul = T(1);
        if constexpr (TR) {
            jul = (T)ln.geo(geo, GEO_JU, -1, 0);
            ju_c = (T)ln.geo(geo, GEO_JU, 0, 0);
            jus_c = (T)ln.geo(geo, GEO_JU, 0, -1);
            jvw0 = (T)ln.geo(geo, GEO_JV, -1, 0);
            jvw1 = (T)ln.geo(geo, GEO_JV, -1, 1);
        }
        const T Ucb = from_below<SG>(Uc[L - 1]);
        ln.load(uu, -2, 0, q0);
#pragma unroll
        for (int d = 0; d < 3; ++d) ln.load(uu, d - 1, 0, uw[d]);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const T mx = TR ? T(0.5) * (jul * Ul[l] + ju_c * Uc[l]) : T(0.5) * (Ul[l] + Uc[l]);
            fxU[l] = mx * kface(q0[l], uw[0][l], uw[1][l], uw[2][l], mx);
        }
        ln.load(vv, -2, 0, q0);
#pragma unroll
        for (int d = 0; d < 3; ++d) ln.load(vv, d - 1, 0, vw[d]);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const T mx = TR ? T(0.5) * (jus_c * Usc[l] + ju_c * Uc[l]) : T(0.5) * (Usc[l] + Uc[l]);
            fxV[l] = mx * kface(q0[l], vw[0][l], vw[1][l], vw[2][l], mx);
        }
        ln.load(ww, -2, 0, q0);
#pragma unroll
        for (int d = 0; d < 3; ++d) ln.load(ww, d - 1, 0, wq[d]);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const T ub = (l == 0) ? Ucb : Uc[l - 1];
            const T mx = TR ? T(0.5) * (ju_c * ub + ju_c * Uc[l]) : T(0.5) * (ub + Uc[l]);
            fxW[l] = mx * kface(q0[l], wq[0][l], wq[1][l], wq[2][l], mx);
        }
        ln.load(th, -2, 0, q0);
#pragma unroll
        for (int d = 0; d < 3; ++d) ln.load(th, d - 1, 0, tw[d]);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const T mx = TR ? ju_c * Uc[l] : Uc[l];
            fxT[l] = mx * (kface(q0[l], tw[0][l], tw[1][l], tw[2][l], mx) -
                           T(0.5) * (tw[0][l] + tw[1][l]));
        }
    }

    for (int i = wh.i; i < iend; ++i) {
        ln.i = i;
        T Up[L], Usp[L], V00[L], V01[L], Vm[L], W0[L], Wsm[L];
        ln.load(uu, 2, 0, uw[3]);
        ln.load(vv, 2, 0, vw[3]);
        ln.load(ww, 2, 0, wq[3]);
        ln.load(th, 2, 0, tw[3]);
        ln.load(U, 1, 0, Up);
        ln.load(U, 1, -1, Usp);
        ln.load(V, 0, 0, V00);
        ln.load(V, 0, 1, V01);
        ln.load(V, 0, -1, Vm);
        ln.load(Wz, 0, 0, W0);
        ln.load(Wz, 0, -1, Wsm);
        T jup = T(1), jusp = T(1), jv00 = T(1), jv01 = T(1), jvm = T(1), jc = T(1);
        if constexpr (TR) {
            jup = (T)ln.geo(geo, GEO_JU, 1, 0);
            jusp = (T)ln.geo(geo, GEO_JU, 1, -1);
            jv00 = (T)ln.geo(geo, GEO_JV, 0, 0);
            jv01 = (T)ln.geo(geo, GEO_JV, 0, 1);
            jvm = (T)ln.geo(geo, GEO_JV, 0, -1);
            jc = (T)ln.geo(geo, GEO_J, 0, 0);
        }
        // S_U
        {
            T qy[4][L], e[L + 4], fz[L + 1], out[L];
            ln.load(uu, 0, -2, qy[0]);
            ln.load(uu, 0, -1, qy[1]);
            ln.load(uu, 0, 1, qy[2]);
            ln.load(uu, 0, 2, qy[3]);
            extend2<SG>(uw[1], e, ln.p, false);
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const T mz = T(0.5) * (Wl[l] + W0[l]);
                const T q = kface(e[l], e[l + 1], e[l + 2], e[l + 3], mz);
                fz[l] = (ln.k0 + l == 0) ? T(0) : mz * q;
            }
            const T fz_a = from_above<SG>(fz[0]);
            fz[L] = top ? T(0) : fz_a;
#pragma unroll
            for (int l = 0; l < L; ++l) {
                T m1, n0, n1;
                if constexpr (TR) {
                    m1 = T(0.5) * (ju_c * Uc[l] + jup * Up[l]);
                    n0 = T(0.5) * (jvw0 * Vw0[l] + jv00 * V00[l]);
                    n1 = T(0.5) * (jvw1 * Vw1[l] + jv01 * V01[l]);
                } else {
                    m1 = T(0.5) * (Uc[l] + Up[l]);
                    n0 = T(0.5) * (Vw0[l] + V00[l]);
                    n1 = T(0.5) * (Vw1[l] + V01[l]);
                }
                const T fx1 = m1 * kface(uw[0][l], uw[1][l], uw[2][l], uw[3][l], m1);
                const T fy0 = n0 * kface(qy[0][l], qy[1][l], uw[1][l], qy[2][l], n0);
                const T fy1 = n1 * kface(qy[1][l], uw[1][l], qy[2][l], qy[3][l], n1);
                const T sum = (fx1 - fxU[l]) * rdx + (fy1 - fy0) * rdy + (fz[l + 1] - fz[l]) * rdz[l];
                if constexpr (TR) out[l] = -sum / ju_c;
                else out[l] = -sum;
                fxU[l] = fx1;
            }
            ln.store(SU, out);
        }
        // S_V
        {
            T qy[4][L], e[L + 4], fz[L + 1], out[L];
            ln.load(vv, 0, -2, qy[0]);
            ln.load(vv, 0, -1, qy[1]);
            ln.load(vv, 0, 1, qy[2]);
            ln.load(vv, 0, 2, qy[3]);
            extend2<SG>(vw[1], e, ln.p, false);
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const T mz = T(0.5) * (Wsm[l] + W0[l]);
                const T q = kface(e[l], e[l + 1], e[l + 2], e[l + 3], mz);
                fz[l] = (ln.k0 + l == 0) ? T(0) : mz * q;
            }
            const T fz_a = from_above<SG>(fz[0]);
            fz[L] = top ? T(0) : fz_a;
#pragma unroll
            for (int l = 0; l < L; ++l) {
                T m1, n0, n1;
                if constexpr (TR) {
                    m1 = T(0.5) * (jusp * Usp[l] + jup * Up[l]);
                    n0 = T(0.5) * (jvm * Vm[l] + jv00 * V00[l]);
                    n1 = T(0.5) * (jv00 * V00[l] + jv01 * V01[l]);
                } else {
                    m1 = T(0.5) * (Usp[l] + Up[l]);
                    n0 = T(0.5) * (Vm[l] + V00[l]);
                    n1 = T(0.5) * (V00[l] + V01[l]);
                }
                const T fx1 = m1 * kface(vw[0][l], vw[1][l], vw[2][l], vw[3][l], m1);
                const T fy0 = n0 * kface(qy[0][l], qy[1][l], vw[1][l], qy[2][l], n0);
                const T fy1 = n1 * kface(qy[1][l], vw[1][l], qy[2][l], qy[3][l], n1);
                const T sum = (fx1 - fxV[l]) * rdx + (fy1 - fy0) * rdy + (fz[l + 1] - fz[l]) * rdz[l];
                if constexpr (TR) out[l] = -sum / jv00;
                else out[l] = -sum;
                fxV[l] = fx1;
            }
            ln.store(SV, out);
        }
        // S_W (level faces; face 0 is the lower lid)
        {
            T qy[4][L], e[L + 4], We[L + 4], fz[L + 1], out[L];
            ln.load(ww, 0, -2, qy[0]);
            ln.load(ww, 0, -1, qy[1]);
            ln.load(ww, 0, 1, qy[2]);
            ln.load(ww, 0, 2, qy[3]);
            const T U1b = from_below<SG>(Up[L - 1]);
            const T V0b = from_below<SG>(V00[L - 1]), V1b = from_below<SG>(V01[L - 1]);
            extend2<SG>(wq[1], e, ln.p, true);
            extend2<SG>(W0, We, ln.p, true);
#pragma unroll
            for (int l = 1; l <= L; ++l) {
                const T mz = T(0.5) * (We[l + 1] + We[l + 2]);
                fz[l] = mz * kface(e[l], e[l + 1], e[l + 2], e[l + 3], mz);
            }
            fz[0] = from_below<SG>(fz[L]);
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const int k = ln.k0 + l;
                const T u1b = (l == 0) ? U1b : Up[l - 1];
                const T v0b = (l == 0) ? V0b : V00[l - 1];
                const T v1b = (l == 0) ? V1b : V01[l - 1];
                T m1, n0, n1;
                if constexpr (TR) {
                    m1 = T(0.5) * (jup * u1b + jup * Up[l]);
                    n0 = T(0.5) * (jv00 * v0b + jv00 * V00[l]);
                    n1 = T(0.5) * (jv01 * v1b + jv01 * V01[l]);
                } else {
                    m1 = T(0.5) * (u1b + Up[l]);
                    n0 = T(0.5) * (v0b + V00[l]);
                    n1 = T(0.5) * (v1b + V01[l]);
                }
                const T fx1 = m1 * kface(wq[0][l], wq[1][l], wq[2][l], wq[3][l], m1);
                const T fy0 = n0 * kface(qy[0][l], qy[1][l], wq[1][l], qy[2][l], n0);
                const T fy1 = n1 * kface(qy[1][l], wq[1][l], qy[2][l], qy[3][l], n1);
                const T sum = (fx1 - fxW[l]) * rdx + (fy1 - fy0) * rdy + (fz[l + 1] - fz[l]) * rdzf[l];
                T sw;
                if constexpr (TR) sw = -sum / jc;
                else sw = -sum;
                out[l] = (k == 0) ? T(0) : sw;
                fxW[l] = fx1;
            }
            ln.store(SW, out);
        }
        // R_Theta
        {
            T qy[4][L], e[L + 4], gz[L + 1], out[L];
            ln.load(th, 0, -2, qy[0]);
            ln.load(th, 0, -1, qy[1]);
            ln.load(th, 0, 1, qy[2]);
            ln.load(th, 0, 2, qy[3]);
            extend2<SG>(tw[1], e, ln.p, false);
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const T mz = W0[l];
                const T tl = kface(e[l], e[l + 1], e[l + 2], e[l + 3], mz);
                const T tcen = a[l] * e[l + 2] + b[l] * e[l + 1];
                gz[l] = (ln.k0 + l == 0) ? T(0) : mz * (tl - tcen);
            }
            const T gz_a = from_above<SG>(gz[0]);
            gz[L] = top ? T(0) : gz_a;
#pragma unroll
            for (int l = 0; l < L; ++l) {
                T m1 = Up[l], n0 = V00[l], n1 = V01[l];
                if constexpr (TR) {
                    m1 = jup * m1;
                    n0 = jv00 * n0;
                    n1 = jv01 * n1;
                }
                const T g1 = m1 * (kface(tw[0][l], tw[1][l], tw[2][l], tw[3][l], m1) -
                                   T(0.5) * (tw[1][l] + tw[2][l]));
                const T h0 = n0 * (kface(qy[0][l], qy[1][l], tw[1][l], qy[2][l], n0) -
                                   T(0.5) * (qy[1][l] + tw[1][l]));
                const T h1 = n1 * (kface(qy[1][l], tw[1][l], qy[2][l], qy[3][l], n1) -
                                   T(0.5) * (tw[1][l] + qy[2][l]));
                const T sum = (g1 - fxT[l]) * rdx + (h1 - h0) * rdy + (gz[l + 1] - gz[l]) * rdz[l];
                if constexpr (TR) out[l] = -sum / jc;
                else out[l] = -sum;
                fxT[l] = g1;
            }
            ln.store(RT, out);
        }
        // slide the windows to column i + 1
#pragma unroll
        for (int l = 0; l < L; ++l) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                uw[d][l] = uw[d + 1][l];
                vw[d][l] = vw[d + 1][l];
                wq[d][l] = wq[d + 1][l];
                tw[d][l] = tw[d + 1][l];
            }
            Uc[l] = Up[l];
            Vw0[l] = V00[l];
            Vw1[l] = V01[l];
            Wl[l] = W0[l];
        }
        ju_c = jup;
        jvw0 = jv00;
        jvw1 = jv01;
    }
}

// --------------------------------------------------------------------------
// short step: horizontally explicit part, then the column solve
// --------------------------------------------------------------------------

// One step of parallel cyclic reduction at distance s: row p (a x_{p-s} +
// x_p + c x_{p+s} = d, normalised) eliminates its neighbours s rows away.
template <int s, int SG, bool DPP, typename S>
__device__ __forceinline__ void pcr_step(int p, S &a, S &c, S &d)
{
    const bool hasm = p >= s, hasp = p + s < SG;
    const S am = shift_up<s, SG, DPP>(a), cm = shift_up<s, SG, DPP>(c);
    const S dm = shift_up<s, SG, DPP>(d);
    const S ap = shift_down<s, SG, DPP>(a), cp = shift_down<s, SG, DPP>(c);
    const S dp = shift_down<s, SG, DPP>(d);
    const S amv = hasm ? am : S(0), cmv = hasm ? cm : S(0), dmv = hasm ? dm : S(0);
    const S apv = hasp ? ap : S(0), cpv = hasp ? cp : S(0), dpv = hasp ? dp : S(0);
    const S rb2 = solve_rcp(S(1) - a * cmv - c * apv);
    const S dn = (d - a * dmv - c * dpv) * rb2;
    const S an = -a * amv * rb2;
    const S cn = -c * cpv * rb2;
    a = an;
    c = cn;
    d = dn;
}

// The rows come from row(l, a, b, c, d), called once per row in the order
// l = 0 .. L-1 (the lane's last row after the others are eliminated), so a
// row's coefficients exist only while it is being eliminated.
template <typename S, int L, int SG, bool DPP = (SG == 16), class Row>
__device__ __forceinline__ void segment_solve(int p, Row &&row, S (&x)[L])
{
    // interior rows 0..L-2 in terms of X_{p-1} (last unknown of the lane
    // below) and X_p (this lane's last unknown): x_l = xg + xa X_{p-1} + xb X_p
    constexpr int n = L - 1;
    S gp[L], yg[L], ya[L], yb[L];
#pragma unroll
    for (int l = 0; l < n; ++l) {
        S Al, Bl, Cl, Dl;
        row(l, Al, Bl, Cl, Dl);
        const S den = (l == 0) ? Bl : Bl - Al * gp[l - 1];
        const S rden = solve_rcp(den);
        gp[l] = (l < n - 1) ? Cl * rden : S(0);
        const S rg = Dl, ra = (l == 0) ? -Al : S(0), rb = (l == n - 1) ? -Cl : S(0);
        if (l == 0) {
            yg[0] = rg * rden;
            ya[0] = ra * rden;
            yb[0] = rb * rden;
        } else {
            yg[l] = (rg - Al * yg[l - 1]) * rden;
            ya[l] = (ra - Al * ya[l - 1]) * rden;
            yb[l] = (rb - Al * yb[l - 1]) * rden;
        }
    }
#pragma unroll
    for (int l = n - 2; l >= 0; --l) {
        yg[l] = yg[l] - gp[l] * yg[l + 1];
        ya[l] = ya[l] - gp[l] * ya[l + 1];
        yb[l] = yb[l] - gp[l] * yb[l + 1];
    }
    S AL, BL, CL, DL;
    row(L - 1, AL, BL, CL, DL);
    // reduced equation of the lane's last row, in X_{p-1}, X_p, X_{p+1}
    const S ga = from_above<SG, DPP>(ya[0]), gb = from_above<SG, DPP>(yb[0]);
    const S gg = from_above<SG, DPP>(yg[0]);
    const S Ab = AL * ya[n - 1];
    const S Bb = BL + AL * yb[n - 1] + CL * ga;
    const S Cb = CL * gb;
    const S Db = DL - AL * yg[n - 1] - CL * gg;
    const S rB = solve_rcp(Bb);
    S a = Ab * rB, c = Cb * rB, d = Db * rB;
    // parallel cyclic reduction over the SG interface rows
    static_assert(SG == 8 || SG == 16 || SG == 32, "8-, 16- or 32-lane segments");
    if constexpr (DPP) {
        pcr_step<1, SG, true>(p, a, c, d);
        pcr_step<2, SG, true>(p, a, c, d);
        pcr_step<4, SG, true>(p, a, c, d);
        pcr_step<8, SG, true>(p, a, c, d);
    } else {
        // shuffles, in a loop (unrolled by the compiler, which schedules this
        // form with fewer registers than the stepwise one)
#pragma unroll
        for (int s = 1; s < SG; s <<= 1) {
            const bool hasm = p >= s, hasp = p + s < SG;
            const S am = __shfl_up(a, (unsigned)s, SG), cm = __shfl_up(c, (unsigned)s, SG);
            const S dm = __shfl_up(d, (unsigned)s, SG);
            const S ap = __shfl_down(a, (unsigned)s, SG), cp = __shfl_down(c, (unsigned)s, SG);
            const S dp = __shfl_down(d, (unsigned)s, SG);
            const S amv = hasm ? am : S(0), cmv = hasm ? cm : S(0), dmv = hasm ? dm : S(0);
            const S apv = hasp ? ap : S(0), cpv = hasp ? cp : S(0), dpv = hasp ? dp : S(0);
            const S rb2 = solve_rcp(S(1) - a * cmv - c * apv);
            const S dn = (d - a * dmv - c * dpv) * rb2;
            const S an = -a * amv * rb2;
            const S cn = -c * cpv * rb2;
            a = an;
            c = cn;
            d = dn;
        }
    }
    const S X = d;
    const S Xs = from_below<SG, DPP>(X);
    const S Xb = (p == 0) ? S(0) : Xs;
#pragma unroll
    for (int l = 0; l < n; ++l) x[l] = yg[l] + ya[l] * Xb + yb[l] * X;
    x[L - 1] = X;
}

// Occupancy target of the short step (waves per SIMD), chosen so that the
// register budget holds the lane's levels without spilling.  16-lane
// segments: float32 4 (also with the terrain terms or a separate evaluation
// state; 3 with the damping, 2 with two of them besides the terrain), float32
// storage with a float64 solve 4 (3 with the terrain terms or a separate
// evaluation state, 2 with the damping or two extras), 1 for 8 levels per
// lane.  32-lane segments (float64 storage, half the levels per
// lane): 4 with 2 levels per lane (2 with the damping); with 4, 2 (1 with
// the terrain terms or the damping).
template <typename T, typename S, int L, bool TR, bool EV, int SG, bool DP>
constexpr int short_waves()
{
    if (SG == 32) {
        if (L < 4) return DP ? 2 : 4;
        return (sizeof(T) == 8 && (TR || DP)) ? 1 : 2;
    }
    if (L >= 8) return 1;
    const int extra = (TR ? 1 : 0) + (EV ? 1 : 0) + (DP ? 1 : 0);
    if (sizeof(T) == 4 && sizeof(S) == 4) {
        if (extra == 0) return 4;
        if (!DP) return extra == 1 ? 4 : 3;
        return extra == 1 ? 3 : 2;
    }
    if (sizeof(T) == 4) return (DP || extra >= 2) ? 2 : (extra == 0 ? 4 : 3);
    if (TR && L >= 4) return 1;
    return 2;
}

// d p / d zeta at the lane's cell centres from a column's p: the mean of the
// differences over the two level faces of the cell, the one inner face at the
// lowest and highest cell.  rdzf[l] = 1/dzf of face k0+l.
template <int SG, typename T, int L>
__device__ __forceinline__ void ddzeta(const T (&pp)[L], const T (&rdzf)[L], int p, int k0, int nz,
                                       T (&g)[L])
{
    T dn[L];
    const T pb = from_below<SG>(pp[L - 1]);
#pragma unroll
    for (int l = 0; l < L; ++l) dn[l] = (pp[l] - ((l == 0) ? pb : pp[l - 1])) * rdzf[l];
    const T dna = from_above<SG>(dn[0]);
    (void)p;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int k = k0 + l;
        const T up = (l < L - 1) ? dn[l + 1] : dna;
        g[l] = (k == 0) ? up : ((k == nz - 1) ? dn[l] : T(0.5) * (dn[l] + up));
    }
}

// Lateral and upper damping of one field's new values in registers (the
// relaxation of the paper's Listing 1): the target is the boundary state
// interpolated in time, mtratio (ref + bnd1) + tratio (ref + bnd2) - ref
// (ref = 0 for the momenta), and each value with a nonzero rate relaxes
// implicitly, v <- (v + c target) / (1 + c), c = dtau (nu_lat + nu_top).
// W's lowest face (the lid) is left as it is.
// (Set up twice per short step, for U and V and for the vertical fields, so
// that nothing stays live across the column solve.)
template <typename T, int L>
struct DampLane {
    bool any;
    T cf[L], rc[L], mt, tr;   // cf = dtau nu (0: not damped), rc = 1/(1 + cf)
};

template <typename T, class Lay, int L, int SG>
__device__ __forceinline__ DampLane<T, L> damp_setup(const Lane<Lay, L, SG> &ln, const MemberDev *m,
                                                     double t, double dtau)
{
    DampLane<T, L> d;
    const double nl = m->nu_lat[(size_t)ln.j * ln.nx + ln.i];
    d.any = false;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const double nu = nl + m->nu_top[ln.k0 + l];
        d.any = d.any || nu != 0.0;
        d.cf[l] = nu != 0.0 ? (T)(dtau * nu) : T(0);
        d.rc[l] = T(1) / (T(1) + d.cf[l]);
    }
    double r = (t - m->t1) / (m->t2 - m->t1);
    r = r < 0.0 ? 0.0 : (r > 1.0 ? 1.0 : r);
    d.tr = (T)r;
    d.mt = (T)(1.0 - r);
    return d;
}

template <typename T, class Lay, int L, int SG, bool TR, typename V>
__device__ __forceinline__ void damp_field(const Lane<Lay, L, SG> &ln, const MemberDev *m,
                                           const DampLane<T, L> &d, int f, V (&v)[L])
{
    if (!d.any) return;
    T b1[L], b2[L], ref[L];
    ln.template load<true>((const T *)m->bnd[0][f], 0, 0, b1);
    ln.template load<true>((const T *)m->bnd[1][f], 0, 0, b2);
#pragma unroll
    for (int l = 0; l < L; ++l) ref[l] = T(0);
    if (f == 0 || f == 4) {
        if constexpr (TR) ln.template load<true>((const T *)m->ref[f == 0 ? 0 : 1], 0, 0, ref);
        else ln.vmet(m->vm, f == 0 ? VM_RHO : VM_RT, ref);
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const T tgt = d.mt * (ref[l] + b1[l]) + d.tr * (ref[l] + b2[l]) - ref[l];
        const T x = (T)v[l];
        const T y = (x + d.cf[l] * tgt) * d.rc[l];
        const bool keep = d.cf[l] == T(0) || (f == 3 && ln.k0 + l == 0);
        v[l] = keep ? v[l] : (V)y;
    }
}

// EV: the explicit terms (p' of the horizontal pressure gradient) and the
// old-time (1 - beta) parts of the vertical coupling come from a second state
// (rpE, WE, tpE), while the increments are added to the first (rp, U, V, W,
// tp): the second stage of the Runge-Kutta short step.  Without EV both are
// the input state (forward-backward step).
// DP: damp the new values toward the member's boundary data at model time
// t_damp before storing them.
template <typename T, typename S, class Lay, int L, bool TR, bool EV, int SG, bool DP>
__device__ __forceinline__ void short_body(
    const Lane<Lay, L, SG> &ln, const MemberDev *dm, double t_damp,
    const double *__restrict__ vm, const double *__restrict__ geo,
    double dtau_d, double beta_d, T rdx, T rdy,
    const T *__restrict__ rp, const T *__restrict__ U, const T *__restrict__ V,
    const T *__restrict__ W, const T *__restrict__ tp, const T *__restrict__ rpE,
    const T *__restrict__ WE, const T *__restrict__ tpE, T *__restrict__ rpo, T *__restrict__ Uo,
    T *__restrict__ Vo, T *__restrict__ Wo, T *__restrict__ tpo, const T *__restrict__ SU,
    const T *__restrict__ SV, const T *__restrict__ SW, const T *__restrict__ RT,
    const T *__restrict__ ths, const T *__restrict__ P0, const T *__restrict__ Cs)
{
    const T dt = (T)dtau_d;
    // segment moves: DPP row shifts in the terrain form, shuffles in the flat
    // one (measured: 2.399 -> 2.280 ms over hills, 0.899 -> 0.907 ms flat)
    constexpr bool kMv = (SG == 16) && TR;
    const T *__restrict__ tpx = EV ? tpE : tp;   // Theta' of the pressure

    // ---- horizontally explicit part (storage precision) ----
    T pc[L], pw[L], pe[L], ps[L], pn[L];
    T P0c[L], Csc[L], tpc[L];
    {
        T a[L], c[L], t[L];
        ln.load(P0, 0, 0, P0c);
        ln.load(Cs, 0, 0, Csc);
        ln.load(tpx, 0, 0, t);
#pragma unroll
        for (int l = 0; l < L; ++l) pc[l] = P0c[l] + Csc[l] * t[l];
        if constexpr (EV) {
            ln.template load<true>(tp, 0, 0, tpc);
        } else {
#pragma unroll
            for (int l = 0; l < L; ++l) tpc[l] = t[l];
        }
        ln.load(P0, -1, 0, a); ln.load(Cs, -1, 0, c); ln.load(tpx, -1, 0, t);
#pragma unroll
        for (int l = 0; l < L; ++l) pw[l] = a[l] + c[l] * t[l];
        ln.load(P0, 1, 0, a); ln.load(Cs, 1, 0, c); ln.load(tpx, 1, 0, t);
#pragma unroll
        for (int l = 0; l < L; ++l) pe[l] = a[l] + c[l] * t[l];
        ln.load(P0, 0, -1, a); ln.load(Cs, 0, -1, c); ln.load(tpx, 0, -1, t);
#pragma unroll
        for (int l = 0; l < L; ++l) ps[l] = a[l] + c[l] * t[l];
        ln.load(P0, 0, 1, a); ln.load(Cs, 0, 1, c); ln.load(tpx, 0, 1, t);
#pragma unroll
        for (int l = 0; l < L; ++l) pn[l] = a[l] + c[l] * t[l];
    }
    // over terrain: metric correction (z_x/J) dp'/dzeta of the four faces
    T cw[L], ce[L], cs[L], cn[L];
    T ju0 = T(1), ju1 = T(1), jv0 = T(1), jv1 = T(1), rjc = T(1);
    T su0 = T(0), su1 = T(0), sv0 = T(0), sv1 = T(0);
    double jcol = 1.0;
    if constexpr (TR) {
        ju0 = (T)ln.geo(geo, GEO_JU, 0, 0);
        ju1 = (T)ln.geo(geo, GEO_JU, 1, 0);
        jv0 = (T)ln.geo(geo, GEO_JV, 0, 0);
        jv1 = (T)ln.geo(geo, GEO_JV, 0, 1);
        su0 = (T)ln.geo(geo, GEO_SU, 0, 0);
        su1 = (T)ln.geo(geo, GEO_SU, 1, 0);
        sv0 = (T)ln.geo(geo, GEO_SV, 0, 0);
        sv1 = (T)ln.geo(geo, GEO_SV, 0, 1);
        jcol = ln.geo(geo, GEO_J, 0, 0);
        rjc = T(1) / (T)jcol;
        T rdzf_t[L], dc[L];
        ln.vmet(vm, VM_RDZF, rdzf_t);
        ln.vmet(vm, VM_DC, dc);
        T gc[L], g1[L], g2[L];
        ddzeta<SG>(pc, rdzf_t, ln.p, ln.k0, ln.nz, gc);
        ddzeta<SG>(pw, rdzf_t, ln.p, ln.k0, ln.nz, g1);
        ddzeta<SG>(pe, rdzf_t, ln.p, ln.k0, ln.nz, g2);
        const T fw = su0 / ju0, fe = su1 / ju1, fs = sv0 / jv0, fn = sv1 / jv1;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            cw[l] = (dc[l] * fw) * (T(0.5) * (g1[l] + gc[l]));
            ce[l] = (dc[l] * fe) * (T(0.5) * (gc[l] + g2[l]));
        }
        ddzeta<SG>(ps, rdzf_t, ln.p, ln.k0, ln.nz, g1);
        ddzeta<SG>(pn, rdzf_t, ln.p, ln.k0, ln.nz, g2);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            cs[l] = (dc[l] * fs) * (T(0.5) * (g1[l] + gc[l]));
            cn[l] = (dc[l] * fn) * (T(0.5) * (gc[l] + g2[l]));
        }
    }
    T thc[L], thw[L], the[L], tsth[L], tnth[L];
    ln.load(ths, 0, 0, thc);
    ln.load(ths, -1, 0, thw);
    ln.load(ths, 1, 0, the);
    ln.load(ths, 0, -1, tsth);
    ln.load(ths, 0, 1, tnth);
    T U0[L], U1[L], SU0[L], SU1[L], V0[L], V1[L], SV0[L], SV1[L];
    ln.load(U, 0, 0, U0);
    ln.load(U, 1, 0, U1);
    ln.load(SU, 0, 0, SU0);
    ln.load(SU, 1, 0, SU1);
    ln.load(V, 0, 0, V0);
    ln.load(V, 0, 1, V1);
    ln.load(SV, 0, 0, SV0);
    ln.load(SV, 0, 1, SV1);
    // rpc, Wbc: the state the increments are added to; rpo_, Wc: old-time values
    T rpc[L], rpold[L], Wc[L], Wbc[L], SWc[L], RTc[L];
    ln.template load<true>(rp, 0, 0, rpc);
    ln.template load<true>(EV ? WE : W, 0, 0, Wc);
    if constexpr (EV) {
        ln.template load<true>(rpE, 0, 0, rpold);
        ln.template load<true>(W, 0, 0, Wbc);
    } else {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            rpold[l] = rpc[l];
            Wbc[l] = Wc[l];
        }
    }
    ln.template load<true>(SW, 0, 0, SWc);
    ln.template load<true>(RT, 0, 0, RTc);

    T Up[L], Vp[L], rt[L], tt[L], mx[L], my[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        T up0, up1, vp0, vp1, div, tdiv;
        const T fw = T(0.5) * (thw[l] + thc[l]), fe = T(0.5) * (thc[l] + the[l]);
        const T fs = T(0.5) * (tsth[l] + thc[l]), fn = T(0.5) * (thc[l] + tnth[l]);
        if constexpr (TR) {
            up0 = U0[l] + dt * (SU0[l] - ((pc[l] - pw[l]) * rdx - cw[l]));
            up1 = U1[l] + dt * (SU1[l] - ((pe[l] - pc[l]) * rdx - ce[l]));
            vp0 = V0[l] + dt * (SV0[l] - ((pc[l] - ps[l]) * rdy - cs[l]));
            vp1 = V1[l] + dt * (SV1[l] - ((pn[l] - pc[l]) * rdy - cn[l]));
            const T mu0 = ju0 * up0, mu1 = ju1 * up1, mv0 = jv0 * vp0, mv1 = jv1 * vp1;
            div = ((mu1 - mu0) * rdx + (mv1 - mv0) * rdy) * rjc;
            tdiv = ((fe * mu1 - fw * mu0) * rdx + (fn * mv1 - fs * mv0) * rdy) * rjc;
            mx[l] = T(0.5) * (su0 * up0 + su1 * up1);
            my[l] = T(0.5) * (sv0 * vp0 + sv1 * vp1);
        } else {
            up0 = U0[l] + dt * (SU0[l] - (pc[l] - pw[l]) * rdx);
            up1 = U1[l] + dt * (SU1[l] - (pe[l] - pc[l]) * rdx);
            vp0 = V0[l] + dt * (SV0[l] - (pc[l] - ps[l]) * rdy);
            vp1 = V1[l] + dt * (SV1[l] - (pn[l] - pc[l]) * rdy);
            div = (up1 - up0) * rdx + (vp1 - vp0) * rdy;
            tdiv = (fe * up1 - fw * up0) * rdx + (fn * vp1 - fs * vp0) * rdy;
        }
        Up[l] = up0;
        Vp[l] = vp0;
        rt[l] = rpc[l] - dt * div;
        tt[l] = tpc[l] + dt * (RTc[l] - tdiv);
    }
    if constexpr (DP) {
        const DampLane<T, L> dl = damp_setup<T>(ln, dm, t_damp, dtau_d);
        damp_field<T, Lay, L, SG, TR>(ln, dm, dl, 1, Up);
        damp_field<T, Lay, L, SG, TR>(ln, dm, dl, 2, Vp);
    }
    ln.store(Uo, Up);
    ln.store(Vo, Vp);

    // ---- vertically implicit part (solve precision S) ----
    const S be = (S)beta_d, dts = (S)dtau_d;
    const S one_m_be = S(1) - be;
    const S mu = be * be * dts * dts;
    const S grav = (S)kGrav;
    const int p = ln.p;
    const bool bot = (p == 0), top = (p == SG - 1);
    // vector loads of the table (one per lane and field)
    constexpr bool kVec = true;
    S rdz[L], rdzf[L], av[L], bv[L];
    ln.template vmet<S, kVec>(vm, VM_RDZ, rdz);
    ln.template vmet<S, kVec>(vm, VM_RDZF, rdzf);
    ln.template vmet<S, kVec>(vm, VM_A, av);
    ln.template vmet<S, kVec>(vm, VM_B, bv);
    // over terrain: the slope part E of Omega on the lane's level faces (from
    // the new horizontal momentum), and thicknesses J dzeta
    S Ef[L + 1];
    if constexpr (TR) {
        const S rj = S(1) / (S)jcol;
        S df[L];
        ln.vmet(vm, VM_DF, df);
        const S mxb = (S)from_below<SG, kMv>(mx[L - 1]), myb = (S)from_below<SG, kMv>(my[L - 1]);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            const int k = ln.k0 + l;
            const S mxm = (l == 0) ? mxb : (S)mx[l - 1];
            const S mym = (l == 0) ? myb : (S)my[l - 1];
            const S e = df[l] * ((av[l] * (S)mx[l] + bv[l] * mxm) + (av[l] * (S)my[l] + bv[l] * mym));
            Ef[l] = (k == 0) ? S(0) : e;
            rdz[l] = rdz[l] * rj;
            rdzf[l] = rdzf[l] * rj;
        }
        const S ea = from_above<SG, kMv>(Ef[0]);
        Ef[L] = top ? S(0) : ea;
    } else {
        (void)mx; (void)my;
    }
    const S rdz_b = from_below<SG, kMv>(rdz[L - 1]);   // 1/dz of the level below the lane

    // theta_s on the lane's level faces k0..k0+L-1, and on face k0+L
    const T th_b = from_below<SG, kMv>(thc[L - 1]);
    S thf[L + 1];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const S tb = (S)((l == 0) ? th_b : thc[l - 1]);
        thf[l] = (ln.k0 + l == 0) ? S(0) : av[l] * (S)thc[l] + bv[l] * tb;
    }
    {
        const S t = from_above<SG, kMv>(thf[0]);
        thf[L] = top ? S(0) : t;
    }
    const T w_up = from_above<SG, kMv>(Wc[0]);
    S Wf[L + 1];
#pragma unroll
    for (int l = 0; l < L; ++l) Wf[l] = (S)Wc[l];
    Wf[L] = top ? S(0) : (S)w_up;

    // the state each cell reaches with W+ = 0
    S thE[L], rhE[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const S f = one_m_be * dts * rdz[l];
        thE[l] = (S)tt[l] - f * (thf[l + 1] * Wf[l + 1] - thf[l] * Wf[l]);
        rhE[l] = (S)rt[l] - f * (Wf[l + 1] - Wf[l]);
        if constexpr (TR) {
            const S g = dts * rdz[l];
            thE[l] = thE[l] + g * (thf[l + 1] * Ef[l + 1] - thf[l] * Ef[l]);
            rhE[l] = rhE[l] + g * (Ef[l + 1] - Ef[l]);
        }
    }
    // off-centred pressure and density of that state, per level (evaluated
    // where a row needs them; the lane's top level also for the lane above)
    auto pE_of = [&](int l) -> S {
        return be * ((S)P0c[l] + (S)Csc[l] * thE[l]) + one_m_be * (S)pc[l];
    };
    auto rEs_of = [&](int l) -> S { return be * rhE[l] + one_m_be * (S)rpold[l]; };
    S Cm = from_below<SG, kMv>((S)Csc[L - 1]), tfm = from_below<SG, kMv>(thf[L - 1]);
    S pEm = from_below<SG, kMv>(pE_of(L - 1)), rEm = from_below<SG, kMv>(rEs_of(L - 1));
    S rdzm = rdz_b;
    // row l of the tridiagonal system in W+ on level face k0 + l; each call
    // passes its level's values on as the "below" values of the next row
    auto row = [&](int l, S &a, S &b, S &c, S &d) {
        const int k = ln.k0 + l;
        const S Cc = (S)Csc[l];
        const S pE = pE_of(l), rEs = rEs_of(l);
        const S rdzp = rdz[l];
        const S fA = -mu * Cm * tfm * (rdzf[l] * rdzm) + mu * grav * bv[l] * rdzm;
        const S fC = -mu * Cc * thf[l + 1] * (rdzf[l] * rdzp) - mu * grav * av[l] * rdzp;
        const S fB = S(1) + mu * thf[l] * (Cc * rdzp + Cm * rdzm) * rdzf[l] +
                     mu * grav * (av[l] * rdzp - bv[l] * rdzm);
        const S fD = (S)Wbc[l] + dts * (S)SWc[l] - (dts * rdzf[l]) * (pE - pEm) -
                     dts * grav * (av[l] * rEs + bv[l] * rEm);
        // the lid row is (0, 1, 0, 0): chosen by bit masks rather than
        // selects, which the compiler turns into a divergent branch here
        const bool lid = (k == 0);
        a = keep_if(!lid, fA);
        b = keep_if(!lid, fB) + keep_if(lid, S(1));
        c = keep_if(!(lid || k == ln.nz - 1), fC);
        d = keep_if(!lid, fD);
        Cm = Cc;
        tfm = thf[l];
        pEm = pE;
        rEm = rEs;
        rdzm = rdzp;
    };
    S x[L];
    segment_solve<S, L, SG, kMv>(p, row, x);

    const S x_up = from_above<SG, kMv>(x[0]);
    const S xt = top ? S(0) : x_up;
    S rpn[L], tpn[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const S xu = (l < L - 1) ? x[l + 1] : xt;
        const S f = be * dts * rdz[l];
        rpn[l] = rhE[l] - f * (xu - x[l]);
        tpn[l] = thE[l] - f * (thf[l + 1] * xu - thf[l] * x[l]);
    }
    (void)bot;
    if constexpr (DP) {
        const DampLane<T, L> dl = damp_setup<T>(ln, dm, t_damp, dtau_d);
        damp_field<T, Lay, L, SG, TR>(ln, dm, dl, 3, x);
        damp_field<T, Lay, L, SG, TR>(ln, dm, dl, 0, rpn);
        damp_field<T, Lay, L, SG, TR>(ln, dm, dl, 4, tpn);
    }
    ln.store(Wo, x);
    ln.store(rpo, rpn);
    ln.store(tpo, tpn);
}

// SG lanes per column, kColsPerBlock columns per block of kColsPerBlock * SG
// threads.
// DP variants damp (members without damping data skip it) at the model time
// sums[2] + offset * dt, the end of this short step.
template <typename T, typename S, class Lay, int L, bool TR, bool EV, int SG, bool DP>
__global__ __launch_bounds__((threads_of<SG, 1>()))
__attribute__((amdgpu_waves_per_eu(short_waves<T, S, L, TR, EV, SG, DP>())))
void k_short_step(Group gr, double frac, double offset)
{
    const Where wh = locate<SG, 1>(gr);
    if (!wh.active) return;
    const MemberDev *m = wh.m;
    const Lane<Lay, L, SG> ln(m->nx, m->ny, m->nz, wh.i, wh.j);
    constexpr bool kDamp = DP;
    if (kDamp && m->nu_lat == nullptr) {
        short_body<T, S, Lay, L, TR, EV, SG, false>(
            ln, m, 0.0, m->vm, m->geo, m->dt * frac, m->beta, (T)m->rdx, (T)m->rdy,
            (const T *)buf(m, gr.src, 0), (const T *)buf(m, gr.src, 1), (const T *)buf(m, gr.src, 2),
            (const T *)buf(m, gr.src, 3), (const T *)buf(m, gr.src, 4), (const T *)buf(m, gr.ev, 0),
            (const T *)buf(m, gr.ev, 3), (const T *)buf(m, gr.ev, 4), (T *)buf(m, gr.dst, 0),
            (T *)buf(m, gr.dst, 1), (T *)buf(m, gr.dst, 2), (T *)buf(m, gr.dst, 3),
            (T *)buf(m, gr.dst, 4), (const T *)m->slow[0], (const T *)m->slow[1],
            (const T *)m->slow[2], (const T *)m->slow[3], (const T *)m->slow[4],
            (const T *)m->slow[5], (const T *)m->slow[6]);
        return;
    }
    short_body<T, S, Lay, L, TR, EV, SG, DP>(
        ln, m, DP ? m->sums[2] + offset * m->dt : 0.0, m->vm, m->geo, m->dt * frac, m->beta,
        (T)m->rdx, (T)m->rdy,
        (const T *)buf(m, gr.src, 0), (const T *)buf(m, gr.src, 1), (const T *)buf(m, gr.src, 2),
        (const T *)buf(m, gr.src, 3), (const T *)buf(m, gr.src, 4), (const T *)buf(m, gr.ev, 0),
        (const T *)buf(m, gr.ev, 3), (const T *)buf(m, gr.ev, 4), (T *)buf(m, gr.dst, 0),
        (T *)buf(m, gr.dst, 1), (T *)buf(m, gr.dst, 2), (T *)buf(m, gr.dst, 3),
        (T *)buf(m, gr.dst, 4), (const T *)m->slow[0], (const T *)m->slow[1],
        (const T *)m->slow[2], (const T *)m->slow[3], (const T *)m->slow[4],
        (const T *)m->slow[5], (const T *)m->slow[6]);
}

// --------------------------------------------------------------------------
// model clock of the damping: one thread per member, time += dt at the end
// of a long step
// --------------------------------------------------------------------------
__global__ void k_clock(Group gr)
{
    const int q = (int)threadIdx.x;
    if (q >= gr.nm) return;
    const MemberDev *m = gr.mem + (gr.nm == 1 ? gr.first : gr.ids[q]);
    m->sums[2] = m->sums[2] + m->dt;
}

// --------------------------------------------------------------------------
// float64 sums with a fixed two-level order
// --------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] = sh[t] + sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// Partial sums of one member: its partial block q accumulates the member's
// 16x1 tiles q, q + P, q + 2P, ... (P = its partial count) in that order, each
// lane in float64, then a fixed tree over the block.  The launch covers the
// partial blocks of every member of a group (gr.blk maps blocks to partials).
template <typename T, class Lay, int L, bool ENERGY, bool TR>
__global__ __launch_bounds__(BLOCK) void k_sum_partial(Group gr)
{
    __shared__ double sh[BLOCK];
    int q = (int)blockIdx.x, id = gr.first;
    if (gr.nm > 1) {
        const unsigned v = gr.blk[blockIdx.x];
        q = (int)(v & 0xFFFFFFu);
        id = (int)(v >> 24);
    }
    const MemberDev *m = gr.mem + id;
    const int tiles_x = (m->nx + kColsPerBlock - 1) / kColsPerBlock;
    const int ntiles = tiles_x * m->ny;
    const double *__restrict__ vm = m->vm;
    const T *__restrict__ s0 = (const T *)buf(m, gr.src, 0);
    const T *__restrict__ s1 = (const T *)buf(m, gr.src, 1);
    const T *__restrict__ s2 = (const T *)buf(m, gr.src, 2);
    const T *__restrict__ s3 = (const T *)buf(m, gr.src, 3);
    const T *__restrict__ s4 = (const T *)buf(m, gr.src, 4);
    double acc = 0.0;
    for (int t = q; t < ntiles; t += m->npart) {
        const int i = (t % tiles_x) * kColsPerBlock + (int)threadIdx.x / SEG;
        const int j = t / tiles_x;
        if (i < m->nx) {
            const Lane<Lay, L> ln(m->nx, m->ny, m->nz, i, j);
            double vol[L];
            ln.vmet(vm, VM_VOL, vol);
            if constexpr (TR) {
                // cell volume J dx dy dzeta
                const double jc = ln.geo(m->geo, GEO_J, 0, 0);
#pragma unroll
                for (int l = 0; l < L; ++l) vol[l] = vol[l] * jc;
            }
            if constexpr (!ENERGY) {
                T r[L];
                ln.template load<true>(s0, 0, 0, r);
#pragma unroll
                for (int l = 0; l < L; ++l) acc += (double)r[l] * vol[l];
            } else {
                T r[L], u0[L], u1[L], v0[L], v1[L], w0[L], th[L];
                ln.load(s0, 0, 0, r);
                ln.load(s1, 0, 0, u0);
                ln.load(s1, 1, 0, u1);
                ln.load(s2, 0, 0, v0);
                ln.load(s2, 0, 1, v1);
                ln.load(s3, 0, 0, w0);
                ln.load(s4, 0, 0, th);
                const T wt = from_above(w0[0]);
                double rref[L], rtref[L], pref[L], zc[L];
                ln.vmet(vm, VM_ZC, zc);
                if constexpr (TR) {
                    T a[L];
                    ln.load((const T *)m->ref[0], 0, 0, a);
#pragma unroll
                    for (int l = 0; l < L; ++l) rref[l] = (double)a[l];
                    ln.load((const T *)m->ref[1], 0, 0, a);
#pragma unroll
                    for (int l = 0; l < L; ++l) rtref[l] = (double)a[l];
                    ln.load((const T *)m->ref[2], 0, 0, a);
#pragma unroll
                    for (int l = 0; l < L; ++l) pref[l] = (double)a[l];
                    // true height of the cell centre
                    double dc[L];
                    ln.vmet(vm, VM_DC, dc);
                    const double h = ln.geo(m->geo, GEO_H, 0, 0);
#pragma unroll
                    for (int l = 0; l < L; ++l) zc[l] = zc[l] + h * dc[l];
                } else {
                    ln.vmet(vm, VM_RHO, rref);
                    ln.vmet(vm, VM_RT, rtref);
                    ln.vmet(vm, VM_P, pref);
                }
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    const double rho = rref[l] + (double)r[l];
                    const double wu = (l < L - 1) ? (double)w0[l + 1] : (ln.p == SEG - 1 ? 0.0 : (double)wt);
                    const double a = (double)u0[l], bb = (double)u1[l], c = (double)v0[l];
                    const double d = (double)v1[l], e = (double)w0[l];
                    const double ke = 0.5 * (0.5 * (a * a + bb * bb) + 0.5 * (c * c + d * d) +
                                             0.5 * (e * e + wu * wu)) / rho;
                    const double pres = pref[l] + pref[l] * expm1(kGamma * log1p((double)th[l] / rtref[l]));
                    acc += (ke + pres / (kGamma - 1.0) + rho * kGrav * zc[l]) * vol[l];
                }
            }
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) (gr.part ? gr.part : m->partials)[q] = s;
}

// Mass partials in the i-fastest layout: one lane per column, consecutive
// lanes at consecutive columns of the (i, j) plane, so every level is one
// coalesced row per wavefront (the segment form above loads a lane's levels
// one row of nx * ny apart).  Partial block q takes the member's chunks of
// BLOCK columns q, q + P, q + 2P, ... (P = its partial count) in that order,
// each lane summing its column bottom to top in float64, then the fixed tree
// over the block.
template <typename T, bool TR>
__global__ __launch_bounds__(BLOCK) void k_sum_mass_cols(Group gr)
{
    __shared__ double sh[BLOCK];
    int q = (int)blockIdx.x, id = gr.first;
    if (gr.nm > 1) {
        const unsigned v = gr.blk[blockIdx.x];
        q = (int)(v & 0xFFFFFFu);
        id = (int)(v >> 24);
    }
    const MemberDev *m = gr.mem + id;
    const int ncol = m->nx * m->ny, nz = m->nz;
    const int nchunk = (ncol + BLOCK - 1) / BLOCK;
    const double *__restrict__ vol = m->vm + (size_t)VM_VOL * nz;
    const T *__restrict__ r = (const T *)buf(m, gr.src, 0);
    double acc = 0.0;
    for (int t = q; t < nchunk; t += m->npart) {
        const int c = t * BLOCK + (int)threadIdx.x;
        if (c < ncol) {
            double jc = 1.0;
            if constexpr (TR) jc = m->geo[(size_t)c * GEO_NFIELDS + GEO_J];
            const T *__restrict__ rc = r + c;
#pragma unroll 8
            for (int k = 0; k < nz; ++k) {
                double v = vol[k];
                if constexpr (TR) v = v * jc;
                acc += (double)__builtin_nontemporal_load(rc + (size_t)k * ncol) * v;
            }
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) (gr.part ? gr.part : m->partials)[q] = s;
}

// One block per member of the group: sum its partials in a fixed order
// (thread t takes t, t + BLOCK, ... with Neumaier compensation, then a tree).
__global__ __launch_bounds__(BLOCK) void k_sum_final(Group gr, int slot)
{
    __shared__ double sh[BLOCK];
    const int id = gr.nm == 1 ? gr.first : gr.ids[blockIdx.x];
    const MemberDev *m = gr.mem + id;
    const double *part = gr.part ? gr.part : m->partials;
    double s = 0.0, c = 0.0;
    for (int q = threadIdx.x; q < m->npart; q += BLOCK) {
        const double x = part[q];
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    const double tot = block_sum(s + c, sh);
    if (threadIdx.x == 0) {
        if (gr.out) {
            gr.out[slot] = slot == 0 ? gr.out_add + tot : tot;
        } else {
            double *sm = m->sums;
            sm[slot] = tot;
            if (slot == 0 && gr.mass_init == id + 1) {
                sm[3] = tot;
                sm[4] = 0.0;
                sm[5] = 0.0;
            } else if (slot == 0 && m->drift_bound > 0.0) {
                // failure detection: relative drift of the total mass since
                // state_init (a non-finite mass fails both comparisons)
                const double d = fabs(tot - sm[3]) / (m->mass_ref + sm[3]);
                if (!(d <= sm[5])) sm[5] = d;
                if (!(d <= m->drift_bound)) sm[4] = 1.0;
            }
        }
    }
}

// Partials of the allocation-free sums (one grid at a time per device; see
// scratch_address).
static __device__ __align__(256) double scratch[kScratchDoubles];

// --------------------------------------------------------------------------
// seven-point diffusion (the bandwidth-model stencil): one read of each
// value and one write per cell with perfect reuse, 7 reads + 1 write without
// any; horizontal neighbours come through the caches, vertical ones by
// segment shuffles.
// --------------------------------------------------------------------------
template <typename T, class Lay, int L>
__device__ __forceinline__ void diffuse_body(const Lane<Lay, L> &ln, T kx, T ky, T kz,
                                             const T *__restrict__ q, T *__restrict__ out)
{
    T c[L], w[L], e[L], s[L], n[L];
    ln.load(q, 0, 0, c);
    ln.load(q, -1, 0, w);
    ln.load(q, 1, 0, e);
    ln.load(q, 0, -1, s);
    ln.load(q, 0, 1, n);
    // shuffles, not DPP row shifts: measured 0.098 vs 0.114 ms per float32
    // step on 1024x1024x64
    const T below = from_below<SEG, false>(c[L - 1]), above = from_above<SEG, false>(c[0]);
    T r[L];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int k = ln.k0 + l;
        const T qd = (l > 0) ? c[l - 1] : (k > 0 ? below : c[l]);
        const T qu = (l < L - 1) ? c[l + 1] : (k < ln.nz - 1 ? above : c[l]);
        const T lx = (w[l] + e[l]) - T(2) * c[l];
        const T ly = (s[l] + n[l]) - T(2) * c[l];
        const T lz = (qd + qu) - T(2) * c[l];
        r[l] = c[l] + ((kx * lx + ky * ly) + kz * lz);
    }
    ln.store(out, r);
}

template <typename T, class Lay, int L>
__global__ __launch_bounds__(BLOCK) void k_diffuse(DiffArgs a)
{
    const int ti = 1 << a.ti_log2, tj = kColsPerBlock >> a.ti_log2;
    const int tiles_x = (a.nx + ti - 1) / ti;
    const int t = (int)blockIdx.x, c = (int)threadIdx.x / SEG;
    const int i = (t % tiles_x) * ti + (c & (ti - 1));
    const int j = (t / tiles_x) * tj + (c >> a.ti_log2);
    if (i >= a.nx || j >= a.ny) return;
    const Lane<Lay, L> ln(a.nx, a.ny, a.nz, i, j);
    diffuse_body<T, Lay, L>(ln, (T)a.kx, (T)a.ky, (T)a.kz, (const T *)a.in, (T *)a.out);
}

// --------------------------------------------------------------------------
// dispatch
// --------------------------------------------------------------------------
template <template <typename, typename, class, int> class F, typename... Args>
hipError_t dispatch(int prec, int layout, int L, Args &&...args)
{
    auto go = [&](auto tag_t, auto tag_s) -> hipError_t {
        using T = decltype(tag_t);
        using S = decltype(tag_s);
        switch ((layout == 1 ? 100 : 0) + L) {
        case 102: return F<T, S, KIJ, 2>::run(args...);
        case 104: return F<T, S, KIJ, 4>::run(args...);
        case 108: return F<T, S, KIJ, 8>::run(args...);
        case 2: return F<T, S, IJK, 2>::run(args...);
        case 4: return F<T, S, IJK, 4>::run(args...);
        case 8: return F<T, S, IJK, 8>::run(args...);
        default: return hipErrorInvalidValue;
        }
    };
    switch (prec) {
    case 0: return go(double(), double());
    case 1: return go(float(), float());
    case 2: return go(float(), double());
    default: return hipErrorInvalidValue;
    }
}

// Lanes per column (segment width) of a launch.  A column of nz = 16 L
// levels can run in segments of 16 lanes (L levels per lane), of 32 lanes
// (L/2 levels, L >= 4) or, for 32 levels, of 8 lanes (4 levels per lane).
// gr.seg names the width (the autotuner's choice); 0 takes the default: 32
// lanes for float64 storage with 4 levels per 16 lanes (half the registers
// per lane, twice the waves per SIMD), else 16.  The other widths are built
// for the column-fastest layout only, and for the short step not in its
// damped form, which keep the default.  The slow sweeps compute every cell
// the same way in any width; the short step's column solve eliminates the
// lane-interior rows in each lane and the segment's interface rows by
// cyclic reduction, so its rounding depends on the width.
template <typename T, int L>
constexpr int default_seg() { return (sizeof(T) == 8 && L == 4) ? 32 : 16; }

template <int V>
using ic = std::integral_constant<int, V>;

// go(ic<SG>, ic<levels per lane>) for the launch's width
template <typename T, int L, bool ALT, class Go>
hipError_t by_seg(int seg, Go &&go)
{
    if (seg == 0 || !ALT) seg = default_seg<T, L>();
    if constexpr (ALT || default_seg<T, L>() == 16) {
        if (seg == 16) return go(ic<16>{}, ic<L>{});
    }
    if constexpr (L >= 4 && (ALT || default_seg<T, L>() == 32)) {
        if (seg == 32) return go(ic<32>{}, ic<L / 2>{});
    }
    if constexpr (L == 2 && ALT) {
        if (seg == 8) return go(ic<8>{}, ic<4>{});
    }
    return hipErrorInvalidValue;
}

template <typename T, typename S, class Lay, int L>
struct RunPrep {
    static hipError_t run(const Group &gr, hipStream_t s)
    {
        return by_seg<T, L, Lay::kContig>(gr.seg, [&](auto sg, auto kl) {
            constexpr int SG = decltype(sg)::value, KL = decltype(kl)::value;
            if (gr.terrain)
                hipLaunchKernelGGL((k_slow_prep<T, Lay, KL, true, SG>), dim3(gr.nblocks * split_of<SG>()),
                                   dim3(threads_of<SG>()), 0, s, gr);
            else
                hipLaunchKernelGGL((k_slow_prep<T, Lay, KL, false, SG>), dim3(gr.nblocks * split_of<SG>()),
                                   dim3(threads_of<SG>()), 0, s, gr);
            return hipGetLastError();
        });
    }
};

template <typename T, typename S, class Lay, int L>
struct RunFlux {
    template <class A>
    static hipError_t go(const Group &gr, hipStream_t s)
    {
        return by_seg<T, L, Lay::kContig>(gr.seg, [&](auto sg, auto kl) {
            constexpr int SG = decltype(sg)::value, KL = decltype(kl)::value;
            if constexpr (Lay::kContig) {
                if (gr.run > 1) {
                    if (gr.terrain)
                        hipLaunchKernelGGL((k_slow_flux_run<T, A, KL, true, SG>), dim3(gr.nblocks * split_of<SG>()),
                                           dim3(threads_of<SG>()), 0, s, gr);
                    else
                        hipLaunchKernelGGL((k_slow_flux_run<T, A, KL, false, SG>), dim3(gr.nblocks * split_of<SG>()),
                                           dim3(threads_of<SG>()), 0, s, gr);
                    return hipGetLastError();
                }
            }
            if (gr.terrain)
                hipLaunchKernelGGL((k_slow_flux<T, A, KL, true, SG>), dim3(gr.nblocks * split_of<SG>()),
                                   dim3(threads_of<SG>()), 0, s, gr);
            else
                hipLaunchKernelGGL((k_slow_flux<T, A, KL, false, SG>), dim3(gr.nblocks * split_of<SG>()),
                                   dim3(threads_of<SG>()), 0, s, gr);
            return hipGetLastError();
        });
    }
    // The slow flux is instruction-heavy enough that 32-bit array offsets pay
    // (float32: 0.973 -> 0.895 ms, float64: 2.50 -> 2.09 ms on 1024x1024x64);
    // the host selects them when every array fits in 4 GiB.  Global
    // instructions for the float64 flux and for the runs (float32 runs: 0.80
    // -> 0.77 ms; float64 runs with flat ones 1.52 -> 1.55 ms), flat ones for
    // the per-column float flux.
    static hipError_t run(const Group &gr, hipStream_t s)
    {
        if (gr.off32 && gr.run > 1) return go<Off32<Lay, true>>(gr, s);
        if (gr.off32) return go<Off32<Lay, sizeof(T) == 8>>(gr, s);
        return go<Lay>(gr, s);
    }
};

// The mixed form keeps 16 lanes by default: with 2 levels per lane the
// cyclic reduction's float64 work per level doubles and outweighs the higher
// occupancy (measured on 1024x1024x64: 1.035 ms with 16 lanes, 1.109 ms with
// 32).
template <typename T, typename S, class Lay, int L>
struct RunShort {
    template <class A, bool TR, bool EV, bool DP>
    static hipError_t launch(const Group &gr, double frac, double offset, hipStream_t s)
    {
        return by_seg<T, L, Lay::kContig && !DP>(gr.seg, [&](auto sg, auto kl) {
            constexpr int SG = decltype(sg)::value, KL = decltype(kl)::value;
            hipLaunchKernelGGL((k_short_step<T, S, A, KL, TR, EV, SG, DP>), dim3(gr.nblocks),
                               dim3(threads_of<SG, 1>()), 0, s, gr, frac, offset);
            return hipGetLastError();
        });
    }
    // 32-bit offsets: with global instructions in the flat, undamped
    // float32 step (measured on 1024 x 1024 x 64: 0.895 -> 0.876 ms; the
    // Runge-Kutta pair unchanged; the damped form loses 4%), with flat
    // instructions in the flat mixed step (global 0.915, flat 0.903 ms) and
    // in the undamped terrain step (over hills, 1600 x 1280 x 64: mixed
    // 2.028 -> 1.974-2.008 ms, FP64 3.70 -> 3.64 ms; global ones 2.00 and
    // 3.74 ms); with global instructions in the flat FP64 step (4x4 tiles,
    // chunked: 1.766 -> 1.754 ms; 1.8-3.7% in the other configurations)
    template <bool TR, bool EV, bool DP>
    static hipError_t go(const Group &gr, double frac, double offset, hipStream_t s)
    {
        if constexpr (sizeof(T) == 4 && !TR && !DP) {
            if (gr.off32) return launch<Off32<Lay, (sizeof(S) == 4)>, TR, EV, DP>(gr, frac, offset, s);
        }
        if constexpr (TR && !DP) {
            if (gr.off32) return launch<Off32<Lay, false>, TR, EV, DP>(gr, frac, offset, s);
        }
        if constexpr (sizeof(T) == 8 && !TR && !DP) {
            if (gr.off32) return launch<Off32<Lay, true>, TR, EV, DP>(gr, frac, offset, s);
        }
        return launch<Lay, TR, EV, DP>(gr, frac, offset, s);
    }
    template <bool TR, bool EV>
    static hipError_t go2(const Group &gr, double frac, double offset, hipStream_t s)
    {
        if (gr.damp) return go<TR, EV, true>(gr, frac, offset, s);
        return go<TR, EV, false>(gr, frac, offset, s);
    }
    static hipError_t run(const Group &gr, double frac, double offset, hipStream_t s)
    {
        const bool ev = gr.ev != gr.src;
        if (gr.terrain) return ev ? go2<true, true>(gr, frac, offset, s) : go2<true, false>(gr, frac, offset, s);
        return ev ? go2<false, true>(gr, frac, offset, s) : go2<false, false>(gr, frac, offset, s);
    }
};

template <typename T, typename S, class Lay, int L>
struct RunSums {
    template <bool TR>
    static void partial(const Group &gr, bool energy, hipStream_t s)
    {
        if (energy)
            hipLaunchKernelGGL((k_sum_partial<T, Lay, L, true, TR>), dim3(gr.nblocks), dim3(BLOCK), 0, s, gr);
        else
            hipLaunchKernelGGL((k_sum_partial<T, Lay, L, false, TR>), dim3(gr.nblocks), dim3(BLOCK), 0, s, gr);
    }
    static hipError_t run(const Group &gr, bool energy, hipStream_t s)
    {
        if (gr.terrain) partial<true>(gr, energy, s);
        else partial<false>(gr, energy, s);
        hipLaunchKernelGGL(k_sum_final, dim3(gr.nm), dim3(BLOCK), 0, s, gr, energy ? 1 : 0);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_slow_prep(int prec, int layout, int L, const Group &gr, hipStream_t s)
{
    if (gr.colmap && layout == 0) return launch_columns(0, prec, gr, 0.0, s);
    return dispatch<RunPrep>(prec, layout, L, gr, s);
}

hipError_t launch_slow_flux(int prec, int layout, int L, const Group &gr, hipStream_t s)
{
    if (gr.colmap && layout == 0) return launch_columns(1, prec, gr, 0.0, s);
    return dispatch<RunFlux>(prec, layout, L, gr, s);
}

hipError_t launch_short_step(int prec, int layout, int L, const Group &gr, double frac, double offset,
                             hipStream_t s)
{
    // the column kernel takes the forward-backward step without damping; the
    // Runge-Kutta and damped forms run in column segments
    if (gr.colmap && layout == 0 && !gr.damp && gr.ev == gr.src)
        return launch_columns(2, prec, gr, frac, s);
    return dispatch<RunShort>(prec, layout, L, gr, frac, offset, s);
}

hipError_t launch_sums(int prec, int layout, int L, const Group &gr, bool energy, hipStream_t s)
{
    if (layout == 0 && !energy) {
        // the i-fastest layout's mass: one lane per column (coalesced rows)
        if (prec == 0) {
            if (gr.terrain) hipLaunchKernelGGL((k_sum_mass_cols<double, true>), dim3(gr.nblocks), dim3(BLOCK), 0, s, gr);
            else hipLaunchKernelGGL((k_sum_mass_cols<double, false>), dim3(gr.nblocks), dim3(BLOCK), 0, s, gr);
        } else if (prec == 1 || prec == 2) {
            if (gr.terrain) hipLaunchKernelGGL((k_sum_mass_cols<float, true>), dim3(gr.nblocks), dim3(BLOCK), 0, s, gr);
            else hipLaunchKernelGGL((k_sum_mass_cols<float, false>), dim3(gr.nblocks), dim3(BLOCK), 0, s, gr);
        } else {
            return hipErrorInvalidValue;
        }
        hipLaunchKernelGGL(k_sum_final, dim3(gr.nm), dim3(BLOCK), 0, s, gr, 0);
        return hipGetLastError();
    }
    return dispatch<RunSums>(prec, layout, L, gr, energy, s);
}

hipError_t scratch_address(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t r = hipGetDevice(&dev);
    if (r != hipSuccess) return r;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the array's name is a host-side stand-in; the device address of
        // this device's copy comes from the runtime
        void *p = nullptr;
        if ((r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return r;
        addr[dev] = (double *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_clock(const Group &gr, hipStream_t s)
{
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(256), 0, s, gr);
    return hipGetLastError();
}

template <typename T, typename S, class Lay, int L>
struct RunDiffuse {
    static hipError_t run(const DiffArgs &a, hipStream_t s)
    {
        const int blocks = tiles_of(a.nx, a.ny, a.ti_log2);
        hipLaunchKernelGGL((k_diffuse<T, Lay, L>), dim3(blocks), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
};

hipError_t launch_diffuse(int prec, int layout, int L, const DiffArgs &a, hipStream_t s)
{
    if (prec == 2) return hipErrorInvalidValue;   // no mixed form
    return dispatch<RunDiffuse>(prec, layout, L, a, s);
}

}  // namespace hv
