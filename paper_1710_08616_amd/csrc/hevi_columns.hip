// hevi_columns.hip -- the one-lane-per-column kernels of the i-fastest
// storage order (slow prep, slow flux, forward-backward short step).
#include "hevi_kernels.h"
#include "hevi_device.h"

#include <cstdint>

namespace hv {
namespace {

// --------------------------------------------------------------------------
// i-fastest layout, native mapping: one lane per column.  A block covers 64
// consecutive columns along x (one wavefront per row) by 4 rows along y, and
// every lane walks its column from the bottom level to the top: each load of
// a level is one coalesced row of 64 values per wavefront, vertical
// neighbours stay in registers, and the per-level constants are uniform
// across the wavefront (scalar loads).  This is the paper's own GPU mapping
// (Sect. 2.3: a thread per (i, j) column, the k loop inside it).  The slow
// sweeps compute every cell exactly as the segment kernels do; the short step
// solves each column's tridiagonal system by a serial Thomas sweep (forward
// elimination on the way up, back substitution on the way down), whose
// intermediate values (modified upper diagonal and right-hand side, the
// state with W+ = 0) go through four workspace arrays.
// --------------------------------------------------------------------------
constexpr int kRowX = 64, kRowY = 4;

struct Col {
    const MemberDev *m;
    int i, j, nx, ny, nz;
    size_t plane;   // nx*ny
    bool active;
    // offset of column (i+di, j+dj) within a level
    __device__ unsigned off(int di, int dj) const
    {
        return (unsigned)wrapc(j + dj, ny) * (unsigned)nx + (unsigned)wrapc(i + di, nx);
    }
};

__device__ __forceinline__ Col locate_col(const Group &gr)
{
    Col c;
    c.m = gr.mem + gr.first;
    c.nx = c.m->nx;
    c.ny = c.m->ny;
    c.nz = c.m->nz;
    const int tx = (c.nx + kRowX - 1) / kRowX;
    const int b = (int)blockIdx.x;
    c.i = (b % tx) * kRowX + (int)threadIdx.x % kRowX;
    c.j = (b / tx) * kRowY + (int)threadIdx.x / kRowX;
    c.active = c.i < c.nx && c.j < c.ny;
    c.plane = (size_t)c.nx * c.ny;
    return c;
}

// Element at byte offset ob of the level that starts lev elements into a:
// lev is uniform across the wavefront (a scalar base per level), ob a 32-bit
// per-lane offset, through global-address-space pointers.
template <typename T>
__device__ __forceinline__ T ld(const T *a, size_t lev, unsigned ob)
{
    using B = const char __attribute__((address_space(1))) *;
    return *(const T __attribute__((address_space(1))) *)((B)(a + lev) + ob);
}
template <typename T>
__device__ __forceinline__ void st(T *a, size_t lev, unsigned ob, T v)
{
    using B = char __attribute__((address_space(1))) *;
    __builtin_nontemporal_store(v, (T __attribute__((address_space(1))) *)((B)(a + lev) + ob));
}

// per-level constant f at level k as type S (float32 kernels read the
// table's float32 copy, as the segment kernels do)
template <typename S>
__device__ __forceinline__ S lev(const double *__restrict__ vm, int nz, int f, int k)
{
    if constexpr (sizeof(S) == sizeof(float))
        return ((const float *)(vm + (size_t)VM_NFIELDS * nz))[(size_t)f * nz + k];
    else
        return (S)vm[(size_t)f * nz + k];
}

template <typename T, bool TR>
__global__ __launch_bounds__(kRowX * kRowY) void k_slow_prep_col(Group gr)
{
    const Col c = locate_col(gr);
    if (!c.active) return;
    const MemberDev *m = c.m;
    const double *__restrict__ vm = m->vm;
    const int nz = c.nz;
    const T *__restrict__ rp = (const T *)buf(m, gr.src, 0);
    const T *__restrict__ U = (const T *)buf(m, gr.src, 1);
    const T *__restrict__ V = (const T *)buf(m, gr.src, 2);
    const T *__restrict__ W = (const T *)buf(m, gr.src, 3);
    const T *__restrict__ tp = (const T *)buf(m, gr.src, 4);
    T *__restrict__ uo = (T *)m->spec[0];
    T *__restrict__ vo = (T *)m->spec[1];
    T *__restrict__ wo = (T *)m->spec[2];
    T *__restrict__ omo = (T *)m->spec[3];
    T *__restrict__ tho = (T *)m->slow[4];
    T *__restrict__ P0o = (T *)m->slow[5];
    T *__restrict__ Cso = (T *)m->slow[6];
    const T *__restrict__ rref3 = (const T *)m->ref[0];
    const T *__restrict__ rtref3 = (const T *)m->ref[1];
    const T *__restrict__ pref3 = (const T *)m->ref[2];
    const unsigned o0 = c.off(0, 0), ow = c.off(-1, 0), os = c.off(0, -1);
    const unsigned oe = c.off(1, 0), on = c.off(0, 1);
    T su0 = T(0), su1 = T(0), sv0 = T(0), sv1 = T(0);
    if constexpr (TR) {
        const double *g = m->geo;
        su0 = (T)g[(size_t)o0 * GEO_NFIELDS + GEO_SU];
        su1 = (T)g[(size_t)oe * GEO_NFIELDS + GEO_SU];
        sv0 = (T)g[(size_t)o0 * GEO_NFIELDS + GEO_SV];
        sv1 = (T)g[(size_t)on * GEO_NFIELDS + GEO_SV];
    }
    T rbelow = T(0), mxb = T(0), myb = T(0);
    for (int k = 0; k < nz; ++k) {
        const size_t L0 = (size_t)k * c.plane;
        T r0 = ld(rp, L0, o0 * (unsigned)sizeof(*rp)), rw = ld(rp, L0, ow * (unsigned)sizeof(*rp)), rs = ld(rp, L0, os * (unsigned)sizeof(*rp));
        const T Uc = ld(U, L0, o0 * (unsigned)sizeof(*U)), Vc = ld(V, L0, o0 * (unsigned)sizeof(*V)), Wc = ld(W, L0, o0 * (unsigned)sizeof(*W)), tc = ld(tp, L0, o0 * (unsigned)sizeof(*tp));
        const T a = lev<T>(vm, nz, VM_A, k), b = lev<T>(vm, nz, VM_B, k);
        T rref, rtref, pref;
        if constexpr (TR) {
            rref = ld(rref3, L0, o0 * (unsigned)sizeof(*rref3));
            r0 = rref + r0;
            rw = ld(rref3, L0, ow * (unsigned)sizeof(*rref3)) + rw;
            rs = ld(rref3, L0, os * (unsigned)sizeof(*rref3)) + rs;
            rtref = ld(rtref3, L0, o0 * (unsigned)sizeof(*rtref3));
            pref = ld(pref3, L0, o0 * (unsigned)sizeof(*pref3));
        } else {
            rref = lev<T>(vm, nz, VM_RHO, k);
            rtref = lev<T>(vm, nz, VM_RT, k);
            pref = lev<T>(vm, nz, VM_P, k);
            r0 = rref + r0;
            rw = rref + rw;
            rs = rref + rs;
        }
        const T u = Uc / (T(0.5) * (rw + r0));
        const T v = Vc / (T(0.5) * (rs + r0));
        const T w = (k == 0) ? T(0) : Wc / (a * r0 + b * rbelow);
        const T th = (rtref + tc) / r0;
        const T pps = pref * xexpm1(T(kGamma) * xlog1p(tc / rtref));
        const T cs = T(kGamma) * (pref + pps) / (rtref + tc);
        st(uo, L0, o0 * (unsigned)sizeof(*uo), u);
        st(vo, L0, o0 * (unsigned)sizeof(*vo), v);
        st(wo, L0, o0 * (unsigned)sizeof(*wo), w);
        st(tho, L0, o0 * (unsigned)sizeof(*tho), th);
        st(P0o, L0, o0 * (unsigned)sizeof(*P0o), pps - cs * tc);
        st(Cso, L0, o0 * (unsigned)sizeof(*Cso), cs);
        if constexpr (TR) {
            const T mx = T(0.5) * (su0 * Uc + su1 * ld(U, L0, oe * (unsigned)sizeof(*U)));
            const T my = T(0.5) * (sv0 * Vc + sv1 * ld(V, L0, on * (unsigned)sizeof(*V)));
            const T df = lev<T>(vm, nz, VM_DF, k);
            const T e = df * ((a * mx + b * mxb) + (a * my + b * myb));
            st(omo, L0, o0 * (unsigned)sizeof(*omo), (k == 0) ? T(0) : Wc - e);
            mxb = mx;
            myb = my;
        }
        rbelow = r0;
    }
}

// Geometry of the faces a column's fluxes use (terrain): the face Jacobians
// and slopes of the neighbouring columns.
template <typename T>
__device__ __forceinline__ T geo_at(const double *__restrict__ g, unsigned o, int f)
{
    return (T)g[(size_t)o * GEO_NFIELDS + f];
}

// Value of a column quantity at level k with the zero-gradient ghost below
// the column and, above it, the top value repeated (cells) or 0 (level
// faces, whose face nz is the rigid lid).
template <typename T>
__device__ __forceinline__ T col_at(const T *__restrict__ a, size_t plane, unsigned o, int k, int nz,
                                    bool zero_top)
{
    if (k >= nz) return zero_top ? T(0) : ld(a, (size_t)(nz - 1) * plane, o * (unsigned)sizeof(T));
    return ld(a, (size_t)(k < 0 ? 0 : k) * plane, o * (unsigned)sizeof(T));
}

template <typename T, bool TR>
__global__ __launch_bounds__(kRowX * kRowY) void k_slow_flux_col(Group gr)
{
    const Col c = locate_col(gr);
    if (!c.active) return;
    const MemberDev *m = c.m;
    const double *__restrict__ vm = m->vm;
    const double *__restrict__ geo = m->geo;
    const int nz = c.nz;
    const size_t P = c.plane;
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
    const unsigned o0 = c.off(0, 0);
    const unsigned oxm2 = c.off(-2, 0), oxm1 = c.off(-1, 0), oxp1 = c.off(1, 0), oxp2 = c.off(2, 0);
    const unsigned oym2 = c.off(0, -2), oym1 = c.off(0, -1), oyp1 = c.off(0, 1), oyp2 = c.off(0, 2);
    const unsigned omp = c.off(-1, 1), opm = c.off(1, -1);
    // face Jacobians (1 on flat ground)
    T jum = T(1), ju0 = T(1), jup = T(1), jvm = T(1), jv0 = T(1), jvp = T(1);
    T jvw0 = T(1), jvw1 = T(1), jus0 = T(1), jus1 = T(1), jc = T(1);
    if constexpr (TR) {
        jum = geo_at<T>(geo, oxm1, GEO_JU);
        ju0 = geo_at<T>(geo, o0, GEO_JU);
        jup = geo_at<T>(geo, oxp1, GEO_JU);
        jvm = geo_at<T>(geo, oym1, GEO_JV);
        jv0 = geo_at<T>(geo, o0, GEO_JV);
        jvp = geo_at<T>(geo, oyp1, GEO_JV);
        jvw0 = geo_at<T>(geo, oxm1, GEO_JV);
        jvw1 = geo_at<T>(geo, omp, GEO_JV);
        jus0 = geo_at<T>(geo, oym1, GEO_JU);
        jus1 = geo_at<T>(geo, opm, GEO_JU);
        jc = geo_at<T>(geo, o0, GEO_J);
    }
    // vertical fluxes through the level face below the current level (S_U,
    // S_V, R_Theta) and through the cell centre below the current level face
    // (S_W), carried from one level to the next
    T fzu = T(0), fzv = T(0), gzt = T(0), fzw = T(0);
    T Ub0 = T(0), Ub1 = T(0), Vb0 = T(0), Vb1 = T(0);
    for (int k = 0; k < nz; ++k) {
        const size_t L0 = (size_t)k * P;
        const T rdz = lev<T>(vm, nz, VM_RDZ, k);
        // ---- S_U ----
        {
            const T ux0 = ld(uu, L0, oxm2 * (unsigned)sizeof(*uu)), ux1 = ld(uu, L0, oxm1 * (unsigned)sizeof(*uu)), ux2 = ld(uu, L0, o0 * (unsigned)sizeof(*uu)), ux3 = ld(uu, L0, oxp1 * (unsigned)sizeof(*uu)),
                    ux4 = ld(uu, L0, oxp2 * (unsigned)sizeof(*uu));
            const T uy0 = ld(uu, L0, oym2 * (unsigned)sizeof(*uu)), uy1 = ld(uu, L0, oym1 * (unsigned)sizeof(*uu)), uy2 = ld(uu, L0, oyp1 * (unsigned)sizeof(*uu)), uy3 = ld(uu, L0, oyp2 * (unsigned)sizeof(*uu));
            // flux through level face k+1 (the lid at the top)
            T fz1 = T(0);
            if (k + 1 < nz) {
                const size_t L1 = L0 + P;
                const T mz = T(0.5) * (ld(Wz, L1, oxm1 * (unsigned)sizeof(*Wz)) + ld(Wz, L1, o0 * (unsigned)sizeof(*Wz)));
                fz1 = mz * kface(col_at(uu, P, o0, k - 1, nz, false), ux2, ld(uu, L1, o0 * (unsigned)sizeof(*uu)),
                                 col_at(uu, P, o0, k + 2, nz, false), mz);
            }
            T m0, m1, n0, n1;
            const T Um = ld(U, L0, oxm1 * (unsigned)sizeof(*U)), U0 = ld(U, L0, o0 * (unsigned)sizeof(*U)), Up = ld(U, L0, oxp1 * (unsigned)sizeof(*U));
            const T Vw0 = ld(V, L0, oxm1 * (unsigned)sizeof(*V)), V00 = ld(V, L0, o0 * (unsigned)sizeof(*V)), Vw1 = ld(V, L0, omp * (unsigned)sizeof(*V)), V01 = ld(V, L0, oyp1 * (unsigned)sizeof(*V));
            if constexpr (TR) {
                m0 = T(0.5) * (jum * Um + ju0 * U0);
                m1 = T(0.5) * (ju0 * U0 + jup * Up);
                n0 = T(0.5) * (jvw0 * Vw0 + jv0 * V00);
                n1 = T(0.5) * (jvw1 * Vw1 + jvp * V01);
            } else {
                m0 = T(0.5) * (Um + U0);
                m1 = T(0.5) * (U0 + Up);
                n0 = T(0.5) * (Vw0 + V00);
                n1 = T(0.5) * (Vw1 + V01);
            }
            const T fx0 = m0 * kface(ux0, ux1, ux2, ux3, m0);
            const T fx1 = m1 * kface(ux1, ux2, ux3, ux4, m1);
            const T fy0 = n0 * kface(uy0, uy1, ux2, uy2, n0);
            const T fy1 = n1 * kface(uy1, ux2, uy2, uy3, n1);
            const T sum = (fx1 - fx0) * rdx + (fy1 - fy0) * rdy + (fz1 - fzu) * rdz;
            T out;
            if constexpr (TR) out = -sum / ju0;
            else out = -sum;
            st(SU, L0, o0 * (unsigned)sizeof(*SU), out);
            fzu = fz1;
        }
        // ---- S_V ----
        {
            const T vy0 = ld(vv, L0, oym2 * (unsigned)sizeof(*vv)), vy1 = ld(vv, L0, oym1 * (unsigned)sizeof(*vv)), vy2 = ld(vv, L0, o0 * (unsigned)sizeof(*vv)), vy3 = ld(vv, L0, oyp1 * (unsigned)sizeof(*vv)),
                    vy4 = ld(vv, L0, oyp2 * (unsigned)sizeof(*vv));
            const T vx0 = ld(vv, L0, oxm2 * (unsigned)sizeof(*vv)), vx1 = ld(vv, L0, oxm1 * (unsigned)sizeof(*vv)), vx2 = ld(vv, L0, oxp1 * (unsigned)sizeof(*vv)), vx3 = ld(vv, L0, oxp2 * (unsigned)sizeof(*vv));
            T fz1 = T(0);
            if (k + 1 < nz) {
                const size_t L1 = L0 + P;
                const T mz = T(0.5) * (ld(Wz, L1, oym1 * (unsigned)sizeof(*Wz)) + ld(Wz, L1, o0 * (unsigned)sizeof(*Wz)));
                fz1 = mz * kface(col_at(vv, P, o0, k - 1, nz, false), vy2, ld(vv, L1, o0 * (unsigned)sizeof(*vv)),
                                 col_at(vv, P, o0, k + 2, nz, false), mz);
            }
            T m0, m1, n0, n1;
            const T Vm = ld(V, L0, oym1 * (unsigned)sizeof(*V)), V0 = ld(V, L0, o0 * (unsigned)sizeof(*V)), Vp = ld(V, L0, oyp1 * (unsigned)sizeof(*V));
            const T Us0 = ld(U, L0, oym1 * (unsigned)sizeof(*U)), U00 = ld(U, L0, o0 * (unsigned)sizeof(*U)), Us1 = ld(U, L0, opm * (unsigned)sizeof(*U)), U10 = ld(U, L0, oxp1 * (unsigned)sizeof(*U));
            if constexpr (TR) {
                m0 = T(0.5) * (jus0 * Us0 + ju0 * U00);
                m1 = T(0.5) * (jus1 * Us1 + jup * U10);
                n0 = T(0.5) * (jvm * Vm + jv0 * V0);
                n1 = T(0.5) * (jv0 * V0 + jvp * Vp);
            } else {
                m0 = T(0.5) * (Us0 + U00);
                m1 = T(0.5) * (Us1 + U10);
                n0 = T(0.5) * (Vm + V0);
                n1 = T(0.5) * (V0 + Vp);
            }
            const T fx0 = m0 * kface(vx0, vx1, vy2, vx2, m0);
            const T fx1 = m1 * kface(vx1, vy2, vx2, vx3, m1);
            const T fy0 = n0 * kface(vy0, vy1, vy2, vy3, n0);
            const T fy1 = n1 * kface(vy1, vy2, vy3, vy4, n1);
            const T sum = (fx1 - fx0) * rdx + (fy1 - fy0) * rdy + (fz1 - fzv) * rdz;
            T out;
            if constexpr (TR) out = -sum / jv0;
            else out = -sum;
            st(SV, L0, o0 * (unsigned)sizeof(*SV), out);
            fzv = fz1;
        }
        // ---- S_W on level face k ----
        {
            const T U0 = ld(U, L0, o0 * (unsigned)sizeof(*U)), U1 = ld(U, L0, oxp1 * (unsigned)sizeof(*U)), V0 = ld(V, L0, o0 * (unsigned)sizeof(*V)), V1 = ld(V, L0, oyp1 * (unsigned)sizeof(*V));
            // flux through the cell centre k (between faces k and k+1)
            const T Wk = ld(Wz, L0, o0 * (unsigned)sizeof(*Wz));
            const T Wk1 = (k + 1 < nz) ? ld(Wz, L0 + P, o0 * (unsigned)sizeof(T)) : T(0);
            const T mz = T(0.5) * (Wk + Wk1);
            const T fc = mz * kface(col_at(ww, P, o0, k - 1, nz, true), ld(ww, L0, o0 * (unsigned)sizeof(*ww)),
                                    col_at(ww, P, o0, k + 1, nz, true), col_at(ww, P, o0, k + 2, nz, true), mz);
            if (k == 0) {
                st(SW, L0, o0 * (unsigned)sizeof(*SW), T(0));
            } else {
                const T wx0 = ld(ww, L0, oxm2 * (unsigned)sizeof(*ww)), wx1 = ld(ww, L0, oxm1 * (unsigned)sizeof(*ww)), wx2 = ld(ww, L0, o0 * (unsigned)sizeof(*ww)), wx3 = ld(ww, L0, oxp1 * (unsigned)sizeof(*ww)),
                        wx4 = ld(ww, L0, oxp2 * (unsigned)sizeof(*ww));
                const T wy0 = ld(ww, L0, oym2 * (unsigned)sizeof(*ww)), wy1 = ld(ww, L0, oym1 * (unsigned)sizeof(*ww)), wy2 = ld(ww, L0, oyp1 * (unsigned)sizeof(*ww)), wy3 = ld(ww, L0, oyp2 * (unsigned)sizeof(*ww));
                const T rdzf = lev<T>(vm, nz, VM_RDZF, k);
                T m0, m1, n0, n1;
                if constexpr (TR) {
                    m0 = T(0.5) * (ju0 * Ub0 + ju0 * U0);
                    m1 = T(0.5) * (jup * Ub1 + jup * U1);
                    n0 = T(0.5) * (jv0 * Vb0 + jv0 * V0);
                    n1 = T(0.5) * (jvp * Vb1 + jvp * V1);
                } else {
                    m0 = T(0.5) * (Ub0 + U0);
                    m1 = T(0.5) * (Ub1 + U1);
                    n0 = T(0.5) * (Vb0 + V0);
                    n1 = T(0.5) * (Vb1 + V1);
                }
                const T fx0 = m0 * kface(wx0, wx1, wx2, wx3, m0);
                const T fx1 = m1 * kface(wx1, wx2, wx3, wx4, m1);
                const T fy0 = n0 * kface(wy0, wy1, wx2, wy2, n0);
                const T fy1 = n1 * kface(wy1, wx2, wy2, wy3, n1);
                const T sum = (fx1 - fx0) * rdx + (fy1 - fy0) * rdy + (fc - fzw) * rdzf;
                T s;
                if constexpr (TR) s = -sum / jc;
                else s = -sum;
                st(SW, L0, o0 * (unsigned)sizeof(*SW), s);
            }
            fzw = fc;
            Ub0 = U0;
            Ub1 = U1;
            Vb0 = V0;
            Vb1 = V1;
        }
        // ---- R_Theta ----
        {
            const T tx0 = ld(th, L0, oxm2 * (unsigned)sizeof(*th)), tx1 = ld(th, L0, oxm1 * (unsigned)sizeof(*th)), tx2 = ld(th, L0, o0 * (unsigned)sizeof(*th)), tx3 = ld(th, L0, oxp1 * (unsigned)sizeof(*th)),
                    tx4 = ld(th, L0, oxp2 * (unsigned)sizeof(*th));
            const T ty0 = ld(th, L0, oym2 * (unsigned)sizeof(*th)), ty1 = ld(th, L0, oym1 * (unsigned)sizeof(*th)), ty2 = ld(th, L0, oyp1 * (unsigned)sizeof(*th)), ty3 = ld(th, L0, oyp2 * (unsigned)sizeof(*th));
            T gz1 = T(0);
            if (k + 1 < nz) {
                const size_t L1 = L0 + P;
                const T mz = ld(Wz, L1, o0 * (unsigned)sizeof(*Wz));
                const T t1 = ld(th, L1, o0 * (unsigned)sizeof(*th));
                const T tl = kface(col_at(th, P, o0, k - 1, nz, false), tx2, t1,
                                   col_at(th, P, o0, k + 2, nz, false), mz);
                T a1, b1;
                if constexpr (TR) {
                    a1 = lev<T>(vm, nz, VM_A, k + 1);
                    b1 = lev<T>(vm, nz, VM_B, k + 1);
                } else {
                    a1 = (T)vm[(size_t)VM_A * nz + k + 1];
                    b1 = (T)vm[(size_t)VM_B * nz + k + 1];
                }
                const T tcen = a1 * t1 + b1 * tx2;
                gz1 = mz * (tl - tcen);
            }
            T m0 = ld(U, L0, o0 * (unsigned)sizeof(*U)), m1 = ld(U, L0, oxp1 * (unsigned)sizeof(*U)), n0 = ld(V, L0, o0 * (unsigned)sizeof(*V)), n1 = ld(V, L0, oyp1 * (unsigned)sizeof(*V));
            if constexpr (TR) {
                m0 = ju0 * m0;
                m1 = jup * m1;
                n0 = jv0 * n0;
                n1 = jvp * n1;
            }
            const T g0 = m0 * (kface(tx0, tx1, tx2, tx3, m0) - T(0.5) * (tx1 + tx2));
            const T g1 = m1 * (kface(tx1, tx2, tx3, tx4, m1) - T(0.5) * (tx2 + tx3));
            const T h0 = n0 * (kface(ty0, ty1, tx2, ty2, n0) - T(0.5) * (ty1 + tx2));
            const T h1 = n1 * (kface(ty1, tx2, ty2, ty3, n1) - T(0.5) * (tx2 + ty2));
            const T sum = (g1 - g0) * rdx + (h1 - h0) * rdy + (gz1 - gzt) * rdz;
            T out;
            if constexpr (TR) out = -sum / jc;
            else out = -sum;
            st(RT, L0, o0 * (unsigned)sizeof(*RT), out);
            gzt = gz1;
        }
    }
}

// One level of the short step's horizontally explicit part in a column:
// its loaded inputs and what the vertical part takes from it.
template <typename T>
struct ColLevel {
    T pc, P0c, Csc, thc, Wc, SWc, rpc;   // own-column inputs (pc = p')
    T rt, tt;                            // rho' and Theta' after the horizontal divergences
    T mx, my;                            // terrain: slope-weighted new momenta at the centre
};

// p' = P0 + C Theta' of column offset o at level k
template <typename T>
__device__ __forceinline__ T pres_at(const T *__restrict__ P0, const T *__restrict__ Cs,
                                     const T *__restrict__ tp, size_t L0, unsigned o)
{
    const unsigned ob = o * (unsigned)sizeof(T);
    return ld(P0, L0, ob) + ld(Cs, L0, ob) * ld(tp, L0, ob);
}

// d p'/d zeta at a cell centre from p' one level below, at and above (the
// mean of the differences over its two level faces; the one inner face at
// the lowest and highest cell), rdzf of the cell's lower and upper faces
template <typename T>
__device__ __forceinline__ T ddz_col(T pm, T p0, T pp, T rdzf_lo, T rdzf_hi, int k, int nz)
{
    const T dlo = (p0 - pm) * rdzf_lo, dhi = (pp - p0) * rdzf_hi;
    return (k == 0) ? dhi : ((k == nz - 1) ? dlo : T(0.5) * (dlo + dhi));
}

template <typename T, typename S, bool TR>
__global__ __launch_bounds__(kRowX * kRowY) void k_short_step_col(Group gr, double frac)
{
    const Col c = locate_col(gr);
    if (!c.active) return;
    const MemberDev *m = c.m;
    const double *__restrict__ vm = m->vm;
    const double *__restrict__ geo = m->geo;
    const int nz = c.nz;
    const size_t P = c.plane;
    const double dtau_d = m->dt * frac;
    const T dt = (T)dtau_d;
    const T rdx = (T)m->rdx, rdy = (T)m->rdy;
    const T *__restrict__ rp = (const T *)buf(m, gr.src, 0);
    const T *__restrict__ U = (const T *)buf(m, gr.src, 1);
    const T *__restrict__ V = (const T *)buf(m, gr.src, 2);
    const T *__restrict__ W = (const T *)buf(m, gr.src, 3);
    const T *__restrict__ tp = (const T *)buf(m, gr.src, 4);
    T *__restrict__ rpo = (T *)buf(m, gr.dst, 0);
    T *__restrict__ Uo = (T *)buf(m, gr.dst, 1);
    T *__restrict__ Vo = (T *)buf(m, gr.dst, 2);
    T *__restrict__ Wo = (T *)buf(m, gr.dst, 3);
    T *__restrict__ tpo = (T *)buf(m, gr.dst, 4);
    const T *__restrict__ SU = (const T *)m->slow[0];
    const T *__restrict__ SV = (const T *)m->slow[1];
    const T *__restrict__ SW = (const T *)m->slow[2];
    const T *__restrict__ RT = (const T *)m->slow[3];
    const T *__restrict__ ths = (const T *)m->slow[4];
    const T *__restrict__ P0 = (const T *)m->slow[5];
    const T *__restrict__ Cs = (const T *)m->slow[6];
    S *__restrict__ cpr = (S *)m->col[0];   // modified upper diagonal
    S *__restrict__ dpr = (S *)m->col[1];   // modified right-hand side
    S *__restrict__ rhs = (S *)m->col[2];   // rho' with W+ = 0
    S *__restrict__ ths_ = (S *)m->col[3];  // Theta' with W+ = 0
    const unsigned o0 = c.off(0, 0), ow = c.off(-1, 0), oe = c.off(1, 0), os = c.off(0, -1),
                   on = c.off(0, 1);
    T ju0 = T(1), ju1 = T(1), jv0 = T(1), jv1 = T(1), rjc = T(1);
    T su0 = T(0), su1 = T(0), sv0 = T(0), sv1 = T(0), fwm = T(0), fem = T(0), fsm = T(0), fnm = T(0);
    double jcol = 1.0;
    if constexpr (TR) {
        ju0 = geo_at<T>(geo, o0, GEO_JU);
        ju1 = geo_at<T>(geo, oe, GEO_JU);
        jv0 = geo_at<T>(geo, o0, GEO_JV);
        jv1 = geo_at<T>(geo, on, GEO_JV);
        su0 = geo_at<T>(geo, o0, GEO_SU);
        su1 = geo_at<T>(geo, oe, GEO_SU);
        sv0 = geo_at<T>(geo, o0, GEO_SV);
        sv1 = geo_at<T>(geo, on, GEO_SV);
        jcol = geo[(size_t)o0 * GEO_NFIELDS + GEO_J];
        rjc = T(1) / (T)jcol;
        fwm = su0 / ju0;
        fem = su1 / ju1;
        fsm = sv0 / jv0;
        fnm = sv1 / jv1;
    }
    // p' of the five columns (centre, west, east, south, north) at three
    // consecutive levels: window[0] = level j - 1, [1] = j, [2] = j + 1 for the
    // level j whose horizontal part comes next (terrain needs d p'/d zeta)
    T pwin[3][5];
    auto load_p = [&](int k, T (&pv)[5]) {
        const size_t L0 = (size_t)k * P;
        pv[0] = pres_at(P0, Cs, tp, L0, o0);
        pv[1] = pres_at(P0, Cs, tp, L0, ow);
        pv[2] = pres_at(P0, Cs, tp, L0, oe);
        pv[3] = pres_at(P0, Cs, tp, L0, os);
        pv[4] = pres_at(P0, Cs, tp, L0, on);
    };
    // horizontally explicit part of level j (p' window centred on j)
    auto horizontal = [&](int j, ColLevel<T> &lv) {
        const size_t L0 = (size_t)j * P;
        const T pc = pwin[1][0], pw = pwin[1][1], pe = pwin[1][2], ps = pwin[1][3], pn = pwin[1][4];
        lv.pc = pc;
        lv.P0c = ld(P0, L0, o0 * (unsigned)sizeof(*P0));
        lv.Csc = ld(Cs, L0, o0 * (unsigned)sizeof(*Cs));
        T cw = T(0), ce = T(0), cs = T(0), cn = T(0);
        if constexpr (TR) {
            const T rlo = lev<T>(vm, nz, VM_RDZF, j), rhi = lev<T>(vm, nz, VM_RDZF, j + 1 < nz ? j + 1 : j);
            const T dc = lev<T>(vm, nz, VM_DC, j);
            T g[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) g[q] = ddz_col(pwin[0][q], pwin[1][q], pwin[2][q], rlo, rhi, j, nz);
            cw = (dc * fwm) * (T(0.5) * (g[1] + g[0]));
            ce = (dc * fem) * (T(0.5) * (g[0] + g[2]));
            cs = (dc * fsm) * (T(0.5) * (g[3] + g[0]));
            cn = (dc * fnm) * (T(0.5) * (g[0] + g[4]));
        }
        const T thc = ld(ths, L0, o0 * (unsigned)sizeof(*ths)), thw = ld(ths, L0, ow * (unsigned)sizeof(*ths)), the = ld(ths, L0, oe * (unsigned)sizeof(*ths)), tsth = ld(ths, L0, os * (unsigned)sizeof(*ths)),
                tnth = ld(ths, L0, on * (unsigned)sizeof(*ths));
        lv.thc = thc;
        const T U0 = ld(U, L0, o0 * (unsigned)sizeof(*U)), U1 = ld(U, L0, oe * (unsigned)sizeof(*U)), SU0 = ld(SU, L0, o0 * (unsigned)sizeof(*SU)), SU1 = ld(SU, L0, oe * (unsigned)sizeof(*SU));
        const T V0 = ld(V, L0, o0 * (unsigned)sizeof(*V)), V1 = ld(V, L0, on * (unsigned)sizeof(*V)), SV0 = ld(SV, L0, o0 * (unsigned)sizeof(*SV)), SV1 = ld(SV, L0, on * (unsigned)sizeof(*SV));
        lv.rpc = ld(rp, L0, o0 * (unsigned)sizeof(*rp));
        lv.Wc = ld(W, L0, o0 * (unsigned)sizeof(*W));
        lv.SWc = ld(SW, L0, o0 * (unsigned)sizeof(*SW));
        const T RTc = ld(RT, L0, o0 * (unsigned)sizeof(*RT)), tpc = ld(tp, L0, o0 * (unsigned)sizeof(*tp));
        const T fw = T(0.5) * (thw + thc), fe = T(0.5) * (thc + the);
        const T fs = T(0.5) * (tsth + thc), fn = T(0.5) * (thc + tnth);
        T up0, up1, vp0, vp1, div, tdiv;
        if constexpr (TR) {
            up0 = U0 + dt * (SU0 - ((pc - pw) * rdx - cw));
            up1 = U1 + dt * (SU1 - ((pe - pc) * rdx - ce));
            vp0 = V0 + dt * (SV0 - ((pc - ps) * rdy - cs));
            vp1 = V1 + dt * (SV1 - ((pn - pc) * rdy - cn));
            const T mu0 = ju0 * up0, mu1 = ju1 * up1, mv0 = jv0 * vp0, mv1 = jv1 * vp1;
            div = ((mu1 - mu0) * rdx + (mv1 - mv0) * rdy) * rjc;
            tdiv = ((fe * mu1 - fw * mu0) * rdx + (fn * mv1 - fs * mv0) * rdy) * rjc;
            lv.mx = T(0.5) * (su0 * up0 + su1 * up1);
            lv.my = T(0.5) * (sv0 * vp0 + sv1 * vp1);
        } else {
            up0 = U0 + dt * (SU0 - (pc - pw) * rdx);
            up1 = U1 + dt * (SU1 - (pe - pc) * rdx);
            vp0 = V0 + dt * (SV0 - (pc - ps) * rdy);
            vp1 = V1 + dt * (SV1 - (pn - pc) * rdy);
            div = (up1 - up0) * rdx + (vp1 - vp0) * rdy;
            tdiv = (fe * up1 - fw * up0) * rdx + (fn * vp1 - fs * vp0) * rdy;
            lv.mx = lv.my = T(0);
        }
        st(Uo, L0, o0 * (unsigned)sizeof(*Uo), up0);
        st(Vo, L0, o0 * (unsigned)sizeof(*Vo), vp0);
        lv.rt = lv.rpc - dt * div;
        lv.tt = tpc + dt * (RTc - tdiv);
    };

    const S be = (S)m->beta, dts = (S)dtau_d;
    const S one_m_be = S(1) - be;
    const S mu = be * be * dts * dts;
    const S grav = (S)kGrav;
    const S rj = S(1) / (S)jcol;
    auto rdz_of = [&](int k) -> S {
        const S r = lev<S>(vm, nz, VM_RDZ, k);
        return TR ? r * rj : r;
    };
    auto rdzf_of = [&](int k) -> S {
        const S r = lev<S>(vm, nz, VM_RDZF, k);
        return TR ? r * rj : r;
    };
    // theta_s on level face k from the cells below and above it (0 on the lids)
    auto face_th = [&](int k, T th_up, T th_dn) -> S {
        if (k == 0 || k >= nz) return S(0);
        return lev<S>(vm, nz, VM_A, k) * (S)th_up + lev<S>(vm, nz, VM_B, k) * (S)th_dn;
    };
    // terrain: the slope part E of Omega on level face k (0 on the lids)
    auto slope_E = [&](int k, T mx_up, T my_up, T mx_dn, T my_dn) -> S {
        if (!TR || k == 0 || k >= nz) return S(0);
        const S a = lev<S>(vm, nz, VM_A, k), b = lev<S>(vm, nz, VM_B, k);
        return lev<S>(vm, nz, VM_DF, k) * ((a * (S)mx_up + b * (S)mx_dn) + (a * (S)my_up + b * (S)my_dn));
    };

    // ---- upward pass: horizontal part one level ahead, then the row of
    // level face k and its forward elimination ----
    if constexpr (TR) {
        load_p(0, pwin[1]);
#pragma unroll
        for (int q = 0; q < 5; ++q) pwin[0][q] = pwin[1][q];   // unused below the column
        if (nz > 1) load_p(1, pwin[2]);
    } else {
        load_p(0, pwin[1]);
    }
    ColLevel<T> cur, nxt;
    horizontal(0, cur);
    S thf_k = S(0), Ef_k = S(0);            // face k (the lower lid for k = 0)
    S Cm = S(0), tfm = S(0), pEm = S(0), rEm = S(0), rdzm = S(0);
    S cprev = S(0), dprev = S(0);
    for (int k = 0; k < nz; ++k) {
        const bool last = (k + 1 == nz);
        if (!last) {
            if constexpr (TR) {
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    pwin[0][q] = pwin[1][q];
                    pwin[1][q] = pwin[2][q];
                }
                if (k + 2 < nz) load_p(k + 2, pwin[2]);
            } else {
                load_p(k + 1, pwin[1]);
            }
            horizontal(k + 1, nxt);
        }
        // the faces of level k: k (carried) and k + 1
        const S thf_k1 = last ? S(0) : face_th(k + 1, nxt.thc, cur.thc);
        const S Ef_k1 = last ? S(0) : slope_E(k + 1, nxt.mx, nxt.my, cur.mx, cur.my);
        const S Wf_k = (S)cur.Wc, Wf_k1 = last ? S(0) : (S)nxt.Wc;
        const S rdzp = rdz_of(k);
        // the state level k reaches with W+ = 0
        const S f = one_m_be * dts * rdzp;
        S thE = (S)cur.tt - f * (thf_k1 * Wf_k1 - thf_k * Wf_k);
        S rhE = (S)cur.rt - f * (Wf_k1 - Wf_k);
        if constexpr (TR) {
            const S g = dts * rdzp;
            thE = thE + g * (thf_k1 * Ef_k1 - thf_k * Ef_k);
            rhE = rhE + g * (Ef_k1 - Ef_k);
        }
        const S Cc = (S)cur.Csc;
        const S pE = be * ((S)cur.P0c + Cc * thE) + one_m_be * (S)cur.pc;
        const S rEs = be * rhE + one_m_be * (S)cur.rpc;
        // row of level face k
        S a, b, cc, d;
        if (k == 0) {
            a = S(0);
            b = S(1);
            cc = S(0);
            d = S(0);
        } else {
            const S rdzf = rdzf_of(k);
            const S av = lev<S>(vm, nz, VM_A, k), bv = lev<S>(vm, nz, VM_B, k);
            a = -mu * Cm * tfm * (rdzf * rdzm) + mu * grav * bv * rdzm;
            cc = last ? S(0) : -mu * Cc * thf_k1 * (rdzf * rdzp) - mu * grav * av * rdzp;
            b = S(1) + mu * thf_k * (Cc * rdzp + Cm * rdzm) * rdzf + mu * grav * (av * rdzp - bv * rdzm);
            d = (S)cur.Wc + dts * (S)cur.SWc - (dts * rdzf) * (pE - pEm) -
                dts * grav * (av * rEs + bv * rEm);
        }
        // Thomas: forward elimination
        const S rden = solve_rcp(k == 0 ? b : b - a * cprev);
        const S cpk = cc * rden;
        const S dpk = (k == 0 ? d : d - a * dprev) * rden;
        const size_t Lk = (size_t)k * P;
        const unsigned sb = o0 * (unsigned)sizeof(S);
        st(cpr, Lk, sb, cpk);
        st(dpr, Lk, sb, dpk);
        st(rhs, Lk, sb, rhE);
        st(ths_, Lk, sb, thE);
        cprev = cpk;
        dprev = dpk;
        Cm = Cc;
        tfm = thf_k;
        pEm = pE;
        rEm = rEs;
        rdzm = rdzp;
        thf_k = thf_k1;
        Ef_k = Ef_k1;
        if (!last) cur = nxt;
    }
    // ---- downward pass: back substitution and the rho', Theta' updates ----
    S xu = S(0);
    const unsigned tb = o0 * (unsigned)sizeof(T), sb = o0 * (unsigned)sizeof(S);
    T th_k = ld(ths, (size_t)(nz - 1) * P, tb);
    S thf_up = S(0);   // face k + 1 (the lid above the top level)
    for (int k = nz - 1; k >= 0; --k) {
        const size_t Lk = (size_t)k * P;
        // the scratch was written by this lane on the way up
        const S x = ld(dpr, Lk, sb) - ld(cpr, Lk, sb) * xu;
        const T th_dn = k > 0 ? ld(ths, Lk - P, tb) : T(0);
        const S thf_k = face_th(k, th_k, th_dn);
        const S f = be * dts * rdz_of(k);
        const S rpn = ld(rhs, Lk, sb) - f * (xu - x);
        const S tpn = ld(ths_, Lk, sb) - f * (thf_up * xu - thf_k * x);
        st(Wo, Lk, tb, (T)x);
        st(rpo, Lk, tb, (T)rpn);
        st(tpo, Lk, tb, (T)tpn);
        xu = x;
        thf_up = thf_k;
        th_k = th_dn;
    }
}

// The one-lane-per-column kernels of the i-fastest layout: kind 0 slow
// prep, 1 slow flux, 2 short step (forward-backward, undamped).
template <typename T, typename S>
hipError_t run_cols(int kind, const Group &gr, double frac, hipStream_t s)
{
    const dim3 grid(((gr.nx1 + kRowX - 1) / kRowX) * ((gr.ny1 + kRowY - 1) / kRowY));
    const dim3 block(kRowX * kRowY);
    if (kind == 0) {
        if (gr.terrain) hipLaunchKernelGGL((k_slow_prep_col<T, true>), grid, block, 0, s, gr);
        else hipLaunchKernelGGL((k_slow_prep_col<T, false>), grid, block, 0, s, gr);
    } else if (kind == 1) {
        if (gr.terrain) hipLaunchKernelGGL((k_slow_flux_col<T, true>), grid, block, 0, s, gr);
        else hipLaunchKernelGGL((k_slow_flux_col<T, false>), grid, block, 0, s, gr);
    } else {
        if (gr.terrain) hipLaunchKernelGGL((k_short_step_col<T, S, true>), grid, block, 0, s, gr, frac);
        else hipLaunchKernelGGL((k_short_step_col<T, S, false>), grid, block, 0, s, gr, frac);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_columns(int kind, int prec, const Group &gr, double frac, hipStream_t s)
{
    if (gr.nm != 1 || gr.nx1 < 1 || gr.ny1 < 1) return hipErrorInvalidValue;
    switch (prec) {
    case 0: return run_cols<double, double>(kind, gr, frac, s);
    case 1: return run_cols<float, float>(kind, gr, frac, s);
    case 2: return run_cols<float, double>(kind, gr, frac, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hv
