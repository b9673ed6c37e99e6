// Per-lane steps of the block-relaxation half-sweep (Section 3 motifs,
// Section 7 3D tweed), written once for the device kernel and for the host
// emulation used by the CPU tests of the block tables.
//
// Every block of one colour is solved exactly with the other colour frozen.
// A workgroup owns whole blocks.  Each lane owns one chunk of <= CH collinear
// points: it builds their right-hand sides (f minus the off-block neighbour
// couplings), eliminates the chunk interior with zero end values and keeps the
// two spikes (responses to the predecessor node and to its own last point).
// The chunk end points form the block's reduced system -- a chain, a spider
// (m-legged Thomas, eq. mLThomas) or a ring (circulant Thomas, eq. CircTri) --
// solved in LDS by one lane per block.  Each lane then back-substitutes its
// chunk from registers, so u is read and written once per half-sweep.
#pragma once

#include "twmg_internal.h"

namespace twmg {

__host__ __device__ __forceinline__ long long dir_off(const Dims &d, int dir)
{
    return (dir & 1) ? d.st[dir >> 1] : -d.st[dir >> 1];
}

// coefficient array of direction d (compile-time d after unrolling)
template <typename T> __host__ __device__ __forceinline__ const T *coef_arr(const Coef<T> &cf, int d)
{
    return (d & 1) ? cf.hi[d >> 1] : cf.lo[d >> 1];
}

// coefficient array of a per-lane direction d (selects, no indexed loads)
template <typename T, int DIM> __host__ __device__ __forceinline__ const T *coef_arr_rt(const Coef<T> &cf, int d)
{
    const T *p = cf.lo[0];
    p = (d == 1) ? cf.hi[0] : p;
    p = (d == 2) ? cf.lo[1] : p;
    p = (d == 3) ? cf.hi[1] : p;
    if (DIM == 3) {
        p = (d == 4) ? cf.lo[2] : p;
        p = (d == 5) ? cf.hi[2] : p;
    }
    return p;
}

template <typename T, int DIM> __host__ __device__ __forceinline__ T diag_at(const Coef<T> &cf, int i, int j, int l)
{
    T s = cf.dg[0][i] + cf.dg[1][j];
    if (DIM == 3) s += cf.dg[2][l];
    return s;
}

// the reduced-system arrays of one workgroup (LDS on the device)
template <typename T> struct RedArrays {
    T *low;  // coupling of node q's row to its predecessor node
    T *ds;   // diagonal (own part)
    T *rs;   // right-hand side (own part)
    T *dn;   // diagonal contribution through the successor chunk's interior
    T *up;   // coupling to the successor node
    T *rn;   // right-hand-side contribution through the successor chunk's interior
    T *x;    // solution
    T *aux;  // coupling of the successor node's row back to q (branch rows)
};

template <typename T> struct LaneState {
    T D[CH], G[CH], S[CH]; // interior elimination: delta, gamma, left spike
    int L, sg, prev, cax;
    bool hp;
    long long p0, step;
    const T *Pfwd;
};

// Phase 1: right-hand sides, chunk-interior elimination, reduced equations.
template <typename T, int DIM>
__host__ __device__ __forceinline__ void sweep_phase1(const Dims &d, const Coef<T> &cf, const T *__restrict__ ub,
                                                      const T *__restrict__ fb, const Chunk &ch, int t,
                                                      const RedArrays<T> &s, LaneState<T> &st)
{
    const int L = ch.len;
    const int ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const uint8_t fl = ch.flags;
    const bool hp = fl & CF_PREV, hn = fl & CF_NEXT, nd = fl & CF_NEXT_DIRECT, jn = fl & CF_JUNCTION;
    const int c0x = ch.c0[0], c0y = ch.c0[1], c0z = (DIM == 3) ? ch.c0[2] : 0;
    const long long step = sg * d.st[ax];
    const long long p0 = c0x + c0y * d.st[1] + (DIM == 3 ? c0z * d.st[2] : 0);
    const int cax = (ax == 0) ? c0x : ((ax == 1) ? c0y : c0z);
    const T *Pback = coef_arr_rt<T, DIM>(cf, ad ^ 1);
    const T *Pfwd = coef_arr_rt<T, DIM>(cf, ad);
    const int ex = (ax == 0) ? sg : 0, ey = (ax == 1) ? sg : 0, ez = (ax == 2) ? sg : 0;
    st.L = L;
    st.sg = sg;
    st.prev = ch.prev;
    st.hp = hp;
    st.p0 = p0;
    st.step = step;
    st.cax = cax;
    st.Pfwd = Pfwd;

    T Gp = 0, Dp = 0, Sp = hp ? T(1) : T(0);
    T rL = 0, aL = 0, bL = 0, cL = 0;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        if (k < L) {
            const int ci = c0x + k * ex, cj = c0y + k * ey, cl = c0z + k * ez;
            const long long idx = p0 + k * step;
            unsigned inb = 0;
            if (k > 0 || hp) inb |= 1u << (ad ^ 1);
            if (k < L - 1) inb |= 1u << ad;
            else {
                if (hn) inb |= 1u << ch.nextdir;
                if (jn) inb |= ch.jmask;
            }
            T r = fb[idx];
#pragma unroll
            for (int dd = 0; dd < 2 * DIM; ++dd) {
                if (!((inb >> dd) & 1u)) {
                    const int cc = (dd >> 1) == 0 ? ci : ((dd >> 1) == 1 ? cj : cl);
                    r -= coef_arr<T>(cf, dd)[cc] * ub[idx + dir_off(d, dd)];
                }
            }
            const T b = diag_at<T, DIM>(cf, ci, cj, cl);
            const int ca = cax + k * sg;
            const T a = Pback[ca];
            if (k < L - 1) {
                const T cc = Pfwd[ca];
                const T inv = T(1) / (b - a * Gp);
                st.G[k] = cc * inv;
                st.D[k] = (r - a * Dp) * inv;
                st.S[k] = -a * Sp * inv;
                Gp = st.G[k];
                Dp = st.D[k];
                Sp = st.S[k];
            } else {
                rL = r;
                aL = a;
                bL = b;
                if (hn) {
                    const int nx = ch.nextdir, na = nx >> 1, ns = (nx & 1) ? 1 : -1;
                    const int cn = (na == 0) ? ci : ((na == 1) ? cj : cl);
                    cL = coef_arr_rt<T, DIM>(cf, nx)[cn];
                    if (nd) {
                        // the successor's row coefficient back toward this point
                        s.aux[t] = coef_arr_rt<T, DIM>(cf, nx ^ 1)[cn + ns];
                    }
                }
            }
        }
    }
    // first-point values of the zero-end interior solution y and its spikes v, w
    T yl = 0, vl = 0, wl = 0, y = 0, v = 0, ww = 0;
#pragma unroll
    for (int k = CH - 2; k >= 0; --k) {
        if (k == L - 2) {
            y = st.D[k];
            v = st.S[k];
            ww = -st.G[k];
            yl = y;
            vl = v;
            wl = ww;
        } else if (k < L - 2) {
            y = st.D[k] - st.G[k] * y;
            v = st.S[k] - st.G[k] * v;
            ww = -st.G[k] * ww;
        }
    }
    if (L >= 2) {
        s.ds[t] = bL + aL * wl;
        s.low[t] = hp ? aL * vl : T(0);
        s.rs[t] = rL - aL * yl;
    } else {
        s.ds[t] = bL;
        s.low[t] = hp ? aL : T(0);
        s.rs[t] = rL;
    }
    if (!hn) {
        s.dn[t] = 0;
        s.up[t] = 0;
        s.rn[t] = 0;
    } else if (nd) {
        s.dn[t] = 0;
        s.up[t] = cL;
        s.rn[t] = 0;
    }
    if (hp && L >= 2) {
        const T cprev = Pfwd[cax - sg];
        s.dn[ch.prev] = cprev * v;
        s.up[ch.prev] = cprev * ww;
        s.rn[ch.prev] = -cprev * y;
    }
}

// Phase 2: one lane solves one block's reduced system.
template <typename T> __host__ __device__ void reduced_solve(const Block &bk, const RedArrays<T> &r)
{
    const int s = bk.first, e = s + bk.count;
    for (int q = s; q < e; ++q) {
        r.ds[q] += r.dn[q];
        r.rs[q] += r.rn[q];
    }
    if (bk.type == BT_CHAIN) {
        T g = 0, dl = 0;
        for (int q = s; q < e; ++q) {
            const T lo = r.low[q];
            const T inv = T(1) / (r.ds[q] - lo * g);
            g = r.up[q] * inv;
            dl = (r.rs[q] - lo * dl) * inv;
            r.up[q] = g;
            r.rs[q] = dl;
        }
        T x = r.rs[e - 1];
        r.x[e - 1] = x;
        for (int q = e - 2; q >= s; --q) {
            x = r.rs[q] - r.up[q] * x;
            r.x[q] = x;
        }
    } else if (bk.type == BT_SPIDER) {
        // m-legged Thomas: eliminate every leg from its tip toward the branch
        // point, solve the branch row, substitute back out to the tips.
        const int J = e - 1;
        T num = r.rs[J], den = r.ds[J];
        int start = s;
        for (int l = 1; l < bk.m; ++l) {
            const int end = bk.ends[l];
            T g = 0, dl = 0;
            for (int q = start; q <= end; ++q) {
                const T lo = r.low[q];
                const T inv = T(1) / (r.ds[q] - lo * g);
                g = r.up[q] * inv;
                dl = (r.rs[q] - lo * dl) * inv;
                r.up[q] = g;
                r.rs[q] = dl;
            }
            const T dJ = r.aux[end];
            num -= dJ * dl;
            den -= dJ * g;
            start = end + 1;
        }
        {
            T g = 0, dl = 0;
            for (int q = start; q < J; ++q) {
                const T lo = r.low[q];
                const T inv = T(1) / (r.ds[q] - lo * g);
                g = r.up[q] * inv;
                dl = (r.rs[q] - lo * dl) * inv;
                r.up[q] = g;
                r.rs[q] = dl;
            }
            if (J > start) {
                const T lo = r.low[J];
                num -= lo * dl;
                den -= lo * g;
            }
        }
        const T xJ = num / den;
        r.x[J] = xJ;
        start = s;
        for (int l = 1; l < bk.m; ++l) {
            const int end = bk.ends[l];
            T x = xJ;
            for (int q = end; q >= start; --q) {
                x = r.rs[q] - r.up[q] * x;
                r.x[q] = x;
            }
            start = end + 1;
        }
        T x = xJ;
        for (int q = J - 1; q >= start; --q) {
            x = r.rs[q] - r.up[q] * x;
            r.x[q] = x;
        }
    } else {
        // ring: border on the last node; the open tridiagonal rows s..B-1 are
        // solved for the right-hand side (y) and for the border's column (z),
        // then the border row closes the system.
        const int B = e - 1;
        const T colS = r.low[s], colE = r.up[B - 1];
        T g = 0, dy = 0, dz = 0;
        for (int q = s; q < B; ++q) {
            const T lo = (q > s) ? r.low[q] : T(0);
            const T up = (q < B - 1) ? r.up[q] : T(0);
            const T col = (q == s ? colS : T(0)) + (q == B - 1 ? colE : T(0));
            const T inv = T(1) / (r.ds[q] - lo * g);
            g = up * inv;
            dy = (r.rs[q] - lo * dy) * inv;
            dz = (col - lo * dz) * inv;
            r.up[q] = g;
            r.rs[q] = dy;
            r.dn[q] = dz;
        }
        T y = r.rs[B - 1], z = r.dn[B - 1];
        r.x[B - 1] = y;
        r.rn[B - 1] = z;
        for (int q = B - 2; q >= s; --q) {
            y = r.rs[q] - r.up[q] * y;
            z = r.dn[q] - r.up[q] * z;
            r.x[q] = y;
            r.rn[q] = z;
        }
        const T lowB = r.low[B], upB = r.up[B];
        const T xB = (r.rs[B] - lowB * r.x[B - 1] - upB * r.x[s]) / (r.ds[B] - lowB * r.rn[B - 1] - upB * r.rn[s]);
        r.x[B] = xB;
        for (int q = s; q < B; ++q) r.x[q] = r.x[q] - xB * r.rn[q];
    }
}

// Phase 3: back-substitution of the chunk interior from the node values.
template <typename T>
__host__ __device__ __forceinline__ void sweep_phase3(T *__restrict__ ub, int t, const RedArrays<T> &s,
                                                      const LaneState<T> &st)
{
    const T Xp = st.hp ? s.x[st.prev] : T(0);
    const T Xo = s.x[t];
    T x = Xo;
#pragma unroll
    for (int k = CH - 2; k >= 0; --k) {
        if (k <= st.L - 2) {
            x = st.D[k] + st.S[k] * Xp - st.G[k] * x;
            ub[st.p0 + k * st.step] = x;
        }
    }
    ub[st.p0 + (st.L - 1) * st.step] = Xo;
}

} // namespace twmg
