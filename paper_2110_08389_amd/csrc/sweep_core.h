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

// coefficient array of a per-lane direction d, and diagonal part of a per-lane
// axis: offsets into the level's coefficient block
template <typename T, int DIM> __host__ __device__ __forceinline__ const T *coef_arr_rt(const Coef<T> &cf, int d)
{
    return cf.base + d * cf.cs;
}
template <typename T> __host__ __device__ __forceinline__ const T *dg_arr_rt(const Coef<T> &cf, int ax)
{
    return cf.base + (6 + ax) * cf.cs;
}

template <typename T, int DIM> __host__ __device__ __forceinline__ T diag_at(const Coef<T> &cf, int i, int j, int l)
{
    T s = cf.dg[0][i] + cf.dg[1][j];
    if (DIM == 3) s += cf.dg[2][l];
    return s;
}

// 1/x: on the device the hardware reciprocal refined by Newton steps (within
// an ulp of the quotient, and far shorter than a correctly rounded division
// in the sequential chunk elimination); on the host a plain division.
template <typename T> __host__ __device__ __forceinline__ T rcp(T x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(T) == 8) {
        double r = __builtin_amdgcn_rcp(x);
        double e = __builtin_fma(-x, r, 1.0);
        r = __builtin_fma(r, e, r);
        e = __builtin_fma(-x, r, 1.0);
        return __builtin_fma(r, e, r);
    } else {
        float r = __builtin_amdgcn_rcpf(x);
        const float e = __builtin_fmaf(-x, r, 1.0f);
        return __builtin_fmaf(r, e, r);
    }
#else
    return T(1) / x;
#endif
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

// C: the longest chunk the lane may own (CH, or fewer in code compiled for
// short chunks)
template <typename T, int C = CH> struct LaneState {
    T D[C], G[C], S[C]; // interior elimination: delta, gamma, left spike
    int L, prev;
    bool hp;
};

// 32-bit slot of node (i, j, l) within one problem's array (set-up rejects a
// grid whose per-problem array would reach 2^31 entries)
__host__ __device__ __forceinline__ int slot32(const Dims &d, int i, int j, int l)
{
    if (d.layout == LAYOUT_ROW) return i + j * (int)d.st[1] + l * (int)d.st[2];
    if (d.layout == LAYOUT_TWEED3) return (int)plane3_slot(d, plane3(d, i, j, l), i, j, l);
    return col_plane(d, i, j) ? (int)d.nn + j + i * (d.n[1] + 1) : i + j * (int)d.st[1];
}

// slots of node (i, j, l) and of its neighbours x-, x+, y-, y+ (, z-, z+).  In
// a split layout a node's neighbours share its plane unless |i' - j'| <= 1,
// so away from that band they are fixed offsets in the plane.
template <int DIM> struct NbSlots {
    int p, nb[2 * DIM];
};
template <int DIM> __host__ __device__ __forceinline__ NbSlots<DIM> nb_slots(const Dims &d, int i, int j, int l)
{
    NbSlots<DIM> s;
    if (DIM == 3 && d.layout == LAYOUT_TWEED3) {
        // a node whose own primed coordinate is at least 2 below the other two
        // has all six neighbours in its plane, at that plane's fixed offsets;
        // nearer the planes' borders every slot is computed
        const int ip = i < d.n[0] - i ? i : d.n[0] - i, jp = j < d.n[1] - j ? j : d.n[1] - j,
                  lp = l < d.n[2] - l ? l : d.n[2] - l;
        const int pl = (ip <= jp && ip <= lp) ? 0 : (jp <= lp ? 1 : 2);
        const int own = pl == 0 ? ip : (pl == 1 ? jp : lp);
        const int o1 = pl == 0 ? jp : ip, o2 = pl == 2 ? jp : lp;
        s.p = (int)plane3_slot(d, pl, i, j, l);
        if (own + 2 <= o1 && own + 2 <= o2) {
            const int S0 = d.n[0] + 1, S1 = d.n[1] + 1, S2 = d.n[2] + 1;
            // strides of x, y, z in the node's plane
            const int sx = pl == 0 ? 1 : (pl == 1 ? S1 : S2);
            const int sy = pl == 0 ? S0 : (pl == 1 ? 1 : S2 * S0);
            const int sz = pl == 0 ? S0 * S1 : (pl == 1 ? S1 * S0 : 1);
            s.nb[0] = s.p - sx;
            s.nb[1] = s.p + sx;
            s.nb[2] = s.p - sy;
            s.nb[3] = s.p + sy;
            s.nb[2 * DIM - 2] = s.p - sz;
            s.nb[2 * DIM - 1] = s.p + sz;
        } else {
            s.nb[0] = slot32(d, i - 1, j, l);
            s.nb[1] = slot32(d, i + 1, j, l);
            s.nb[2] = slot32(d, i, j - 1, l);
            s.nb[3] = slot32(d, i, j + 1, l);
            s.nb[2 * DIM - 2] = slot32(d, i, j, l - 1);
            s.nb[2 * DIM - 1] = slot32(d, i, j, l + 1);
        }
        return s;
    }
    if (DIM == 3 || d.layout == LAYOUT_ROW) {
        const int S1 = (int)d.st[1], S2 = (int)d.st[2];
        s.p = i + j * S1 + (DIM == 3 ? l * S2 : 0);
        s.nb[0] = s.p - 1;
        s.nb[1] = s.p + 1;
        s.nb[2] = s.p - S1;
        s.nb[3] = s.p + S1;
        if (DIM == 3) {
            s.nb[4] = s.p - S2;
            s.nb[5] = s.p + S2;
        }
        return s;
    }
    const int ip = i < d.n[0] - i ? i : d.n[0] - i, jp = j < d.n[1] - j ? j : d.n[1] - j;
    const int dl = ip - jp;
    if (d.layout != LAYOUT_COLUMNS && dl > -2 && dl < 2) {
        s.p = slot32(d, i, j, 0);
        s.nb[0] = slot32(d, i - 1, j, 0);
        s.nb[1] = slot32(d, i + 1, j, 0);
        s.nb[2] = slot32(d, i, j - 1, 0);
        s.nb[3] = slot32(d, i, j + 1, 0);
        return s;
    }
    const bool col = d.layout == LAYOUT_TWEED ? dl > 0 : (d.layout == LAYOUT_WIREFRAME ? dl < 0 : true);
    if (col) {
        const int S = d.n[1] + 1;
        s.p = (int)d.nn + j + i * S;
        s.nb[0] = s.p - S;
        s.nb[1] = s.p + S;
        s.nb[2] = s.p - 1;
        s.nb[3] = s.p + 1;
    } else {
        const int S = (int)d.st[1];
        s.p = i + j * S;
        s.nb[0] = s.p - 1;
        s.nb[1] = s.p + 1;
        s.nb[2] = s.p - S;
        s.nb[3] = s.p + S;
    }
    return s;
}

// in-block directions of point k of a chunk (bit d set: the neighbour in
// direction d belongs to the block)
__host__ __device__ __forceinline__ unsigned inblock_dirs(const Chunk &ch, int k)
{
    const int L = ch.len, ad = ch.axdir;
    unsigned inb = 0;
    if (k > 0 || (ch.flags & CF_PREV)) inb |= 1u << (ad ^ 1);
    if (k < L - 1) inb |= 1u << ad;
    else {
        if (ch.flags & CF_NEXT) inb |= 1u << ch.nextdir;
        if (ch.flags & CF_JUNCTION) inb |= ch.jmask;
    }
    return inb;
}

// Right-hand side of point k of a chunk without its along-axis couplings: f
// minus the couplings to the neighbours across the chunk axis that lie outside
// the block.  Along the axis every neighbour is in the block except possibly
// at the chunk's two ends (chunk_end_terms).
template <typename T, int DIM>
__host__ __device__ __forceinline__ T point_rhs_across(const Dims &d, const Coef<T> &cf, const T *__restrict__ ub,
                                                       const T *__restrict__ fb, const Chunk &ch, int k)
{
    const int ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int ci = ch.c0[0] + (ax == 0 ? sg * k : 0), cj = ch.c0[1] + (ax == 1 ? sg * k : 0),
              cl = (DIM == 3) ? ch.c0[2] + (ax == 2 ? sg * k : 0) : 0;
    const NbSlots<DIM> s = nb_slots<DIM>(d, ci, cj, cl);
    const unsigned inb = inblock_dirs(ch, k);
    T r = fb[s.p];
#pragma unroll
    for (int q = 0; q < DIM - 1; ++q) {
        // q-th axis other than ax (chosen by selects: compile-time indices only)
        const int a2 = (DIM == 2) ? 1 - ax : (q == 0 ? (ax == 0 ? 1 : 0) : (ax == 2 ? 1 : 2));
        int sm = s.nb[0], sp = s.nb[1];
        if (a2 == 1) {
            sm = s.nb[2];
            sp = s.nb[3];
        }
        if (DIM == 3 && a2 == 2) {
            sm = s.nb[2 * DIM - 2];
            sp = s.nb[2 * DIM - 1];
        }
        const int cc = a2 == 0 ? ci : (a2 == 1 ? cj : cl);
        const T tm = cf.base[(2 * a2) * cf.cs + cc] * ub[sm];
        const T tp = cf.base[(2 * a2 + 1) * cf.cs + cc] * ub[sp];
        r -= ((inb >> (2 * a2)) & 1u) ? T(0) : tm;
        r -= ((inb >> (2 * a2 + 1)) & 1u) ? T(0) : tp;
    }
    return r;
}

// Along-axis couplings of a chunk's end points to neighbours outside the
// block: tb for the first point's predecessor, tf for the last point's
// successor (0 when in the block).
template <typename T, int DIM>
__host__ __device__ __forceinline__ void chunk_end_terms(const Dims &d, const Coef<T> &cf, const T *__restrict__ ub,
                                                         const Chunk &ch, T &tb, T &tf)
{
    const int L = ch.len, ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int e[3] = {ax == 0 ? sg : 0, ax == 1 ? sg : 0, ax == 2 ? sg : 0};
    const int i0 = ch.c0[0], j0 = ch.c0[1], l0 = DIM == 3 ? ch.c0[2] : 0;
    const int iL = i0 + (L - 1) * e[0], jL = j0 + (L - 1) * e[1], lL = l0 + (L - 1) * e[2];
    const int cax0 = ax == 0 ? i0 : (ax == 1 ? j0 : l0), caxL = cax0 + (L - 1) * sg;
    const bool boff = !((inblock_dirs(ch, 0) >> (ad ^ 1)) & 1u);
    const bool foff = !((inblock_dirs(ch, L - 1) >> ad) & 1u);
    // only neighbours outside the block are read (an in-block neighbour is a
    // point of the colour being relaxed, whose cache lines are otherwise only
    // written)
    T ubk = 0, ufw = 0;
    if (boff) ubk = ub[slot32(d, i0 - e[0], j0 - e[1], DIM == 3 ? l0 - e[2] : 0)];
    if (foff) ufw = ub[slot32(d, iL + e[0], jL + e[1], DIM == 3 ? lL + e[2] : 0)];
    tb = boff ? coef_arr_rt<T, DIM>(cf, ad ^ 1)[cax0] * ubk : T(0);
    tf = foff ? coef_arr_rt<T, DIM>(cf, ad)[caxL] * ufw : T(0);
}

// The chunk's two neighbours along its axis: ubk before the first point, ufw
// after the last, each read only when it lies outside the block (otherwise 0;
// chunk_end_terms_v drops its coupling).
template <typename T, int DIM>
__host__ __device__ __forceinline__ void chunk_end_u(const Dims &d, const T *__restrict__ ub, const Chunk &ch, T &ubk,
                                                     T &ufw)
{
    const int L = ch.len, ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int e[3] = {ax == 0 ? sg : 0, ax == 1 ? sg : 0, ax == 2 ? sg : 0};
    const int i0 = ch.c0[0], j0 = ch.c0[1], l0 = DIM == 3 ? ch.c0[2] : 0;
    const int iL = i0 + (L - 1) * e[0], jL = j0 + (L - 1) * e[1], lL = l0 + (L - 1) * e[2];
    const bool boff = !((inblock_dirs(ch, 0) >> (ad ^ 1)) & 1u);
    const bool foff = !((inblock_dirs(ch, L - 1) >> ad) & 1u);
    ubk = 0;
    ufw = 0;
    if (boff) ubk = ub[slot32(d, i0 - e[0], j0 - e[1], DIM == 3 ? l0 - e[2] : 0)];
    if (foff) ufw = ub[slot32(d, iL + e[0], jL + e[1], DIM == 3 ? lL + e[2] : 0)];
}

// chunk_end_terms from the loaded neighbours and the two coefficients: ab, the
// first point's coupling toward its predecessor, and cf_last, the last
// point's toward its successor.
template <typename T>
__host__ __device__ __forceinline__ void chunk_end_terms_v(const Chunk &ch, T ab, T cf_last, T ubk, T ufw, T &tb,
                                                           T &tf)
{
    const int L = ch.len, ad = ch.axdir;
    const bool boff = !((inblock_dirs(ch, 0) >> (ad ^ 1)) & 1u);
    const bool foff = !((inblock_dirs(ch, L - 1) >> ad) & 1u);
    tb = boff ? ab * ubk : T(0);
    tf = foff ? cf_last * ufw : T(0);
}

// Addressing record of a 2D chunk (host, at setup).  Returns false when the
// chunk has more than one point whose cross neighbours are not at the regular
// offsets (never the case for the motifs' layouts; the caller rejects it).
inline bool make_chunk_addr(const Dims &d, const Chunk &ch, ChunkAddr &a)
{
    const int L = ch.len, ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int ex = ax == 0 ? sg : 0, ey = ax == 1 ? sg : 0;
    const int qx = ax == 0 ? 0 : 1, qy = ax == 0 ? 1 : 0; // unit step across the chunk axis
    const int plane = (d.layout != LAYOUT_ROW && col_plane(d, ch.c0[0], ch.c0[1])) ? 1 : 0;
    const int S = plane ? d.n[1] + 1 : (int)d.st[1];
    const bool unit = ax == plane;
    const int dp = sg * (unit ? 1 : S), reg = unit ? S : 1;
    const int p0 = slot32(d, ch.c0[0], ch.c0[1], 0);
    int km = 31, kp = 31, irr_m = 0, irr_p = 0;
    for (int k = 0; k < L; ++k) {
        const int i = ch.c0[0] + k * ex, j = ch.c0[1] + k * ey;
        const int p = slot32(d, i, j, 0);
        if (p != p0 + k * dp) return false; // the chunk leaves its plane
        const int sm = slot32(d, i - qx, j - qy, 0), sp = slot32(d, i + qx, j + qy, 0);
        if (sm != p - reg) {
            if (km != 31) return false;
            km = k;
            irr_m = sm;
        }
        if (sp != p + reg) {
            if (kp != 31) return false;
            kp = k;
            irr_p = sp;
        }
    }
    const unsigned lastinb = inblock_dirs(ch, L - 1);
    const int qd = 2 * (1 - ax); // direction code of the cross axis toward -
    a.p0 = p0;
    a.irr_m = irr_m;
    a.irr_p = irr_p;
    a.meta = (uint32_t)L | ((uint32_t)km << 5) | ((uint32_t)kp << 10) | (((lastinb >> qd) & 1u) << 15) |
             (((lastinb >> (qd + 1)) & 1u) << 16) | ((uint32_t)plane << 17) | ((uint32_t)ax << 18) |
             ((uint32_t)(sg > 0) << 19);
    return true;
}

// addressing record of a 2D chunk of a row-major array (no exceptional points)
__host__ __device__ __forceinline__ ChunkAddr row_chunk_addr(const Dims &d, const Chunk &ch)
{
    const int L = ch.len, ax = ch.axdir >> 1, up = ch.axdir & 1;
    const unsigned lastinb = inblock_dirs(ch, L - 1);
    const int qd = 2 * (1 - ax);
    ChunkAddr a;
    a.p0 = ch.c0[0] + ch.c0[1] * (int)d.st[1];
    a.irr_m = 0;
    a.irr_p = 0;
    a.meta = (uint32_t)L | (31u << 5) | (31u << 10) | (((lastinb >> qd) & 1u) << 15) |
             (((lastinb >> (qd + 1)) & 1u) << 16) | ((uint32_t)ax << 18) | ((uint32_t)up << 19);
    return a;
}

// slot of point k of a chunk from its addressing record
__host__ __device__ __forceinline__ int rec_slot(const Dims &d, const ChunkAddr &a, int k)
{
    const int plane = (a.meta >> 17) & 1, ax = (a.meta >> 18) & 1, up = (a.meta >> 19) & 1;
    const int S = plane ? d.n[1] + 1 : (int)d.st[1];
    const int m = ax == plane ? 1 : S;
    return a.p0 + k * (up ? m : -m);
}

// 2D gather with the addressing record: f minus the off-block cross
// couplings (cm toward -, cp toward +; constant along the chunk) of point k
// The slots point k reads (its own, p, and its cross neighbours pm, pp) and
// whether the last point's neighbours are in the block (skm, skp).
struct RecSlots {
    int p, pm, pp;
    bool skm, skp;
};
__host__ __device__ __forceinline__ RecSlots rec_point_slots(const Dims &d, const ChunkAddr &a, int k)
{
    const uint32_t mt = a.meta;
    const int L = mt & 31, km = (mt >> 5) & 31, kp = (mt >> 10) & 31;
    const int plane = (mt >> 17) & 1, ax = (mt >> 18) & 1, up = (mt >> 19) & 1;
    const int S = plane ? d.n[1] + 1 : (int)d.st[1];
    const bool unit = ax == plane;
    const int m = unit ? 1 : S, reg = unit ? S : 1;
    RecSlots r;
    r.p = a.p0 + k * (up ? m : -m);
    r.pm = k == km ? a.irr_m : r.p - reg;
    r.pp = k == kp ? a.irr_p : r.p + reg;
    const bool last = k == L - 1;
    r.skm = last && ((mt >> 15) & 1);
    r.skp = last && ((mt >> 16) & 1);
    return r;
}

// f minus the two cross couplings, from the loaded values
template <typename T>
__host__ __device__ __forceinline__ T rec_rhs_combine(T fp, T um, T upv, T cm, T cp, bool skm, bool skp)
{
    T r = fp;
    const T tm = cm * um, tp = cp * upv;
    r -= skm ? T(0) : tm;
    r -= skp ? T(0) : tp;
    return r;
}

template <typename T>
__host__ __device__ __forceinline__ T point_rhs_rec(const Dims &d, const ChunkAddr &a, T cm, T cp,
                                                    const T *__restrict__ ub, const T *__restrict__ fb, int k)
{
    const RecSlots q = rec_point_slots(d, a, k);
    return rec_rhs_combine<T>(fb[q.p], ub[q.pm], ub[q.pp], cm, cp, q.skm, q.skp);
}

// the chunk's cross-axis coefficients (2D): toward - and + across its axis
template <typename T>
__host__ __device__ __forceinline__ void chunk_cross_coefs(const Coef<T> &cf, const Chunk &ch, T &cm, T &cp)
{
    const int a2 = 1 - (ch.axdir >> 1);
    // (a select, not ch.c0[a2]: a run-time index would put the chunk in
    // private memory)
    const int cc = a2 == 0 ? ch.c0[0] : ch.c0[1];
    cm = cf.base[(2 * a2) * cf.cs + cc];
    cp = cf.base[(2 * a2 + 1) * cf.cs + cc];
}

// ---- 3D addressing records -------------------------------------------------
// the two axes across chunk axis ax, in increasing order
__host__ __device__ __forceinline__ int cross_axis3(int ax, int q) { return q == 0 ? (ax == 0 ? 1 : 0) : (ax == 2 ? 1 : 2); }

// signed stride between consecutive points of a 3D chunk
__host__ __device__ __forceinline__ int rec3_step(const Dims &d, uint32_t meta)
{
    const int ax = (meta >> 18) & 3, up = (meta >> 20) & 1;
    const int m = d.layout == LAYOUT_TWEED3 ? 1 : (ax == 0 ? 1 : (ax == 1 ? (int)d.st[1] : (int)d.st[2]));
    return up ? m : -m;
}

// Addressing record of a 3D chunk (host, at setup).  Returns false when a
// point leaves the chunk's run of slots or more than one point has cross
// neighbours off the regular offsets (the caller rejects the level).
inline bool make_chunk_addr3(const Dims &d, const Chunk &ch, ChunkAddr3 &a)
{
    const int L = ch.len, ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int e[3] = {ax == 0 ? sg : 0, ax == 1 ? sg : 0, ax == 2 ? sg : 0};
    const int q0 = cross_axis3(ax, 0), q1 = cross_axis3(ax, 1);
    const int c0[3] = {ch.c0[0], ch.c0[1], ch.c0[2]};
    auto slot_at = [&](int k, int qa, int dq) {
        int c[3] = {c0[0] + k * e[0], c0[1] + k * e[1], c0[2] + k * e[2]};
        if (qa >= 0) c[qa] += dq;
        return slot32(d, c[0], c[1], c[2]);
    };
    const int p0 = slot_at(0, -1, 0);
    // regular cross strides: those of the axes in the chunk's plane
    const int S0 = d.n[0] + 1, S1 = d.n[1] + 1, S2 = d.n[2] + 1;
    const int pl = d.layout == LAYOUT_TWEED3 ? plane3(d, c0[0], c0[1], c0[2]) : 0;
    const int str[3][3] = {{1, S0, S0 * S1}, {S1, 1, S1 * S0}, {S2, S2 * S0, 1}};
    const int s0 = str[pl][q0], s1 = str[pl][q1];
    uint32_t meta = (uint32_t)L | ((uint32_t)ax << 18) | ((uint32_t)(sg > 0) << 20);
    a.p0 = p0;
    a.s[0] = s0;
    a.s[1] = s1;
    a.irr[0] = a.irr[1] = a.irr[2] = a.irr[3] = 0;
    const int step = rec3_step(d, meta);
    int kx = 31;
    uint32_t xmask = 0;
    for (int k = 0; k < L; ++k) {
        const int p = slot_at(k, -1, 0);
        if (p != p0 + k * step) return false;
        const int nb[4] = {slot_at(k, q0, -1), slot_at(k, q0, 1), slot_at(k, q1, -1), slot_at(k, q1, 1)};
        const int rg[4] = {p - s0, p + s0, p - s1, p + s1};
        for (int dd = 0; dd < 4; ++dd) {
            if (nb[dd] == rg[dd]) continue;
            if (kx != 31 && kx != k) return false;
            kx = k;
            xmask |= 1u << dd;
            a.irr[dd] = nb[dd];
        }
    }
    const unsigned lastinb = inblock_dirs(ch, L - 1);
    uint32_t lastbits = 0;
    for (int q = 0; q < 2; ++q) {
        const int qa = cross_axis3(ax, q);
        lastbits |= ((lastinb >> (2 * qa)) & 1u) << (2 * q);
        lastbits |= ((lastinb >> (2 * qa + 1)) & 1u) << (2 * q + 1);
    }
    a.meta = meta | ((uint32_t)kx << 5) | (xmask << 10) | (lastbits << 14);
    return true;
}

// slot of point k of a 3D chunk from its record
__host__ __device__ __forceinline__ int rec3_slot(const Dims &d, const ChunkAddr3 &a, int k)
{
    return a.p0 + k * rec3_step(d, a.meta);
}

// The slots point k of a 3D chunk reads (its own and its four cross
// neighbours) and whether the last point's cross neighbours are in the block.
struct Rec3Slots {
    int p, nb[4];
    unsigned skip; // bit dd: drop the coupling toward cross neighbour dd
};
__host__ __device__ __forceinline__ Rec3Slots rec3_point_slots(const Dims &d, const ChunkAddr3 &a, int k)
{
    const uint32_t mt = a.meta;
    const int L = mt & 31, kx = (mt >> 5) & 31;
    const unsigned xm = k == kx ? (mt >> 10) & 15u : 0u;
    Rec3Slots r;
    r.p = a.p0 + k * rec3_step(d, mt);
    r.nb[0] = (xm & 1u) ? a.irr[0] : r.p - a.s[0];
    r.nb[1] = (xm & 2u) ? a.irr[1] : r.p + a.s[0];
    r.nb[2] = (xm & 4u) ? a.irr[2] : r.p - a.s[1];
    r.nb[3] = (xm & 8u) ? a.irr[3] : r.p + a.s[1];
    r.skip = k == L - 1 ? (mt >> 14) & 15u : 0u;
    return r;
}

// f minus the four cross couplings, from the loaded values (same order as
// point_rhs_across: the lower cross axis first, each toward - then +)
template <typename T>
__host__ __device__ __forceinline__ T rec3_rhs_combine(T fp, const T (&uv)[4], const T (&cc)[4], unsigned skip)
{
    T r = fp;
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        const T t = cc[dd] * uv[dd];
        r -= ((skip >> dd) & 1u) ? T(0) : t;
    }
    return r;
}

template <typename T>
__host__ __device__ __forceinline__ T point_rhs_rec3(const Dims &d, const ChunkAddr3 &a, const T (&cc)[4],
                                                     const T *__restrict__ ub, const T *__restrict__ fb, int k)
{
    const Rec3Slots q = rec3_point_slots(d, a, k);
    const T uv[4] = {ub[q.nb[0]], ub[q.nb[1]], ub[q.nb[2]], ub[q.nb[3]]};
    return rec3_rhs_combine<T>(fb[q.p], uv, cc, q.skip);
}

// the chunk's four cross coefficients (3D), in the records' order
template <typename T>
__host__ __device__ __forceinline__ void chunk_cross_coefs3(const Coef<T> &cf, const Chunk &ch, T (&cc)[4])
{
    const int ax = ch.axdir >> 1;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int a2 = cross_axis3(ax, q);
        const int c = a2 == 0 ? ch.c0[0] : (a2 == 1 ? ch.c0[1] : ch.c0[2]);
        cc[2 * q] = cf.base[(2 * a2) * cf.cs + c];
        cc[2 * q + 1] = cf.base[(2 * a2 + 1) * cf.cs + c];
    }
}

// slot of point k of a chunk
__host__ __device__ __forceinline__ int point_index(const Dims &d, const Chunk &ch, int k)
{
    const int ax = ch.axdir >> 1, sg = (ch.axdir & 1) ? 1 : -1;
    return slot32(d, ch.c0[0] + (ax == 0 ? sg * k : 0), ch.c0[1] + (ax == 1 ? sg * k : 0),
                  ch.c0[2] + (ax == 2 ? sg * k : 0));
}

// Phase 1: right-hand sides, chunk-interior elimination, reduced equations.
// DATA: build the right-hand-side part (reads u, f); MATRIX: build the
// geometry-only reduced matrix (low, ds, dn, up, aux), used at setup to factor
// the reduced systems once.  The kernel runs DATA only.
// rr(k) returns the right-hand side of point k (point_rhs) for k < C - 1; it
// is called once per k, in increasing order, so it may compute the value on
// the spot.  rL is the right-hand side of the last point (index len - 1).
// The along-axis coefficients come in as values: Av[k] toward the predecessor
// point, Cv[k] toward the successor and Bv[k] the along-axis part of the
// diagonal, for k < C (entries from len - 1 on are computed with but never
// used); aL and bLax are those of the last point.
// DIAG_FROM_OFF: the along-axis part of the diagonal is -(a + c) (Bv unused);
// valid for the FP64 forward operator, whose stored diagonal arrays are
// exactly -(lo + hi) (the same rounding).
// The chunk's scalar coefficients used by phase 1: the fixed part of the
// diagonal (the other axes' parts, constant along the chunk), the last
// point's coupling to its successor (cL, 0 without one) and the first point's
// predecessor's coupling back to it (cprev, 0 without a predecessor).
template <typename T> struct ChunkScalars {
    T bfix, cL, cprev;
};
template <typename T, int DIM>
__host__ __device__ __forceinline__ ChunkScalars<T> chunk_scalars(const Coef<T> &cf, const Chunk &ch)
{
    const int L = ch.len;
    const int ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int c0x = ch.c0[0], c0y = ch.c0[1], c0z = (DIM == 3) ? ch.c0[2] : 0;
    const int cax = (ax == 0) ? c0x : ((ax == 1) ? c0y : c0z);
    // every load is made unconditionally (all indices are valid positions)
    // and the unused ones are dropped by selects, so that the loads issue
    // together
    const T g0 = cf.dg[0][c0x], g1 = cf.dg[1][c0y], g2 = (DIM == 3) ? cf.dg[2][c0z] : T(0);
    ChunkScalars<T> r{0, 0, 0};
    r.bfix = T(0) + (ax != 0 ? g0 : g1);
    if (DIM == 3) r.bfix += (ax == 2 ? g1 : g2);
    const int nx = ch.nextdir, na = nx >> 1;
    const int cn = (na == 0 ? c0x : (na == 1 ? c0y : c0z)) + (na == ax ? (L - 1) * sg : 0);
    const T cLv = coef_arr_rt<T, DIM>(cf, nx)[cn];
    const T cpv = coef_arr_rt<T, DIM>(cf, ad)[cax - sg];
    r.cL = (ch.flags & CF_NEXT) ? cLv : T(0);
    r.cprev = ((ch.flags & CF_PREV) && L >= 2) ? cpv : T(0);
    return r;
}

template <typename T, int DIM, bool MATRIX, bool DATA, bool DIAG_FROM_OFF, int C, typename RR>
__host__ __device__ __forceinline__ void sweep_phase1_coefs(const Dims &d, const Coef<T> &cf, RR &&rr, T rL,
                                                            const Chunk &ch, int t, const RedArrays<T> &s,
                                                            LaneState<T, C> &st, const T *Av, const T *Cv,
                                                            const T *Bv, T aL, T bLax, const ChunkScalars<T> &sc)
{
    const int L = ch.len;
    const int ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const uint8_t fl = ch.flags;
    const bool hp = fl & CF_PREV, hn = fl & CF_NEXT, nd = fl & CF_NEXT_DIRECT;
    const int c0x = ch.c0[0], c0y = ch.c0[1], c0z = (DIM == 3) ? ch.c0[2] : 0;
    const int ex = (ax == 0) ? sg : 0, ey = (ax == 1) ? sg : 0, ez = (ax == 2) ? sg : 0;
    st.L = L;
    st.prev = ch.prev;
    st.hp = hp;

    // the diagonal b = along-axis part + fixed part (the other axes' parts)
    const T bfix = sc.bfix;
    // the last point's row (the node): a, b, its right-hand side, and its
    // coupling to the successor
    const T bL = (ax == 0) ? bLax + bfix : bfix + bLax;
    const T cL = sc.cL;
    if (MATRIX && hn && nd) {
        // the successor's row coefficient back toward this point
        const int li = c0x + (L - 1) * ex, lj = c0y + (L - 1) * ey, ll = c0z + (L - 1) * ez;
        const int nx = ch.nextdir, na = nx >> 1, ns = (nx & 1) ? 1 : -1;
        const int cn = (na == 0) ? li : ((na == 1) ? lj : ll);
        s.aux[t] = coef_arr_rt<T, DIM>(cf, nx ^ 1)[cn + ns];
    }
    // elimination of the interior (points 0..L-2) with zero end values; run
    // branch-free over all C positions, entries from L-1 on are not used
    T Gp = 0, Dp = 0, Sp = hp ? T(1) : T(0);
#pragma unroll
    for (int k = 0; k < C - 1; ++k) {
        const T r = DATA ? rr(k) : T(0);
        const T bk = DIAG_FROM_OFF ? -(Av[k] + Cv[k]) : Bv[k];
        const T b = (ax == 0) ? bk + bfix : bfix + bk;
        const T a = Av[k];
        const T inv = rcp<T>(b - a * Gp);
        st.G[k] = Cv[k] * inv;
        st.D[k] = (r - a * Dp) * inv;
        st.S[k] = -a * Sp * inv;
        Gp = st.G[k];
        Dp = st.D[k];
        Sp = st.S[k];
    }
    // first-point values of the zero-end interior solution y and its spikes v, w
    T yl = 0, vl = 0, wl = 0, y = 0, v = 0, ww = 0;
#pragma unroll
    for (int k = C - 2; k >= 0; --k) {
        const bool last = (k == L - 2), in = (k < L - 2);
        y = last ? st.D[k] : (in ? st.D[k] - st.G[k] * y : y);
        yl = last ? y : yl;
        if (MATRIX) {
            v = last ? st.S[k] : (in ? st.S[k] - st.G[k] * v : v);
            ww = last ? -st.G[k] : (in ? -st.G[k] * ww : ww);
            vl = last ? v : vl;
            wl = last ? ww : wl;
        }
    }
    // own row: a_L x_{L-2} + b_L X + c_L x_next = r_L with x_{L-2} = y + v X_prev + w X
    if (DATA) s.rs[t] = (L >= 2) ? rL - aL * yl : rL;
    if (MATRIX) {
        s.ds[t] = (L >= 2) ? bL + aL * wl : bL;
        s.low[t] = hp ? ((L >= 2) ? aL * vl : aL) : T(0);
    }
    // the successor's first interior point couples the successor node's row to
    // this interior; without one, the coupling is direct (or absent)
    if (!hn || nd) {
        if (DATA) s.rn[t] = 0;
        if (MATRIX) {
            s.dn[t] = 0;
            s.up[t] = hn ? cL : T(0);
        }
    }
    if (hp && L >= 2) {
        const T cprev = sc.cprev;
        if (DATA) s.rn[ch.prev] = -cprev * y;
        if (MATRIX) {
            s.dn[ch.prev] = cprev * v;
            s.up[ch.prev] = cprev * ww;
        }
    }
}

// Phase 1 loading the chunk's along-axis coefficients itself (one lane per
// chunk), all before the elimination chain so that their latency is paid once.
template <typename T, int DIM, bool MATRIX, bool DATA, bool DIAG_FROM_OFF = false, int C = CH, typename RR>
__host__ __device__ __forceinline__ void sweep_phase1(const Dims &d, const Coef<T> &cf, RR &&rr, T rL,
                                                      const Chunk &ch, int t, const RedArrays<T> &s,
                                                      LaneState<T, C> &st)
{
    const int L = ch.len;
    const int ad = ch.axdir, ax = ad >> 1;
    const int sg = (ad & 1) ? 1 : -1;
    const int cax = (ax == 0) ? ch.c0[0] : ((ax == 1) ? ch.c0[1] : ch.c0[2]);
    const T *Pback = coef_arr_rt<T, DIM>(cf, ad ^ 1);
    const T *Pfwd = coef_arr_rt<T, DIM>(cf, ad);
    const T *Pdg = dg_arr_rt<T>(cf, ax);
    T Av[C], Cv[C], Bv[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const int ca = (k < L) ? cax + k * sg : cax; // clamped: stays inside the arrays
        Av[k] = Pback[ca];
        Cv[k] = Pfwd[ca];
        Bv[k] = DIAG_FROM_OFF ? T(0) : Pdg[ca];
    }
    const int cL_ = cax + (L - 1) * sg;
    sweep_phase1_coefs<T, DIM, MATRIX, DATA, DIAG_FROM_OFF, C>(d, cf, rr, rL, ch, t, s, st, Av, Cv, Bv, Pback[cL_],
                                                             Pdg[cL_], chunk_scalars<T, DIM>(cf, ch));
}

// Phase 2 on the host: the reduced systems of one workgroup solved node by
// node with the setup-time factors, in the order the device scans use.
// rhs[q] = rs[q] + rn[q]; on return x[q] holds every node value.
template <typename T>
__host__ void reduced_solve_seq(int n, const Chunk *ch, const NodeFac<T> *fac, const T *rhs, T *dl, T *x)
{
    // forward elimination along segments
    T carry = 0;
    for (int q = 0; q < n; ++q) {
        const bool head = ch[q].nflags & NF_HEAD;
        dl[q] = (head ? T(0) : fac[q].alpha * carry) + rhs[q] * fac[q].inv;
        carry = dl[q];
    }
    // branch points
    for (int q = 0; q < n; ++q)
        if (ch[q].nflags & NF_J) {
            // branch row: legs 1..m-1 end next to the branch point (coupling z
            // of their last node); leg 0's last node precedes it (coupling gam)
            const int p0 = (ch[q].flags & CF_PREV) ? ch[q].prev : -1;
            T num = rhs[q];
            for (int p = 0; p < n; ++p)
                if ((ch[p].nflags & NF_EXTJ) && ch[p].ext == q && p != p0) num -= fac[p].z * dl[p];
            if (p0 >= 0) num -= fac[q].gam * dl[p0];
            x[q] = num * fac[q].inv;
        }
    // back substitution along segments
    T next = 0;
    for (int q = n - 1; q >= 0; --q) {
        const uint8_t f = ch[q].nflags;
        if (f & (NF_J | NF_B)) continue;
        if (f & NF_TAIL) next = (f & NF_EXTJ) ? x[ch[q].ext] : T(0);
        x[q] = dl[q] - fac[q].gam * next;
        next = x[q];
    }
    // ring borders, then the ring corrections
    for (int q = 0; q < n; ++q)
        if (ch[q].nflags & NF_B) {
            int s = q;
            while (s > 0 && (ch[s - 1].nflags & NF_RING) && ch[s - 1].ext == q) --s;
            x[q] = (rhs[q] - fac[q].alpha * x[q - 1] - fac[q].gam * x[s]) * fac[q].inv;
        }
    for (int q = 0; q < n; ++q)
        if (ch[q].nflags & NF_RING) x[q] -= x[ch[q].ext] * fac[q].z;
}

// Phase 3 with a store callback: put(k, x_k) for k = 0 .. len-1 (used where u
// is written in place, as in the coarse-level kernel).
template <typename T, int C = CH, typename F>
__host__ __device__ __forceinline__ void sweep_phase3_each(int t, const RedArrays<T> &s, const LaneState<T, C> &st,
                                                           F &&put)
{
    const T Xp = st.hp ? s.x[st.prev] : T(0);
    const T Xo = s.x[t];
    T x = Xo;
#pragma unroll
    for (int k = C - 2; k >= 0; --k) {
        const T xn = st.D[k] + st.S[k] * Xp - st.G[k] * x;
        x = (k <= st.L - 2) ? xn : x;
        if (k <= st.L - 2) put(k, x);
    }
    put(st.L - 1, Xo);
}

// Phase 3: back-substitution of the chunk interior from the node values;
// xx[k] receives the new value of point k (the caller scatters it to u).
template <typename T, int C = CH>
__host__ __device__ __forceinline__ void sweep_phase3(T *__restrict__ xx, int t, const RedArrays<T> &s,
                                                      const LaneState<T, C> &st)
{
    const T Xp = st.hp ? s.x[st.prev] : T(0);
    const T Xo = s.x[t];
    T x = Xo;
    // branch-free: positions past the interior keep x = Xo; entries k >= L of
    // xx are scratch and never scattered
#pragma unroll
    for (int k = C - 2; k >= 0; --k) {
        const T xn = st.D[k] + st.S[k] * Xp - st.G[k] * x;
        x = (k <= st.L - 2) ? xn : x;
        xx[k] = x;
    }
    xx[st.L - 1] = Xo;
}

} // namespace twmg
