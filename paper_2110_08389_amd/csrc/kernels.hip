// Device kernels of the tweed / wireframe multigrid (gfx950).
//
// Everything here is memory-bound stencil or line-solve work (about half a
// flop per byte), so no MFMA: the design goals are single-pass HBM traffic,
// coalesced rows and enough independent waves per CU.
#include "sweep_core.h"

#include <mutex>

namespace twmg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// A node of the 3D split layout: its slot, the strides of x, y and z in its
// plane, and how far it lies inside that plane's region (its own primed
// coordinate below the smaller of the other two).  With margin >= 2 its six
// axis neighbours share its plane; with margin >= 3 so does every node of its
// 3 x 3 x 3 box (a diagonal step can tie the primed coordinates, and a tie
// goes to the lower axis).
struct P3 {
    long long p;
    long long sx, sy, sz;
    int margin;
};
__device__ __forceinline__ P3 p3_at(const Dims &d, int i, int j, int l)
{
    const int ip = i < d.n[0] - i ? i : d.n[0] - i, jp = j < d.n[1] - j ? j : d.n[1] - j,
              lp = l < d.n[2] - l ? l : d.n[2] - l;
    const int pl = (ip <= jp && ip <= lp) ? 0 : (jp <= lp ? 1 : 2);
    const int own = pl == 0 ? ip : (pl == 1 ? jp : lp);
    const int o1 = pl == 0 ? jp : ip, o2 = pl == 2 ? jp : lp;
    const long long S0 = d.n[0] + 1, S1 = d.n[1] + 1, S2 = d.n[2] + 1;
    P3 q;
    q.p = plane3_slot(d, pl, i, j, l);
    q.sx = pl == 0 ? 1 : (pl == 1 ? S1 : S2);
    q.sy = pl == 0 ? S0 : (pl == 1 ? 1 : S2 * S0);
    q.sz = pl == 0 ? S0 * S1 : (pl == 1 ? S1 * S0 : 1);
    q.margin = (o1 < o2 ? o1 : o2) - own;
    return q;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double block_max(double v)
{
    __shared__ double s[16];
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) s[wv] = v;
    __syncthreads();
    if (wv == 0) {
        v = (lane < (int)(blockDim.x >> 6)) ? s[lane] : 0.0;
        v = wave_max(v);
    }
    return v;
}

__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || b != b) ? __builtin_nan("") : fmax(a, b); }

// slots of interior node (i, j, l) and of its neighbours x-, x+, y-, y+, z-, z+
template <int DIM> struct Stencil {
    long long p, nb[2 * DIM];
};
template <int DIM> __device__ __forceinline__ Stencil<DIM> stencil_at(const Dims &d, int i, int j, int l)
{
    Stencil<DIM> s;
    if (DIM == 2 && d.layout != LAYOUT_ROW) {
        s.p = nidx(d, i, j, 0);
        s.nb[0] = nidx(d, i - 1, j, 0);
        s.nb[1] = nidx(d, i + 1, j, 0);
        s.nb[2] = nidx(d, i, j - 1, 0);
        s.nb[3] = nidx(d, i, j + 1, 0);
    } else if (DIM == 3 && d.layout != LAYOUT_ROW) {
        // the slots of the 3D split layout: fixed offsets in the node's plane
        // unless it lies within 2 of the plane's border
        const P3 q = p3_at(d, i, j, l);
        s.p = q.p;
        if (q.margin >= 2) {
            s.nb[0] = q.p - q.sx;
            s.nb[1] = q.p + q.sx;
            s.nb[2] = q.p - q.sy;
            s.nb[3] = q.p + q.sy;
            s.nb[2 * DIM - 2] = q.p - q.sz;
            s.nb[2 * DIM - 1] = q.p + q.sz;
        } else {
            s.nb[0] = nidx(d, i - 1, j, l);
            s.nb[1] = nidx(d, i + 1, j, l);
            s.nb[2] = nidx(d, i, j - 1, l);
            s.nb[3] = nidx(d, i, j + 1, l);
            s.nb[2 * DIM - 2] = nidx(d, i, j, l - 1);
            s.nb[2 * DIM - 1] = nidx(d, i, j, l + 1);
        }
    } else {
        s.p = i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0);
#pragma unroll
        for (int dd = 0; dd < 2 * DIM; ++dd) s.nb[dd] = s.p + dir_off(d, dd);
    }
    return s;
}

// defect f - L u at interior node (i, j, l)
template <typename T, int DIM>
__device__ __forceinline__ T defect_at(const Dims &d, const Coef<T> &cf, const T *__restrict__ u,
                                       const T *__restrict__ f, int i, int j, int l)
{
    const Stencil<DIM> q = stencil_at<DIM>(d, i, j, l);
    T s = cf.lo[0][i] * u[q.nb[0]] + cf.hi[0][i] * u[q.nb[1]];
    s += cf.lo[1][j] * u[q.nb[2]] + cf.hi[1][j] * u[q.nb[3]];
    T dg = cf.dg[0][i] + cf.dg[1][j];
    if (DIM == 3) {
        s += cf.lo[2][l] * u[q.nb[4]] + cf.hi[2][l] * u[q.nb[5]];
        dg += cf.dg[2][l];
    }
    return f[q.p] - (s + dg * u[q.p]);
}

template <int DIM> __device__ __forceinline__ bool interior(const Dims &d, int i, int j, int l)
{
    bool in = i > 0 && i < d.n[0] && j > 0 && j < d.n[1];
    if (DIM == 3) in = in && l > 0 && l < d.n[2];
    return in;
}

// rows of a row-major node array: (j, l) pairs; row r -> j = r % (ny+1), l = r / (ny+1)
__device__ __forceinline__ int nrows(const Dims &d, int DIM)
{
    return (d.n[1] + 1) * (DIM == 3 ? d.n[2] + 1 : 1);
}

// Storage-order traversal of a node array, so that consecutive threads touch
// consecutive slots: LAYOUT_ROW has the rows (j, l) of nx+1 nodes; a 2D split
// layout has the ny+1 rows of plane R, then the nx+1 columns (ny+1 nodes) of
// plane C; the 3D split layout has the (j, l) rows of plane 0, the (i, l)
// rows of plane 1 and the (i, j) rows of plane 2.
__device__ __forceinline__ int lrows(const Dims &d, int DIM)
{
    if (d.layout == LAYOUT_TWEED3)
        return (d.n[1] + 1) * (d.n[2] + 1) + (d.n[0] + 1) * (d.n[2] + 1) + (d.n[0] + 1) * (d.n[1] + 1);
    return d.layout == LAYOUT_ROW ? nrows(d, DIM) : (d.n[1] + 1) + (d.n[0] + 1);
}
__device__ __forceinline__ int lrow_len(const Dims &d, int row)
{
    if (d.layout == LAYOUT_TWEED3) {
        const int r0 = (d.n[1] + 1) * (d.n[2] + 1), r1 = (d.n[0] + 1) * (d.n[2] + 1);
        return row < r0 ? d.n[0] + 1 : (row < r0 + r1 ? d.n[1] + 1 : d.n[2] + 1);
    }
    return (d.layout != LAYOUT_ROW && row > d.n[1]) ? d.n[1] + 1 : d.n[0] + 1;
}
// node q of row `row`: its coordinates and slot; false when the node is kept
// in another plane (each node is visited exactly once over all rows)
template <int DIM>
__device__ __forceinline__ bool lnode(const Dims &d, int row, int q, int &i, int &j, int &l, long long &p)
{
    if (DIM == 3 && d.layout == LAYOUT_TWEED3) {
        const int r0 = (d.n[1] + 1) * (d.n[2] + 1), r1 = (d.n[0] + 1) * (d.n[2] + 1);
        int pl;
        if (row < r0) {
            pl = 0;
            i = q;
            j = row % (d.n[1] + 1);
            l = row / (d.n[1] + 1);
        } else if (row < r0 + r1) {
            pl = 1;
            const int rr = row - r0;
            j = q;
            i = rr % (d.n[0] + 1);
            l = rr / (d.n[0] + 1);
        } else {
            pl = 2;
            const int rr = row - r0 - r1;
            l = q;
            i = rr % (d.n[0] + 1);
            j = rr / (d.n[0] + 1);
        }
        p = plane3_slot(d, pl, i, j, l);
        return plane3(d, i, j, l) == pl;
    }
    if (d.layout == LAYOUT_ROW) {
        j = row % (d.n[1] + 1);
        l = DIM == 3 ? row / (d.n[1] + 1) : 0;
        i = q;
        p = i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0);
        return true;
    }
    l = 0;
    if (row <= d.n[1]) {
        j = row;
        i = q;
        p = i + j * d.st[1];
        return !col_plane(d, i, j);
    }
    i = row - (d.n[1] + 1);
    j = q;
    p = d.nn + j + (long long)i * (d.n[1] + 1);
    return col_plane(d, i, j);
}

static int lrow_grid(const Dims &d)
{
    long long r;
    if (d.layout == LAYOUT_TWEED3)
        r = (long long)(d.n[1] + 1) * (d.n[2] + 1) + (long long)(d.n[0] + 1) * (d.n[2] + 1) +
            (long long)(d.n[0] + 1) * (d.n[1] + 1);
    else
        r = d.layout == LAYOUT_ROW ? (long long)(d.n[1] + 1) * (d.dim == 3 ? d.n[2] + 1 : 1) : d.n[0] + d.n[1] + 2;
    return r < 65535 ? (int)r : 65535;
}

// ---------------------------------------------------------------------------
// Block relaxation half-sweep: one workgroup per group of whole blocks of one
// colour.  Phase 1 and phase 3 (chunk elimination and back substitution) are
// per-lane steps in sweep_core.h.  The reduced systems of all blocks of the
// workgroup are solved together with two workgroup-wide affine scans:
//   forward   delta_q = alpha_q delta_{q-1} + rhs_q inv_q   (alpha = 0 at segment heads)
//   backward  x_q     = delta_q - gam_q x_{q+1}             (x_{q+1} -> branch value at tails)
// with the setup-time factors, so the depth is logarithmic in the block size.
// ---------------------------------------------------------------------------

// ---- wave-level building blocks of the scans -------------------------------
// DPP row shifts move values between the 16 lanes of a row at VALU latency;
// a lane whose source lies outside its row keeps 'old' (the identity map).
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v, double old)
{
    const long long vi = __builtin_bit_cast(long long, v), oi = __builtin_bit_cast(long long, old);
    const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)vi, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(vi >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL> __device__ __forceinline__ float dpp_mov(float v, float old)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_value(double v, int lane)
{
    const long long vi = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)vi, lane), hi = __builtin_amdgcn_readlane((int)(vi >> 32), lane);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Inclusive scan of affine maps x -> A x + B in lane order: lane t ends with
// the composition of the maps of lanes 0..t (later maps applied last).  Rows
// of 16 lanes by DPP shifts, the 4 rows of a wave through their totals (lane
// reads), the waves of the workgroup through per-wave totals sa/sb in LDS.
// ONEWAVE: only wavefront 0 takes part (all other lanes of the workgroup are
// elsewhere), so the wavefront's own scan is the whole scan
template <typename T, bool ONEWAVE = false> __device__ __forceinline__ void scan_fwd(T &A, T &B, T *sa, T *sb)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, row = lane >> 4;
    {
        T Ap = dpp_mov<0x111>(A, T(1)), Bp = dpp_mov<0x111>(B, T(0)); // row_shr:1
        B = A * Bp + B;
        A = A * Ap;
        Ap = dpp_mov<0x112>(A, T(1));
        Bp = dpp_mov<0x112>(B, T(0));
        B = A * Bp + B;
        A = A * Ap;
        Ap = dpp_mov<0x114>(A, T(1));
        Bp = dpp_mov<0x114>(B, T(0));
        B = A * Bp + B;
        A = A * Ap;
        Ap = dpp_mov<0x118>(A, T(1));
        Bp = dpp_mov<0x118>(B, T(0));
        B = A * Bp + B;
        A = A * Ap;
    }
    {
        // prefixes of the rows before this lane's row
        const T A0 = lane_value(A, 15), B0 = lane_value(B, 15);
        const T A1 = lane_value(A, 31), B1 = lane_value(B, 31);
        const T A2 = lane_value(A, 47), B2 = lane_value(B, 47);
        const T P2A = A1 * A0, P2B = A1 * B0 + B1;
        const T P3A = A2 * P2A, P3B = A2 * P2B + B2;
        const T pA = row == 0 ? T(1) : (row == 1 ? A0 : (row == 2 ? P2A : P3A));
        const T pB = row == 0 ? T(0) : (row == 1 ? B0 : (row == 2 ? P2B : P3B));
        B = A * pB + B;
        A = A * pA;
    }
    if constexpr (ONEWAVE) return;
    if (lane == 63) {
        sa[wv] = A;
        sb[wv] = B;
    }
    __syncthreads();
    T pA = 1, pB = 0;
    for (int k = 0; k < wv; ++k) {
        pB = sa[k] * pB + sb[k];
        pA = sa[k] * pA;
    }
    B = A * pB + B;
    A = A * pA;
    __syncthreads();
}

// the same over lanes in decreasing order (composition of the maps of lanes t..NT-1)
template <typename T, bool ONEWAVE = false> __device__ __forceinline__ void scan_bwd(T &A, T &B, T *sa, T *sb)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6, row = lane >> 4;
    {
        T An = dpp_mov<0x101>(A, T(1)), Bn = dpp_mov<0x101>(B, T(0)); // row_shl:1
        B = A * Bn + B;
        A = A * An;
        An = dpp_mov<0x102>(A, T(1));
        Bn = dpp_mov<0x102>(B, T(0));
        B = A * Bn + B;
        A = A * An;
        An = dpp_mov<0x104>(A, T(1));
        Bn = dpp_mov<0x104>(B, T(0));
        B = A * Bn + B;
        A = A * An;
        An = dpp_mov<0x108>(A, T(1));
        Bn = dpp_mov<0x108>(B, T(0));
        B = A * Bn + B;
        A = A * An;
    }
    {
        // suffixes of the rows after this lane's row (row totals at lanes 16 r)
        const T A1 = lane_value(A, 16), B1 = lane_value(B, 16);
        const T A2 = lane_value(A, 32), B2 = lane_value(B, 32);
        const T A3 = lane_value(A, 48), B3 = lane_value(B, 48);
        const T S2A = A2 * A3, S2B = A2 * B3 + B2;
        const T S1A = A1 * S2A, S1B = A1 * S2B + B1;
        const T pA = row == 3 ? T(1) : (row == 2 ? A3 : (row == 1 ? S2A : S1A));
        const T pB = row == 3 ? T(0) : (row == 2 ? B3 : (row == 1 ? S2B : S1B));
        B = A * pB + B;
        A = A * pA;
    }
    if constexpr (ONEWAVE) return;
    if (lane == 0) {
        sa[wv] = A;
        sb[wv] = B;
    }
    __syncthreads();
    T pA = 1, pB = 0;
    for (int k = nw - 1; k > wv; --k) {
        pB = sa[k] * pB + sb[k];
        pA = sa[k] * pA;
    }
    B = A * pB + B;
    A = A * pA;
    __syncthreads();
}

// Workgroup barrier, or with ONEWAVE (only wavefront 0 runs this code) the
// ordering of one wavefront's LDS accesses: a wavefront's LDS instructions
// execute in issue order, so only the compiler has to be kept from moving
// them across this point.
template <bool ONEWAVE> __device__ __forceinline__ void wg_sync()
{
    if constexpr (ONEWAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Block-relaxation half-sweep: one lane per chunk.  The workgroup's points are
// gathered point-major (consecutive lanes read consecutive points of a chunk,
// so rows are read in whole cache lines) into an LDS staging buffer; each lane
// then eliminates its chunk's interior (Thomas with zero end values and a left
// spike), the chunk end points form the blocks' reduced systems, solved by
// workgroup-wide affine scans with setup-time factors, and each lane
// back-substitutes its chunk in LDS before the point-major scatter.
// Phase 2: the reduced systems of the workgroup's blocks (lane = node), from
// the node rows s_rs + s_rn left by phase 1; the node values land in s_x.
// bk is the block of index t (lanes t < w.nblock), loaded by the caller.  With
// s_nf (4 NT entries of LDS that are free during this phase), each node
// publishes its factors there and the branch-point and ring-border lanes read
// them from LDS; without it they read fac.
template <typename T, bool ONEWAVE = false>
__device__ __forceinline__ void reduced_solve_wg(const WGDesc &w, bool act, uint8_t nfl, int ext, const NodeFac<T> &nf,
                                                 const Block &bk, const NodeFac<T> *__restrict__ fac, int rings,
                                                 T *s_rs, T *s_rn, T *s_dl, T *s_x, T *s_a, T *s_b, T *s_nf)
{
    const int t = threadIdx.x, nt = blockDim.x;
    auto node_fac = [&](int q) -> NodeFac<T> {
        if (!s_nf) return fac[w.chunk0 + q];
        NodeFac<T> r;
        r.alpha = s_nf[q];
        r.inv = s_nf[nt + q];
        r.gam = s_nf[2 * nt + q];
        r.z = s_nf[3 * nt + q];
        return r;
    };
    if (s_nf && act) {
        s_nf[t] = nf.alpha;
        s_nf[nt + t] = nf.inv;
        s_nf[2 * nt + t] = nf.gam;
        s_nf[3 * nt + t] = nf.z;
    }
    // forward elimination along segments
    T rhs = 0, A = 0, B = 0;
    if (act) {
        rhs = s_rs[t] + s_rn[t];
        A = (nfl & NF_HEAD) ? T(0) : nf.alpha;
        B = rhs * nf.inv;
    }
    scan_fwd<T, ONEWAVE>(A, B, s_a, s_b);
    const T dl = B;
    s_dl[t] = dl;
    wg_sync<ONEWAVE>();
    // branch points of the spiders
    if (t < w.nblock && bk.type == BT_SPIDER) {
        const int first = bk.first, J = first + bk.count - 1, m = bk.m;
        const NodeFac<T> fj = node_fac(J);
        T num = s_rs[J] + s_rn[J];
#pragma unroll
        for (int l = 1; l < 7; ++l)
            if (l < m) {
                const int e = bk.ends[l];
                num -= node_fac(e).z * s_dl[e];
            }
        if (J > first) num -= fj.gam * s_dl[J - 1];
        s_x[J] = num * fj.inv;
    }
    wg_sync<ONEWAVE>();
    // back substitution along segments
    A = 0;
    B = 0;
    if (act) {
        if (nfl & NF_TAIL) {
            const T next = (nfl & NF_EXTJ) ? s_x[ext] : T(0);
            B = dl - nf.gam * next;
        } else {
            A = -nf.gam;
            B = dl;
        }
    }
    scan_bwd<T, ONEWAVE>(A, B, s_a, s_b);
    T x = B;
    if (act && !(nfl & (NF_J | NF_B))) s_x[t] = x;
    if (rings) {
        wg_sync<ONEWAVE>();
        if (t < w.nblock && bk.type == BT_RING) {
            const int s0 = bk.first, Bn = bk.first + bk.count - 1;
            const NodeFac<T> fb_ = node_fac(Bn);
            s_x[Bn] = (s_rs[Bn] + s_rn[Bn] - fb_.alpha * s_x[Bn - 1] - fb_.gam * s_x[s0]) * fb_.inv;
        }
        wg_sync<ONEWAVE>();
        if (act && (nfl & NF_RING)) x -= s_x[ext] * nf.z;
        wg_sync<ONEWAVE>();
        if (act && (nfl & NF_RING)) s_x[t] = x;
    }
}

// Orders LDS accesses of the lanes of one wavefront: a wavefront's LDS
// instructions execute in issue order, so only the compiler has to be kept
// from moving them across this point.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The along-axis coefficients of a chunk's C positions from one coefficient
// array P (out[k] at position cax + k for up, cax - k otherwise; entries from
// the chunk's length on are values of neighbouring positions and go unused).
// The C-position window is read as C/2 + 1 aligned pairs: the arrays start
// at even offsets from a 16-byte aligned block with CH + 2 >= C + 2 spare entries
// before and after it, so every window stays inside the allocation.
template <typename T, int C>
__device__ __forceinline__ void chunk_coef_window(const T *__restrict__ P, int cax, int up, T (&out)[C])
{
    typedef T V2 __attribute__((ext_vector_type(2)));
    const int lo = up ? cax : cax - (C - 1);
    const int e0 = lo & ~1, off = lo - e0;
    const V2 *p2 = reinterpret_cast<const V2 *>(P + e0);
    T W[C + 2];
#pragma unroll
    for (int q = 0; q < C / 2 + 1; ++q) {
        const V2 v = p2[q];
        W[2 * q] = v.x;
        W[2 * q + 1] = v.y;
    }
    // selections by bit masks: written as selects between neighbouring
    // entries, they are turned into an indexed read of W through scratch
    // memory
    typedef typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned>::type U;
    const U mo = off ? ~U(0) : U(0), mu = up ? ~U(0) : U(0);
    auto bits = [](T v) { return __builtin_bit_cast(U, v); };
#pragma unroll
    for (int k = 0; k < C; ++k) {
        const U a = (bits(W[k]) & ~mo) | (bits(W[k + 1]) & mo);
        const U b = (bits(W[C - 1 - k]) & ~mo) | (bits(W[C - k]) & mo);
        out[k] = __builtin_bit_cast(T, (b & ~mu) | (a & mu));
    }
}

// addressing record type of a chunk, by dimension
template <int DIM> struct RecOf {
    using type = ChunkAddr;
};
template <> struct RecOf<3> {
    using type = ChunkAddr3;
};

// The work of one workgroup descriptor w; all NT lanes of the workgroup must
// call it.  REC (workgroups of at most NT/2 lanes, 2D and 3D): the points are
// addressed through the chunks' precomputed records (addrs), and each
// wavefront gathers the points of its own 64 chunks; otherwise (the NT-lane
// workgroups of the largest blocks) in general form, each point's slots
// computed from its coordinates.
// C: the chunk capacity (CH, or fewer for the small levels' short chunks;
// records path only).

template <typename T, int DIM, int NT, bool DOFF, bool REC, int C = CH>
__device__ __forceinline__ void sweep_wg(const Dims &d, const Coef<T> &cf, T *__restrict__ ub,
                                         const T *__restrict__ fb, const Chunk *__restrict__ chunks,
                                         const typename RecOf<DIM>::type *__restrict__ addrs,
                                         const T *__restrict__ cross,
                                         const Block *__restrict__ blocks, const WGDesc w,
                                         const NodeFac<T> *__restrict__ fac, int rings)
{
    static_assert(REC || C == CH, "short chunks only on the records path");
    static_assert(64 % C == 0 && C <= CH, "chunk capacity");
    constexpr int PS = C + 1; // padded row of the point staging buffer (bank-conflict free)
    constexpr int CPS = 64 / C; // a wavefront's chunks per gather step
    __shared__ T s_pt[NT * PS + 1];
    // chunk descriptors (general) or addressing records and along-axis start
    // coordinates (REC)
    __shared__ Chunk s_ch[REC ? 1 : NT];
    __shared__ typename RecOf<DIM>::type s_ca[REC ? NT : 1];
    __shared__ T s_rs[NT], s_rn[NT], s_dl[NT], s_x[NT];
    __shared__ T s_a[NT / 64], s_b[NT / 64];
    const RedArrays<T> red{nullptr, nullptr, s_rs, nullptr, nullptr, s_rn, s_x, nullptr};
    const int t = threadIdx.x;
    const bool act = t < w.nchunk;
    Chunk chl; // this lane's chunk
    if (act) {
        chl = chunks[w.chunk0 + t];
        if (REC) {
            // the record, and the chunk's cross coefficients (constant along
            // it) in s_rs / s_rn (3D: also s_dl / s_x) until phase 1 and the
            // reduced solve reuse them
            s_ca[t] = addrs[w.chunk0 + t];
            constexpr int NCC = DIM == 2 ? 2 : 4;
            s_rs[t] = cross[NCC * (w.chunk0 + t)];
            s_rn[t] = cross[NCC * (w.chunk0 + t) + 1];
            if (DIM == 3) {
                s_dl[t] = cross[NCC * (w.chunk0 + t) + 2];
                s_x[t] = cross[NCC * (w.chunk0 + t) + 3];
            }
        } else {
            s_ch[t] = chl;
        }
    }
    // REC: each wavefront gathers only its own chunks, whose records and
    // cross coefficients its own lanes wrote (positions past the workgroup's
    // end use the wavefront's first chunk; a wavefront without chunks skips
    // the gather)
    if (REC)
        wave_sync();
    else
        __syncthreads();
    LaneState<T, C> st;
    uint8_t nfl = 0;
    int ext = -1;
    // the lane's node factors and (lanes t < nblock) block t, for phase 2;
    // loaded before phase 1 so that its arithmetic covers their latency
    NodeFac<T> nf{0, 0, 0, 0};
    Block bkl;
    bkl.type = BT_CHAIN;
    if constexpr (REC) {
        // wavefront-local gather of the right-hand sides (f minus the
        // off-block cross couplings): in step m, lane l takes point l % C of
        // the wavefront's chunk (64 / C) m + l / C (64 consecutive points per
        // load)
        // and stores it in the chunk's row of s_pt.  Positions past a chunk's
        // end repeat its first point; chunks past the workgroup's end read the
        // wavefront's first chunk and land in the spare entry.  Two batches,
        // each issuing all its loads before storing.
        const int lane = t & 63, c0w = t & ~63;
        constexpr int GB = C < 8 ? C : 8;
        if constexpr (DIM == 2) {
            if (c0w < w.nchunk) {
#pragma unroll
                for (int m0 = 0; m0 < C; m0 += GB) {
                    // all of a batch's loads are issued before any is used
                    T fv[GB], um[GB], upv[GB], cm[GB], cp[GB];
                    bool skm[GB], skp[GB];
                    int dst[GB];
#pragma unroll
                    for (int m = 0; m < GB; ++m) {
                        const int c = c0w + CPS * (m0 + m) + lane / C, k = lane % C;
                        const bool inc = c < w.nchunk;
                        const int cc = inc ? c : c0w;
                        const ChunkAddr a = s_ca[cc];
                        const bool valid = inc && k < (int)(a.meta & 31);
                        const RecSlots q = rec_point_slots(d, a, valid ? k : 0);
                        fv[m] = fb[q.p];
                        um[m] = ub[q.pm];
                        upv[m] = ub[q.pp];
                        skm[m] = q.skm;
                        skp[m] = q.skp;
                        cm[m] = s_rs[cc];
                        cp[m] = s_rn[cc];
                        dst[m] = inc ? c * PS + k : NT * PS;
                    }
                    // keep the scheduler from starting the arithmetic (and its
                    // waits) before the batch's last load has issued
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int m = 0; m < GB; ++m)
                        s_pt[dst[m]] = rec_rhs_combine<T>(fv[m], um[m], upv[m], cm[m], cp[m], skm[m], skp[m]);
                }
            }
        } else {
            // 3D: f and four cross neighbours per point; the chunk's four
            // cross coefficients are read from LDS after the batch's loads
            if (c0w < w.nchunk) {
#pragma unroll
                for (int m0 = 0; m0 < C; m0 += GB) {
                    T fv[GB], uv[GB][4];
                    unsigned skip[GB];
                    int dst[GB], ccx[GB];
#pragma unroll
                    for (int m = 0; m < GB; ++m) {
                        const int c = c0w + CPS * (m0 + m) + lane / C, k = lane % C;
                        const bool inc = c < w.nchunk;
                        const int cc = inc ? c : c0w;
                        const ChunkAddr3 a = s_ca[cc];
                        const bool valid = inc && k < (int)(a.meta & 31);
                        const Rec3Slots q = rec3_point_slots(d, a, valid ? k : 0);
                        fv[m] = fb[q.p];
#pragma unroll
                        for (int dd = 0; dd < 4; ++dd) uv[m][dd] = ub[q.nb[dd]];
                        skip[m] = q.skip;
                        ccx[m] = cc;
                        dst[m] = inc ? c * PS + k : NT * PS;
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int m = 0; m < GB; ++m) {
                        const T cc4[4] = {s_rs[ccx[m]], s_rn[ccx[m]], s_dl[ccx[m]], s_x[ccx[m]]};
                        s_pt[dst[m]] = rec3_rhs_combine<T>(fv[m], uv[m], cc4, skip[m]);
                    }
                }
            }
        }
        if (t < w.nblock) bkl = blocks[w.block0 + t];
        // phase 1 writes s_rn of other wavefronts' chunks, which they read in
        // the gather
        __syncthreads();
        if (act) {
            nfl = chl.nflags;
            ext = chl.ext;
            nf = fac[w.chunk0 + t];
            // the chunk's along-axis coefficients (as aligned pairs), its
            // neighbours outside it along its axis and its scalar coefficients
            const int ad = chl.axdir, ax = ad >> 1, up = ad & 1, L = chl.len;
            const int cax = ax == 0 ? chl.c0[0] : (ax == 1 ? chl.c0[1] : (DIM == 3 ? chl.c0[2] : 0));
            const int cL_ = cax + (up ? L - 1 : 1 - L);
            T Av[C], Cv[C], Bv[C], ubk, ufw;
            const T aL = cf.base[(ad ^ 1) * cf.cs + cL_], bLax = cf.base[(6 + ax) * cf.cs + cL_];
            const T cLf = cf.base[ad * cf.cs + cL_];
            chunk_end_u<T, DIM>(d, ub, chl, ubk, ufw);
            const ChunkScalars<T> sc = chunk_scalars<T, DIM>(cf, chl);
            chunk_coef_window<T, C>(cf.base + (ad ^ 1) * cf.cs, cax, up, Av);
            chunk_coef_window<T, C>(cf.base + ad * cf.cs, cax, up, Cv);
            if (!DOFF) chunk_coef_window<T, C>(cf.base + (6 + ax) * cf.cs, cax, up, Bv);
            T tb, tf;
            chunk_end_terms_v<T>(chl, Av[0], cLf, ubk, ufw, tb, tf);
            const T *rp = &s_pt[t * PS];
            const T rL = rp[L - 1] - tf - (L == 1 ? tb : T(0));
            sweep_phase1_coefs<T, DIM, false, true, DOFF, C>(
                d, cf, [&](int k) { return k == 0 ? rp[0] - tb : rp[k]; }, rL, chl, t, red, st, Av, Cv, Bv, aL,
                bLax, sc);
        }
    } else {
        // gather: point-major over the workgroup's chunks, so that consecutive
        // lanes read consecutive points of a chunk (whole cache lines along rows)
        // each batch's loads are issued before any of its results is stored;
        // slots past the workgroup's points read chunk 0's first point and land
        // in the spare entry
        constexpr int GB = (DIM == 2) ? 8 : 4;
#pragma unroll
        for (int m0 = 0; m0 < CH; m0 += GB) {
            T rv[GB];
            int dst[GB];
#pragma unroll
            for (int m = 0; m < GB; ++m) {
                const int P = t + (m0 + m) * NT, c = P / CH, k = P % CH;
                const int cc = c < w.nchunk ? c : 0;
                const Chunk ch = s_ch[cc];
                const bool valid = c < w.nchunk && k < ch.len;
                rv[m] = point_rhs_across<T, DIM>(d, cf, ub, fb, ch, valid ? k : 0);
                dst[m] = valid ? c * PS + k : NT * PS;
            }
#pragma unroll
            for (int m = 0; m < GB; ++m) s_pt[dst[m]] = rv[m];
        }
        if (t < w.nblock) bkl = blocks[w.block0 + t];
        __syncthreads();
        if (act) {
            nfl = chl.nflags;
            ext = chl.ext;
            nf = fac[w.chunk0 + t];
            T tb, tf;
            chunk_end_terms<T, DIM>(d, cf, ub, chl, tb, tf);
            const T *rp = &s_pt[t * PS];
            const int L = chl.len;
            const T rL = rp[L - 1] - tf - (L == 1 ? tb : T(0));
            sweep_phase1<T, DIM, false, true, DOFF>(
                d, cf, [&](int k) { return k == 0 ? rp[0] - tb : rp[k]; }, rL, chl, t, red, st);
        }
    }
    __syncthreads();
    // the staging buffer is free until phase 3: it carries the node factors
    reduced_solve_wg<T>(w, act, nfl, ext, nf, bkl, fac, rings, s_rs, s_rn, s_dl, s_x, s_a, s_b, s_pt);
    __syncthreads();
    if (act) sweep_phase3<T, C>(&s_pt[t * PS], t, red, st);
    if constexpr (REC) {
        // scatter over the wavefront's own chunks (it reads only its own rows,
        // so a wavefront-level order suffices), point-major like the gather;
        // every slot and value is read before the stores, which are masked
        // rather than branched
        wave_sync();
        const int lane = t & 63, c0w = t & ~63;
        const int cfb = c0w < w.nchunk ? c0w : 0;
        int slot[C];
        T val[C];
        bool ok[C];
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const int c = c0w + CPS * m + lane / C, k = lane % C;
            const bool inc = c < w.nchunk;
            const int cc = inc ? c : cfb;
            const auto a = s_ca[cc];
            ok[m] = inc && k < (int)(a.meta & 31);
            if constexpr (DIM == 2)
                slot[m] = rec_slot(d, a, ok[m] ? k : 0);
            else
                slot[m] = rec3_slot(d, a, ok[m] ? k : 0);
            val[m] = s_pt[cc * PS + k];
        }
#pragma unroll
        for (int m = 0; m < C; ++m)
            if (ok[m]) ub[slot[m]] = val[m];
    } else {
        __syncthreads();
        // scatter, point-major like the gather
#pragma unroll 4
        for (int m = 0; m < CH; ++m) {
            const int P = t + m * NT, c = P / CH, k = P % CH;
            if (c >= w.nchunk) continue;
            if (k < s_ch[c].len) ub[point_index(d, s_ch[c], k)] = s_pt[c * PS + k];
        }
    }
}

// DOFF: FP64 forward operator (diagonal from the off-diagonal coefficients);
// workgroups of at most NT/2 lanes address their points through the records
// Workgroups of at most NT/2 lanes: at least three waves per SIMD, so at most
// 168 VGPRs per lane
template <typename T, int DIM, int NT, bool DOFF, int C = CH>
__global__ void __launch_bounds__(NT, NT <= twmg::NT / 2 ? 3 : 2) k_block_sweep(Dims d, Coef<T> cf, T *__restrict__ u, const T *__restrict__ f,
                                                    const Chunk *__restrict__ chunks,
                                                    const typename RecOf<DIM>::type *__restrict__ addrs,
                                                    const T *__restrict__ cross, const Block *__restrict__ blocks,
                                                    const WGDesc *__restrict__ wgs, const NodeFac<T> *__restrict__ fac,
                                                    int rings)
{
    constexpr bool REC = NT <= twmg::NT / 2;
    const long long boff = (long long)blockIdx.y * d.bs;
    sweep_wg<T, DIM, NT, DOFF, REC, C>(d, cf, u + boff, f + boff, chunks, addrs, cross, blocks, wgs[blockIdx.x], fac,
                                       rings);
}

// the addressing records of a table, by dimension
template <int DIM> static const typename RecOf<DIM>::type *rec_table(const SweepTable &tab);
template <> const ChunkAddr *rec_table<2>(const SweepTable &tab) { return tab.addrs; }
template <> const ChunkAddr3 *rec_table<3>(const SweepTable &tab) { return tab.addrs3; }

template <typename T, int DIM, bool DOFF>
static hipError_t launch_sweep_dim(const Dims &d, const Coef<T> &c, T *u, const T *f, const SweepTable &tab,
                                   const NodeFac<T> *fac, const T *cross, int batch, hipStream_t s,
                                   const SideStream &side)
{
    const int rings = tab.rings ? 1 : 0;
    const typename RecOf<DIM>::type *recs = rec_table<DIM>(tab);
    // workgroups holding a block of more than NT/2 chunks come first and run
    // with NT lanes; the rest run with NT/2 lanes (a third of the LDS), so that
    // several workgroups share a CU and hide each other's memory waits.  With
    // a side stream the NT-lane launch overlaps the other one.
    // the NT-lane launch goes first, on the caller's stream, so that its few
    // large workgroups are placed before the NT/2-lane ones fill the CUs
    const bool both = tab.nwg_big > 0 && tab.nwg > tab.nwg_big;
    const bool fork = both && side.aux != nullptr;
    hipStream_t ss = s;
    if (fork) {
        hipError_t e = hipEventRecord(side.fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side.aux, side.fork, 0);
        if (e != hipSuccess) return e;
        ss = side.aux;
    }
    if (tab.nwg_big > 0)
        hipLaunchKernelGGL((k_block_sweep<T, DIM, NT, DOFF>), dim3(tab.nwg_big, batch), dim3(NT), 0, s, d, c, u, f,
                           tab.chunks, recs, cross, tab.blocks, tab.wgs, fac, rings);
    if (tab.nwg > tab.nwg_big) {
        const dim3 grid(tab.nwg - tab.nwg_big, batch);
        const WGDesc *wsm = tab.wgs + tab.nwg_big;
        if (tab.nts == NT / 2 && tab.cap == CH) {
            hipLaunchKernelGGL((k_block_sweep<T, DIM, NT / 2, DOFF>), grid, dim3(NT / 2), 0, ss, d, c, u, f,
                               tab.chunks, recs, cross, tab.blocks, wsm, fac, rings);
        } else {
            {
                // narrow workgroups (levels bound by a workgroup's latency),
                // with chunks of up to 16 or of up to 8 points
                if (tab.nts == 64 && tab.cap == CH)
                    hipLaunchKernelGGL((k_block_sweep<T, DIM, 64, DOFF>), grid, dim3(64), 0, ss, d, c, u, f,
                                       tab.chunks, recs, cross, tab.blocks, wsm, fac, rings);
                else if (tab.nts == 128 && tab.cap == CH)
                    hipLaunchKernelGGL((k_block_sweep<T, DIM, 128, DOFF>), grid, dim3(128), 0, ss, d, c, u, f,
                                       tab.chunks, recs, cross, tab.blocks, wsm, fac, rings);
                else if (tab.nts == 64 && tab.cap == SHORT_CH)
                    hipLaunchKernelGGL((k_block_sweep<T, DIM, 64, DOFF, SHORT_CH>), grid, dim3(64), 0, ss, d, c, u, f,
                                       tab.chunks, recs, cross, tab.blocks, wsm, fac, rings);
                else if (tab.nts == 128 && tab.cap == SHORT_CH)
                    hipLaunchKernelGGL((k_block_sweep<T, DIM, 128, DOFF, SHORT_CH>), grid, dim3(128), 0, ss, d, c, u,
                                       f, tab.chunks, recs, cross, tab.blocks, wsm, fac, rings);
                else if (tab.nts == NT / 2 && tab.cap == SHORT_CH)
                    hipLaunchKernelGGL((k_block_sweep<T, DIM, NT / 2, DOFF, SHORT_CH>), grid, dim3(NT / 2), 0, ss, d, c,
                                       u, f, tab.chunks, recs, cross, tab.blocks, wsm, fac, rings);
                else
                    return hipErrorInvalidValue;
            }
        }
    }
    if (fork) {
        hipError_t e = hipEventRecord(side.join, side.aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, side.join, 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_block_sweep(const Dims &d, const Coef<T> &c, T *u, const T *f, const SweepTable &tab, int adj,
                              int batch, hipStream_t s, const SideStream &side)
{
    if (tab.nwg == 0) return hipSuccess;
    const NodeFac<T> *fac;
    const T *cross;
    if constexpr (sizeof(T) == 8) {
        fac = tab.fac64[adj];
        cross = tab.cross64[adj];
    } else {
        fac = tab.fac32[adj];
        cross = tab.cross32[adj];
    }
    const bool doff = sizeof(T) == 8 && adj == 0;
    hipError_t e;
    if (d.dim == 2) {
        if (doff) e = launch_sweep_dim<T, 2, true>(d, c, u, f, tab, fac, cross, batch, s, side);
        else e = launch_sweep_dim<T, 2, false>(d, c, u, f, tab, fac, cross, batch, s, side);
    } else {
        if (doff) e = launch_sweep_dim<T, 3, true>(d, c, u, f, tab, fac, cross, batch, s, side);
        else e = launch_sweep_dim<T, 3, false>(d, c, u, f, tab, fac, cross, batch, s, side);
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Checkerboard (red-black point Gauss-Seidel) half-sweep: Section 2, Fig. 1.
// red = (i + j [+ l]) even.
// ---------------------------------------------------------------------------

// point Gauss-Seidel value at interior node (i, j, l)
template <typename T, int DIM>
__device__ __forceinline__ T point_gs(const Dims &d, const Coef<T> &cf, const T *ub, const T *fb, int i, int j, int l)
{
    const Stencil<DIM> q = stencil_at<DIM>(d, i, j, l);
    T s = fb[q.p] - cf.lo[0][i] * ub[q.nb[0]] - cf.hi[0][i] * ub[q.nb[1]] - cf.lo[1][j] * ub[q.nb[2]] -
          cf.hi[1][j] * ub[q.nb[3]];
    if (DIM == 3) s -= cf.lo[2][l] * ub[q.nb[4]] + cf.hi[2][l] * ub[q.nb[5]];
    return s / diag_at<T, DIM>(cf, i, j, l);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_checker(Dims d, Coef<T> cf, T *__restrict__ u, const T *__restrict__ f,
                                                 int colour)
{
    const long long boff = (long long)blockIdx.y * d.bs;
    T *ub = u + boff;
    const T *fb = f + boff;
    const int rows = lrows(d, DIM);
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int len = lrow_len(d, r);
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            int i, j, l;
            long long p;
            if (!lnode<DIM>(d, r, q, i, j, l, p) || !interior<DIM>(d, i, j, l) || ((i + j + l) & 1) != colour) continue;
            ub[p] = point_gs<T, DIM>(d, cf, ub, fb, i, j, l);
        }
    }
}

static int row_grid(const Dims &d) { return lrow_grid(d); }

template <typename T>
hipError_t launch_checker(const Dims &d, const Coef<T> &c, T *u, const T *f, int colour, int batch, hipStream_t s)
{
    dim3 grid(row_grid(d), batch);
    if (d.dim == 2) hipLaunchKernelGGL((k_checker<T, 2>), grid, dim3(256), 0, s, d, c, u, f, colour);
    else hipLaunchKernelGGL((k_checker<T, 3>), grid, dim3(256), 0, s, d, c, u, f, colour);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Defect d = f - L u (Section 4 step 3), 0 on boundary nodes.
// ---------------------------------------------------------------------------
// r has its own layout (dout): the caller's row-major array or the level's
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_residual(Dims d, Dims dout, Coef<T> cf, const T *__restrict__ u,
                                                  const T *__restrict__ f, T *__restrict__ r)
{
    const long long boff = (long long)blockIdx.y * d.bs, roff = (long long)blockIdx.y * dout.bs;
    const int rows = lrows(d, DIM);
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int len = lrow_len(d, row);
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            int i, j, l;
            long long p;
            if (!lnode<DIM>(d, row, q, i, j, l, p)) continue;
            r[roff + nidx(dout, i, j, l)] =
                interior<DIM>(d, i, j, l) ? defect_at<T, DIM>(d, cf, u + boff, f + boff, i, j, l) : T(0);
        }
    }
}

template <typename T>
hipError_t launch_residual(const Dims &d, const Dims &dout, const Coef<T> &c, const T *u, const T *f, T *r, int batch,
                           hipStream_t s)
{
    dim3 grid(row_grid(d), batch);
    if (d.dim == 2) hipLaunchKernelGGL((k_residual<T, 2>), grid, dim3(256), 0, s, d, dout, c, u, f, r);
    else hipLaunchKernelGGL((k_residual<T, 3>), grid, dim3(256), 0, s, d, dout, c, u, f, r);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused defect + full-weighting restriction (Section 4, fused step 3): one
// thread per coarse interior node sums (1/4,1/2,1/4)^dim weighted fine defects
// around fine node 2I; also clears the coarse correction u_c there (step 4).
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__device__ __forceinline__ T restrict_at(const Dims &fd, const Coef<T> &cf, const T *ub, const T *fb, int I, int J,
                                         int K)
{
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = 0;
#pragma unroll
    for (int c = (DIM == 3 ? -1 : 0); c <= (DIM == 3 ? 1 : 0); ++c) {
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            T rowacc = 0;
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
                const int i = 2 * I + a, j = 2 * J + b, l = (DIM == 3) ? 2 * K + c : 0;
                if (interior<DIM>(fd, i, j, l)) rowacc += w3[a + 1] * defect_at<T, DIM>(fd, cf, ub, fb, i, j, l);
            }
            acc += (DIM == 3 ? w3[c + 1] : T(1)) * w3[b + 1] * rowacc;
        }
    }
    return acc;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_residual_restrict(Dims fd, Dims cd, Coef<T> cf, const T *__restrict__ u,
                                                           const T *__restrict__ f, T *__restrict__ fc,
                                                           T *__restrict__ uc)
{
    const T *ub = u + (long long)blockIdx.y * fd.bs;
    const T *fb = f + (long long)blockIdx.y * fd.bs;
    const long long cboff = (long long)blockIdx.y * cd.bs;
    const int rows = lrows(cd, DIM);
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int len = lrow_len(cd, row);
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            int I, J, K;
            long long p;
            if (!lnode<DIM>(cd, row, q, I, J, K, p) || !interior<DIM>(cd, I, J, K)) continue;
            fc[cboff + p] = restrict_at<T, DIM>(fd, cf, ub, fb, I, J, K);
            uc[cboff + p] = T(0);
        }
    }
}

// ---------------------------------------------------------------------------
// 2D tiles: the stencil kernels of the transfer operators and the norm stage a
// node rectangle of u in LDS once (instead of five neighbour loads per node),
// in the thread order of the plane that holds the rectangle, so that the loads
// are contiguous in either layout.
// ---------------------------------------------------------------------------
// Workgroup w of a 1D grid of n runs on XCD w % 8 (the dispatcher deals them
// out round-robin): give each XCD a contiguous range of tiles, so that
// neighbouring tiles, which share their halo cache lines, meet in one L2.
__device__ __forceinline__ int xcd_tile(int w, int n)
{
    const int q = n / 8, r = n % 8, x = w % 8, k = w / 8;
    return x * q + (x < r ? x : r) + k;
}

// does plane C (column-major) hold node (i, j)?  (false for LAYOUT_ROW)
__device__ __forceinline__ bool in_col(const Dims &d, int i, int j)
{
    return d.layout != LAYOUT_ROW && col_plane(d, i, j);
}

// A node rectangle read by a 256-lane workgroup in two steps: load() issues
// every read of the thread's share (fixed count, indices clamped into the grid
// and the values outside it zeroed, so that no branch separates the reads),
// store() puts them into LDS (row pitch P).  Consecutive threads take
// consecutive nodes along the fast axis of the plane holding the rectangle.
template <typename T, int W, int H> struct RectBuf {
    static constexpr int NQ = (W * H + 255) / 256;
    T v[NQ];
    __device__ __forceinline__ void load(const Dims &d, const T *__restrict__ a, int ia, int ja, bool jfast)
    {
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            const int q = threadIdx.x + 256 * r;
            const int x = jfast ? q / H : q % W, y = jfast ? q % H : q / W;
            const int i = ia + x, j = ja + y;
            const bool ok = q < W * H && i >= 0 && i <= d.n[0] && j >= 0 && j <= d.n[1];
            const int ic = min(max(i, 0), d.n[0]), jc = min(max(j, 0), d.n[1]);
            const T val = a[nidx(d, ic, jc, 0)];
            v[r] = ok ? val : T(0);
        }
    }
    __device__ __forceinline__ void store(T *t, int P, bool jfast) const
    {
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            const int q = threadIdx.x + 256 * r;
            const int x = jfast ? q / H : q % W, y = jfast ? q % H : q / W;
            if (q < W * H) t[y * P + x] = v[r];
        }
    }
};

// The coefficients along a tile's two axes, for nodes ia .. ia+W-1 along x
// and ja .. ja+W-1 along y (clamped into the arrays; entries past the grid are
// never used): s[0..2][x] = lo_x, hi_x, dg_x; s[3..5][y] = lo_y, hi_y, dg_y.
// One read per thread (6 W <= 256).
template <typename T, int W>
__device__ __forceinline__ T tile_coef_load(const Dims &d, const Coef<T> &cf, int ia, int ja)
{
    const int q = threadIdx.x, a = q / W, k = q % W;
    if (q >= 6 * W) return T(0);
    const int ax = a / 3, kind = a % 3;
    const int idx = min(max((ax ? ja : ia) + k, 0), ax ? d.n[1] : d.n[0]);
    // the block's arrays by offset (an index into the pointer arrays would be
    // a read of a private copy of the descriptor)
    const int arr = kind == 2 ? 6 + ax : 2 * ax + kind;
    return cf.base[arr * cf.cs + idx];
}

// fused defect + full weighting, 16 x 16 coarse interior nodes per workgroup:
// u on the 35 x 35 fine rectangle around them and the defect on the inner
// 33 x 33 are staged in LDS, each fine defect computed once
template <typename T>
__global__ void __launch_bounds__(256) k_restrict_tile(Dims fd, Dims cd, Coef<T> cf, const T *__restrict__ u,
                                                       const T *__restrict__ f, T *__restrict__ fc,
                                                       T *__restrict__ uc)
{
    constexpr int CT = 16, FW = 2 * CT + 1, UW = FW + 2;
    __shared__ T su[UW * UW];
    __shared__ T sd[FW * FW];
    const int tx = (cd.n[0] - 1 + CT - 1) / CT, ty = (cd.n[1] - 1 + CT - 1) / CT;
    const int tile = xcd_tile(blockIdx.x, tx * ty);
    const int I0 = 1 + (tile % tx) * CT, J0 = 1 + (tile / tx) * CT;
    const int fi = 2 * I0 - 1, fj = 2 * J0 - 1; // first fine node of the defect rectangle
    const T *ub = u + (long long)blockIdx.y * fd.bs;
    const T *fb = f + (long long)blockIdx.y * fd.bs;
    const bool jf = in_col(fd, fi + CT, fj + CT);
    __shared__ T sc[6 * FW];
    {
        // every read of the workgroup issued before any is stored
        RectBuf<T, UW, UW> ru;
        RectBuf<T, FW, FW> rf;
        ru.load(fd, ub, fi - 1, fj - 1, jf);
        rf.load(fd, fb, fi, fj, jf);
        const T cv = tile_coef_load<T, FW>(fd, cf, fi, fj);
        __builtin_amdgcn_sched_barrier(0);
        ru.store(su, UW, jf);
        rf.store(sd, FW, jf);
        if (threadIdx.x < 6 * FW) sc[threadIdx.x] = cv;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (FW * FW + 255) / 256; ++r) {
        const int q = threadIdx.x + 256 * r;
        if (q >= FW * FW) break;
        const int x = jf ? q / FW : q % FW, y = jf ? q % FW : q / FW;
        const int i = fi + x, j = fj + y;
        T rd = 0;
        if (i > 0 && i < fd.n[0] && j > 0 && j < fd.n[1]) {
            const T *c = &su[(y + 1) * UW + (x + 1)];
            T sum = sc[x] * c[-1] + sc[FW + x] * c[1];
            sum += sc[3 * FW + y] * c[-UW] + sc[4 * FW + y] * c[UW];
            const T dg = sc[2 * FW + x] + sc[5 * FW + y];
            rd = sd[y * FW + x] - (sum + dg * c[0]);
        }
        sd[y * FW + x] = rd;
    }
    __syncthreads();
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};
    const long long cb = (long long)blockIdx.y * cd.bs;
    for (int q = threadIdx.x; q < CT * CT; q += blockDim.x) {
        const int a = jf ? q / CT : q % CT, b = jf ? q % CT : q / CT;
        const int I = I0 + a, J = J0 + b;
        if (I >= cd.n[0] || J >= cd.n[1]) continue;
        const T *c = &sd[(2 * b + 1) * FW + (2 * a + 1)];
        T acc = 0;
#pragma unroll
        for (int bb = -1; bb <= 1; ++bb) {
            T rowacc = 0;
#pragma unroll
            for (int aa = -1; aa <= 1; ++aa) rowacc += w3[aa + 1] * c[bb * FW + aa];
            acc += w3[bb + 1] * rowacc;
        }
        const long long p = cb + nidx(cd, I, J, 0);
        fc[p] = acc;
        uc[p] = T(0);
    }
}

// bilinear prolongation + update, 32 x 32 fine nodes per workgroup; the coarse
// 17 x 17 rectangle under them is staged in LDS
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_tile(Dims fd, Dims cd, const T *__restrict__ ec, T *__restrict__ u)
{
    constexpr int FT = 32, CW = FT / 2 + 1;
    __shared__ T se[CW * CW];
    const int tx = (fd.n[0] + FT) / FT, ty = (fd.n[1] + FT) / FT;
    const int tile = xcd_tile(blockIdx.x, tx * ty);
    const int i0 = (tile % tx) * FT, j0 = (tile / tx) * FT;
    T *ub = u + (long long)blockIdx.y * fd.bs;
    const T *eb = ec + (long long)blockIdx.y * cd.bs;
    const bool jf = in_col(fd, i0 + FT / 2, j0 + FT / 2);
    // the fine values this thread updates are read together with the coarse
    // rectangle
    constexpr int NQ = FT * FT / 256;
    T uf[NQ];
    long long pf[NQ];
    bool okf[NQ];
    {
        RectBuf<T, CW, CW> re;
        re.load(cd, eb, i0 / 2, j0 / 2, jf);
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            const int q = threadIdx.x + 256 * r;
            const int x = jf ? q / FT : q % FT, y = jf ? q % FT : q / FT;
            const int i = i0 + x, j = j0 + y;
            okf[r] = i > 0 && i < fd.n[0] && j > 0 && j < fd.n[1];
            pf[r] = nidx(fd, min(i, fd.n[0]), min(j, fd.n[1]), 0);
            uf[r] = ub[pf[r]];
        }
        __builtin_amdgcn_sched_barrier(0);
        re.store(se, CW, jf);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const int q = threadIdx.x + 256 * r;
        const int x = jf ? q / FT : q % FT, y = jf ? q % FT : q / FT;
        const int i = i0 + x, j = j0 + y;
        // coarse neighbours in the rectangle: (I - i0/2, J - j0/2)
        const int X0 = (i >> 1) - i0 / 2, X1 = ((i + 1) >> 1) - i0 / 2;
        const int Y0 = (j >> 1) - j0 / 2, Y1 = ((j + 1) >> 1) - j0 / 2;
        const T r0 = (X0 == X1) ? se[Y0 * CW + X0] : T(0.5) * (se[Y0 * CW + X0] + se[Y0 * CW + X1]);
        const T r1 = (X0 == X1) ? se[Y1 * CW + X0] : T(0.5) * (se[Y1 * CW + X0] + se[Y1 * CW + X1]);
        const T v = (Y0 == Y1) ? r0 : T(0.5) * (r0 + r1);
        if (okf[r]) ub[pf[r]] = uf[r] + v;
    }
}

// interpolated coarse correction at fine interior node (i, j, l): weights 1
// (even index) or 1/2 + 1/2 (odd index) per axis
template <typename T, int DIM>
__device__ __forceinline__ T prolong_at(const Dims &cd, const T *eb, int i, int j, int l)
{
    const int I0 = i >> 1, I1 = (i + 1) >> 1, J0 = j >> 1, J1 = (j + 1) >> 1;
    const int K0 = l >> 1, K1 = (l + 1) >> 1;
    // 3D split coarse level: the 2 x 2 x 2 coarse box at fixed offsets in the
    // plane of its first corner when that corner lies 3 or more inside it
    bool fast = false;
    P3 q0{0, 0, 0, 0, 0};
    if (DIM == 3 && cd.layout == LAYOUT_TWEED3) {
        q0 = p3_at(cd, I0, J0, K0);
        fast = q0.margin >= 3;
    }
    auto cval = [&](int I, int J, int K) -> T {
        if (DIM == 3 && cd.layout == LAYOUT_TWEED3 && fast)
            return eb[q0.p + (I - I0) * q0.sx + (J - J0) * q0.sy + (K - K0) * q0.sz];
        return eb[nidx(cd, I, J, K)];
    };
    T pl[2];
#pragma unroll
    for (int kk = 0; kk < (DIM == 3 ? 2 : 1); ++kk) {
        const int K = kk ? K1 : K0;
        const T r0 = (I0 == I1) ? cval(I0, J0, K) : T(0.5) * (cval(I0, J0, K) + cval(I1, J0, K));
        const T r1 = (I0 == I1) ? cval(I0, J1, K) : T(0.5) * (cval(I0, J1, K) + cval(I1, J1, K));
        pl[kk] = (J0 == J1) ? r0 : T(0.5) * (r0 + r1);
    }
    if (DIM == 2) return pl[0];
    return (K0 == K1) ? pl[0] : T(0.5) * (pl[0] + pl[1]);
}

// the axes of plane PL: fast axis PL, then (y, z) for 0, (x, z) for 1, (x, y) for 2
template <int PL> struct PlaneAxes {
    static constexpr int F = PL, A = PL == 0 ? 1 : 0, B = PL == 2 ? 1 : 2;
};
template <int PL> struct PlaneC {
    static constexpr int value = PL;
};
// tiles of plane PL: 16 nodes along F, 4 along A, 4 NB along B
template <int PL, int NB> __host__ __device__ __forceinline__ int ptiles(const Dims &d)
{
    using X = PlaneAxes<PL>;
    return ((d.n[X::F] + 16) / 16) * ((d.n[X::A] + 4) / 4) * ((d.n[X::B] + 4 * NB) / (4 * NB));
}
template <int PL> __device__ __forceinline__ int slot_in_plane(const Dims &d, int i, int j, int l)
{
    const int S0 = d.n[0] + 1, S1 = d.n[1] + 1, S2 = d.n[2] + 1, nn = (int)d.nn;
    if (PL == 0) return i + S0 * (j + S1 * l);
    if (PL == 1) return nn + j + S1 * (i + S0 * l);
    return 2 * nn + l + S2 * (i + S0 * j);
}
// (i, j, l) of the node at (f, a, b) in plane PL's axes
template <int PL> __device__ __forceinline__ void plane_xyz(int f, int a, int b, int &i, int &j, int &l)
{
    using X = PlaneAxes<PL>;
    int c[3];
    c[X::F] = f;
    c[X::A] = a;
    c[X::B] = b;
    i = c[0];
    j = c[1];
    l = c[2];
}

// The tile of plane PL at (f0, a0, b0) (along F, A, B): this thread's column
// of NB consecutive nodes along B, op(PlaneC<PL>, f, a, b) with the first
// node's coordinates (b a multiple of NB) unless the whole column lies
// outside the grid.
template <int PL, int NB, typename Op>
__device__ __forceinline__ void tile3_plane(const Dims &d, int f0, int a0, int b0, Op &&op)
{
    using X = PlaneAxes<PL>;
    const int q = threadIdx.x;
    const int f = f0 + (q & 15), a = a0 + ((q >> 4) & 3), b = b0 + NB * (q >> 6);
    if (f > d.n[X::F] || a > d.n[X::A] || b > d.n[X::B]) return;
    op(PlaneC<PL>(), f, a, b);
}

// 3D stencil kernels walk the nodes of every plane of the layout in tiles of
// 16 along the plane's fast axis F by 4 along A by 4 NB along B, a thread
// holding NB consecutive nodes along B (a wavefront reads four whole 128-byte
// runs per load): the loads of a column are issued together and the values
// its nodes share (coefficients along F and A, coarse values) are read once.
// A tile handles only the nodes kept in its plane, so the three tile families
// visit every node once; the row-major layout has plane 0 only.  The levels
// carry their tile lists with each tile's plane and origin (on the split
// layout only the tiles that hold nodes of their plane); arrays without one
// (a caller's row-major array) decode the tile number.  The plane is uniform
// per workgroup and a template argument below the branch, so no coordinate is
// picked by a run-time axis index.
template <int NB> __device__ __forceinline__ void tile3_decode(const Dims &d, int k, int &pl, int &f0, int &a0, int &b0)
{
    if (d.tiles) {
        const Tile3E e = d.tiles[k];
        pl = e.x & 3;
        f0 = e.x >> 2;
        a0 = e.y & 0xffff;
        b0 = e.y >> 16;
    } else {
        // row-major: plane 0 only
        const int tf = (d.n[0] + 16) / 16, ta = (d.n[1] + 4) / 4;
        pl = 0;
        f0 = (k % tf) * 16;
        a0 = ((k / tf) % ta) * 4;
        b0 = (k / (tf * ta)) * (4 * NB);
    }
}
template <int NB, typename Op> __device__ __forceinline__ void tile3_visit(const Dims &d, int k, Op &&op)
{
    int pl, f0, a0, b0;
    tile3_decode<NB>(d, k, pl, f0, a0, b0);
    if (pl == 0)
        tile3_plane<0, NB>(d, f0, a0, b0, op);
    else if (pl == 1)
        tile3_plane<1, NB>(d, f0, a0, b0, op);
    else
        tile3_plane<2, NB>(d, f0, a0, b0, op);
}
// Tiles a launch visits: the level's list, else every tile of the row-major
// layout
template <int NB> __host__ __device__ __forceinline__ int tile3_count(const Dims &d)
{
    return d.tiles ? d.ntiles : ptiles<0, NB>(d);
}
// Tile of grid-stride iteration it: xcd_tile is a bijection of [0, nt), and
// with a grid of a multiple of 8 workgroups (or one per tile) every iteration
// of a workgroup stays on its XCD, which works through one contiguous range of
// the tiles
__device__ __forceinline__ int tile3_index(int it, int nt) { return xcd_tile(it, nt); }

// The NB nodes of a column: coordinates, slots in plane PL, ok (in the grid
// and kept in plane PL) and in (also interior)
template <int NB> struct Col3 {
    int i[NB], j[NB], l[NB], sl[NB];
    bool ok[NB], in[NB];
};
template <int PL, int NB> __device__ __forceinline__ Col3<NB> col3(const Dims &d, int f, int a, int b)
{
    using X = PlaneAxes<PL>;
    Col3<NB> c;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        plane_xyz<PL>(f, a, b + k, c.i[k], c.j[k], c.l[k]);
        c.ok[k] = b + k <= d.n[X::B] && (d.layout != LAYOUT_TWEED3 || plane3(d, c.i[k], c.j[k], c.l[k]) == PL);
        c.in[k] = c.ok[k] && interior<3>(d, c.i[k], c.j[k], c.l[k]);
        c.sl[k] = slot_in_plane<PL>(d, c.i[k], c.j[k], c.l[k]);
    }
    return c;
}

// 32-bit slot of a 3D node and its plane's strides (every per-problem array
// is below 2^31 entries, which set-up checks); margin as for P3.  For the
// row-major layout the strides are the row-major ones and margin is large.
struct P3i {
    int p, sx, sy, sz, margin;
};
__device__ __forceinline__ P3i p3i_at(const Dims &d, int i, int j, int l)
{
    const int S0 = d.n[0] + 1, S1 = d.n[1] + 1, S2 = d.n[2] + 1;
    P3i q;
    if (d.layout != LAYOUT_TWEED3) {
        q.p = i + S0 * (j + S1 * l);
        q.sx = 1;
        q.sy = S0;
        q.sz = S0 * S1;
        q.margin = 1 << 20;
        return q;
    }
    const int ip = min(i, d.n[0] - i), jp = min(j, d.n[1] - j), lp = min(l, d.n[2] - l);
    const int pl = (ip <= jp && ip <= lp) ? 0 : (jp <= lp ? 1 : 2);
    const int nn = (int)d.nn;
    if (pl == 0) {
        q.p = i + S0 * (j + S1 * l);
        q.sx = 1;
        q.sy = S0;
        q.sz = S0 * S1;
        q.margin = min(jp, lp) - ip;
    } else if (pl == 1) {
        q.p = nn + j + S1 * (i + S0 * l);
        q.sx = S1;
        q.sy = 1;
        q.sz = S1 * S0;
        q.margin = min(ip, lp) - jp;
    } else {
        q.p = 2 * nn + l + S2 * (i + S0 * j);
        q.sx = S2;
        q.sy = S2 * S0;
        q.sz = 1;
        q.margin = min(ip, jp) - lp;
    }
    return q;
}
__device__ __forceinline__ int slot3(const Dims &d, int i, int j, int l) { return p3i_at(d, i, j, l).p; }

// nodes per thread of the 3D stencil kernels (the restriction reads a 3 x 3
// box per fine plane of its column, so it holds fewer)
constexpr int COL_NB = 2, COL_NB_RESTRICT = 2;

// Defects of a thread's column of nodes (0 where not interior), with u read
// from a box staged in LDS: the workgroup's tile of plane PL at (F0, A0, B0) plus a
// one-node halo, BX_F x BX_A x BX_B nodes in (F, A, B) order, each read once
// from its own slot whatever plane keeps it (0 off the grid).  A wavefront's
// loads then cover runs along F, and a node's six neighbours come from LDS
// instead of six more loads through the vector cache.  Every thread of the
// workgroup calls it (it synchronises the workgroup); c receives the
// thread's column (no node of a column off the grid is ok).  Same summation
// order as defect_at.
constexpr int BX_F = 16 + 2, BX_A = 4 + 2, BX_B = 4 * COL_NB + 2, BX_N = BX_F * BX_A * BX_B;
template <typename T, int PL>
__device__ __forceinline__ void tile3_defects(const Dims &d, const Coef<T> &cf, const T *__restrict__ ub,
                                              const T *__restrict__ fb, int F0, int A0, int B0, T *s_u,
                                              Col3<COL_NB> &c, T (&out)[COL_NB])
{
    using X = PlaneAxes<PL>;
    constexpr int NB = COL_NB, NQ = (BX_N + 255) / 256;
    const int t = threadIdx.x;
    const int f = F0 + (t & 15), a = A0 + ((t >> 4) & 3), b = B0 + NB * (t >> 6);
    const bool colin = f <= d.n[X::F] && a <= d.n[X::A];
    c = col3<PL, NB>(d, colin ? f : 0, colin ? a : 0, b);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        c.ok[k] = c.ok[k] && colin;
        c.in[k] = c.in[k] && colin;
    }
    // every load of the tile issued before any is used: the box, the
    // column's f, the coefficients
    T v[NQ];
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const int q = t + 256 * r;
        const int qq = q < BX_N ? q : 0;
        int cc[3];
        cc[X::F] = F0 - 1 + qq % BX_F;
        cc[X::A] = A0 - 1 + (qq / BX_F) % BX_A;
        cc[X::B] = B0 - 1 + qq / (BX_F * BX_A);
        const bool in = q < BX_N && cc[0] >= 0 && cc[0] <= d.n[0] && cc[1] >= 0 && cc[1] <= d.n[1] &&
                        cc[2] >= 0 && cc[2] <= d.n[2];
        const T val = ub[slot3(d, in ? cc[0] : 0, in ? cc[1] : 0, in ? cc[2] : 0)];
        v[r] = in ? val : T(0);
    }
    T fv[NB], lb[NB], hb[NB], gb[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        fv[k] = fb[c.in[k] ? c.sl[k] : 0];
        const int bk = min(b + k, d.n[X::B]);
        lb[k] = cf.lo[X::B][bk];
        hb[k] = cf.hi[X::B][bk];
        gb[k] = cf.dg[X::B][bk];
    }
    const int fc = min(f, d.n[X::F]), ac = min(a, d.n[X::A]);
    const T lf = cf.lo[X::F][fc], hf = cf.hi[X::F][fc], gf = cf.dg[X::F][fc];
    const T la = cf.lo[X::A][ac], ha = cf.hi[X::A][ac], ga = cf.dg[X::A][ac];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const int q = t + 256 * r;
        if (q < BX_N) s_u[q] = v[r];
    }
    __syncthreads();
    int st[3];
    st[X::F] = 1;
    st[X::A] = BX_F;
    st[X::B] = BX_F * BX_A;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int p = (1 + NB * (t >> 6) + k) * (BX_F * BX_A) + (1 + ((t >> 4) & 3)) * BX_F + 1 + (t & 15);
        T lo[3], hi[3], dg[3];
        lo[X::F] = lf;
        hi[X::F] = hf;
        dg[X::F] = gf;
        lo[X::A] = la;
        hi[X::A] = ha;
        dg[X::A] = ga;
        lo[X::B] = lb[k];
        hi[X::B] = hb[k];
        dg[X::B] = gb[k];
        T sum = lo[0] * s_u[p - st[0]] + hi[0] * s_u[p + st[0]];
        sum += lo[1] * s_u[p - st[1]] + hi[1] * s_u[p + st[1]];
        T g = dg[0] + dg[1];
        sum += lo[2] * s_u[p - st[2]] + hi[2] * s_u[p + st[2]];
        g += dg[2];
        out[k] = c.in[k] ? fv[k] - (sum + g * s_u[p]) : T(0);
    }
}

// Runs body(PlaneC<PL>(), F0, A0, B0) for each tile of the workgroup's
// grid-stride iterations, with the whole workgroup (after a barrier, so that
// the previous tile's LDS reads are done)
template <typename Body> __device__ __forceinline__ void tile3_wg_loop(const Dims &d, Body &&body)
{
    const int nt = tile3_count<COL_NB>(d);
    for (int it = blockIdx.x; it < nt; it += gridDim.x) {
        int pl, F0, A0, B0;
        tile3_decode<COL_NB>(d, tile3_index(it, nt), pl, F0, A0, B0);
        __syncthreads();
        if (pl == 0)
            body(PlaneC<0>(), F0, A0, B0);
        else if (pl == 1)
            body(PlaneC<1>(), F0, A0, B0);
        else
            body(PlaneC<2>(), F0, A0, B0);
    }
}

// defect d = f - L u of every node (0 on boundary nodes) into r (layout of d)
template <typename T>
__global__ void __launch_bounds__(256) k_residual3(Dims d, Coef<T> cf, const T *__restrict__ u,
                                                   const T *__restrict__ f, T *__restrict__ r)
{
    __shared__ T s_u[BX_N];
    const long long boff = (long long)blockIdx.y * d.bs;
    tile3_wg_loop(d, [&](auto plc, int F0, int A0, int B0) {
        constexpr int PL = decltype(plc)::value;
        Col3<COL_NB> c;
        T dv[COL_NB];
        tile3_defects<T, PL>(d, cf, u + boff, f + boff, F0, A0, B0, s_u, c, dv);
#pragma unroll
        for (int k = 0; k < COL_NB; ++k)
            if (c.ok[k]) r[boff + c.sl[k]] = dv[k];
    });
}

// per-workgroup maximum of |f - L u| over interior nodes (optionally the
// defect rounded to FP32 into r32)
template <typename T, bool TO32>
__global__ void __launch_bounds__(256) k_resnorm3(Dims d, Coef<T> cf, const T *__restrict__ u,
                                                  const T *__restrict__ f, float *__restrict__ r32,
                                                  double *__restrict__ partial)
{
    __shared__ T s_u[BX_N];
    const long long boff = (long long)blockIdx.y * d.bs;
    double m = 0.0;
    bool nan = false;
    tile3_wg_loop(d, [&](auto plc, int F0, int A0, int B0) {
        constexpr int PL = decltype(plc)::value;
        Col3<COL_NB> c;
        T dv[COL_NB];
        tile3_defects<T, PL>(d, cf, u + boff, f + boff, F0, A0, B0, s_u, c, dv);
#pragma unroll
        for (int k = 0; k < COL_NB; ++k) {
            if (TO32 && c.ok[k]) r32[boff + c.sl[k]] = (float)dv[k];
            const double av = fabs((double)dv[k]);
            nan = nan || (av != av);
            m = fmax(m, av);
        }
    });
    if (nan) m = __builtin_inf();
    m = block_max(m);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = m;
}


// u += P e_c over a column of fine nodes (b even).  The column interpolates
// from a coarse box of 2 x 2 across by NB/2 + 1 along B, read once: at the
// strides of one coarse plane when the box lies in it, otherwise with every
// slot in general form.  Same arithmetic as prolong_at.
template <typename T, int PL, int NB>
__device__ __forceinline__ void col_prolong(const Dims &fd, const Dims &cd, const T *__restrict__ eb,
                                            T *__restrict__ ub, const Col3<NB> &c, int f, int a, int b)
{
    using X = PlaneAxes<PL>;
    constexpr int MB = NB / 2 + 1;
    // the box's first corner (coarse coordinates along F, A, B), clamped into
    // the coarse grid for columns that reach past the fine interior (their
    // values are not used)
    const int F0 = min(f >> 1, cd.n[X::F] - 1), A0 = min(a >> 1, cd.n[X::A] - 1),
              B0 = min(b >> 1, cd.n[X::B] - (MB - 1));
    int I0, J0, K0;
    plane_xyz<PL>(F0, A0, B0, I0, J0, K0);
    const P3i q = p3i_at(cd, I0, J0, K0);
    const bool reg = q.margin >= 2 * (MB - 1) + 1 && q.margin >= 3;
    int st[3];
    st[0] = q.sx;
    st[1] = q.sy;
    st[2] = q.sz;
    const int sF = st[X::F], sA = st[X::A], sB = st[X::B];
    int slot[MB][2][2];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int iff = 0; iff < 2; ++iff) {
                int I, J, K;
                plane_xyz<PL>(F0 + iff, A0 + ia, B0 + m, I, J, K);
                slot[m][ia][iff] = reg ? q.p + m * sB + ia * sA + iff * sF : slot3(cd, I, J, K);
            }
    T cv[MB][2][2], uv[NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int iff = 0; iff < 2; ++iff) cv[m][ia][iff] = eb[slot[m][ia][iff]];
#pragma unroll
    for (int k = 0; k < NB; ++k) uv[k] = ub[c.in[k] ? c.sl[k] : c.sl[0]];
    __builtin_amdgcn_sched_barrier(0);
    // equal end indices (the fine coordinate is even) per x, y, z
    const bool eqF = !(f & 1), eqA = !(a & 1);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        bool eq[3];
        eq[X::F] = eqF;
        eq[X::A] = eqA;
        eq[X::B] = !(k & 1);
        // coarse value at selectors (sx, sy, sz) in {0, 1}: index 0 is the
        // lower end, 1 the upper
        auto cval = [&](int sx, int sy, int sz) -> T {
            int sel[3];
            sel[0] = sx;
            sel[1] = sy;
            sel[2] = sz;
            const int mb = sel[X::B] ? (k + 1) >> 1 : k >> 1;
            return cv[mb][sel[X::A]][sel[X::F]];
        };
        T pl2[2];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const T r0 = eq[0] ? cval(0, 0, kk) : T(0.5) * (cval(0, 0, kk) + cval(1, 0, kk));
            const T r1 = eq[0] ? cval(0, 1, kk) : T(0.5) * (cval(0, 1, kk) + cval(1, 1, kk));
            pl2[kk] = eq[1] ? r0 : T(0.5) * (r0 + r1);
        }
        if (c.in[k]) ub[c.sl[k]] = uv[k] + (eq[2] ? pl2[0] : T(0.5) * (pl2[0] + pl2[1]));
    }
}

// u += P e_c at fine interior nodes
template <typename T>
__global__ void __launch_bounds__(256) k_prolong3(Dims fd, Dims cd, const T *__restrict__ ec, T *__restrict__ u)
{
    T *ub = u + (long long)blockIdx.y * fd.bs;
    const T *eb = ec + (long long)blockIdx.y * cd.bs;
    const int nt = tile3_count<COL_NB>(fd);
    for (int it = blockIdx.x; it < nt; it += gridDim.x)
        tile3_visit<COL_NB>(fd, tile3_index(it, nt), [&](auto plc, int fq, int aq, int bq) {
            constexpr int PL = decltype(plc)::value;
            const Col3<COL_NB> c = col3<PL, COL_NB>(fd, fq, aq, bq);
            col_prolong<T, PL, COL_NB>(fd, cd, eb, ub, c, fq, aq, bq);
        });
}

// full weighting of the defect array dr (fine layout, 0 on boundary nodes)
// at coarse interior nodes, over coarse tiles; clears the coarse correction.
// A column of coarse nodes reads the fine 3 x 3 boxes of its 2 NB + 1 fine
// planes along B once when every node's fine 3 x 3 x 3 box lies 3 or more
// inside one fine plane (then all of them lie in the same one); otherwise
// each node is addressed in general form.  Same weights and summation order
// as restrict_at.
template <typename T, int PL, int NB>
__device__ __forceinline__ void col_restrict(const Dims &fd, const Dims &cd, const T *__restrict__ db,
                                             T *__restrict__ fcb, T *__restrict__ ucb, const Col3<NB> &c)
{
    using X = PlaneAxes<PL>;
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};
    bool fast = true;
#pragma unroll
    for (int k = 0; k < NB; ++k)
        fast = fast && c.in[k] && p3i_at(fd, 2 * c.i[k], 2 * c.j[k], 2 * c.l[k]).margin >= 3;
    if (fast) {
        const P3i pc = p3i_at(fd, 2 * c.i[0], 2 * c.j[0], 2 * c.l[0]);
        int st[3];
        st[0] = pc.sx;
        st[1] = pc.sy;
        st[2] = pc.sz;
        const int sF = st[X::F], sA = st[X::A], sB = st[X::B];
        // fine planes m = 0 .. 2 NB along B from the first node's centre - 1
        T v[2 * NB + 1][3][3];
#pragma unroll
        for (int m = 0; m < 2 * NB + 1; ++m)
#pragma unroll
            for (int oa = 0; oa < 3; ++oa)
#pragma unroll
                for (int of = 0; of < 3; ++of) v[m][oa][of] = db[pc.p + (m - 1) * sB + (oa - 1) * sA + (of - 1) * sF];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            T acc = 0;
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz) {
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy) {
                    T rowacc = 0;
#pragma unroll
                    for (int cx = -1; cx <= 1; ++cx) {
                        int o[3];
                        o[0] = cx;
                        o[1] = cy;
                        o[2] = cz;
                        rowacc += w3[cx + 1] * v[2 * k + 1 + o[X::B]][o[X::A] + 1][o[X::F] + 1];
                    }
                    acc += w3[cz + 1] * w3[cy + 1] * rowacc;
                }
            }
            fcb[c.sl[k]] = acc;
            ucb[c.sl[k]] = T(0);
        }
    } else {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (!c.in[k]) continue;
            const int I = c.i[k], J = c.j[k], K = c.l[k];
            T acc = 0;
#pragma unroll
            for (int cz = -1; cz <= 1; ++cz) {
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy) {
                    T rowacc = 0;
#pragma unroll
                    for (int cx = -1; cx <= 1; ++cx)
                        rowacc += w3[cx + 1] * db[slot3(fd, 2 * I + cx, 2 * J + cy, 2 * K + cz)];
                    acc += w3[cz + 1] * w3[cy + 1] * rowacc;
                }
            }
            fcb[c.sl[k]] = acc;
            ucb[c.sl[k]] = T(0);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fw_restrict3(Dims fd, Dims cd, const T *__restrict__ dr, T *__restrict__ fc,
                                                      T *__restrict__ uc)
{
    const T *db = dr + (long long)blockIdx.y * fd.bs;
    const long long cboff = (long long)blockIdx.y * cd.bs;
    constexpr int NB = COL_NB_RESTRICT;
    const int nt = tile3_count<NB>(cd);
    for (int it = blockIdx.x; it < nt; it += gridDim.x)
        tile3_visit<NB>(cd, tile3_index(it, nt), [&](auto plc, int fq, int aq, int bq) {
            constexpr int PL = decltype(plc)::value;
            const Col3<NB> c = col3<PL, NB>(cd, fq, aq, bq);
            col_restrict<T, PL, NB>(fd, cd, db, fc + cboff, uc + cboff, c);
        });
}

// u += e at interior nodes (FP64 update of iterative refinement), 3D tiles
__global__ void __launch_bounds__(256) k_ir_update3(Dims d, double *__restrict__ u, const float *__restrict__ e)
{
    const long long boff = (long long)blockIdx.y * d.bs;
    const int nt = tile3_count<COL_NB>(d);
    for (int it = blockIdx.x; it < nt; it += gridDim.x)
        tile3_visit<COL_NB>(d, tile3_index(it, nt), [&](auto plc, int fq, int aq, int bq) {
            constexpr int PL = decltype(plc)::value;
            const Col3<COL_NB> c = col3<PL, COL_NB>(d, fq, aq, bq);
            double uv[COL_NB];
            float ev[COL_NB];
#pragma unroll
            for (int k = 0; k < COL_NB; ++k) {
                const long long p = boff + (c.in[k] ? c.sl[k] : c.sl[0]);
                uv[k] = u[p];
                ev[k] = e[p];
            }
#pragma unroll
            for (int k = 0; k < COL_NB; ++k)
                if (c.in[k]) u[boff + c.sl[k]] = uv[k] + (double)ev[k];
        });
}

// workgroups of a 3D tile launch: one per tile
template <int NB> static int tile3_grid(const Dims &d) { return tile3_count<NB>(d); }

// host: whether tile t of plane pl holds nodes of its plane.  Away from the
// centre lines n/2 the primed coordinates are monotone along each axis inside
// a tile, so the plane's region (an intersection of half-spaces in them)
// meets the tile only if it holds one of the tile's corners; a tile that
// straddles a centre line is kept.
template <int PL, int NB> static bool tile3_active(const Dims &d, int t)
{
    using X = PlaneAxes<PL>;
    constexpr int TB = 4 * NB;
    const int tf = (d.n[X::F] + 16) / 16, ta = (d.n[X::A] + 4) / 4;
    const int f0 = (t % tf) * 16, a0 = ((t / tf) % ta) * 4, b0 = (t / (tf * ta)) * TB;
    const int nf = d.n[X::F], na = d.n[X::A], nb = d.n[X::B];
    const int f1 = std::min(f0 + 15, nf), a1 = std::min(a0 + 3, na), b1 = std::min(b0 + TB - 1, nb);
    if ((f0 < nf / 2 && f1 > nf / 2) || (a0 < na / 2 && a1 > na / 2) || (b0 < nb / 2 && b1 > nb / 2)) return true;
    for (int k = 0; k < 8; ++k) {
        int c[3];
        c[X::F] = (k & 1) ? f1 : f0;
        c[X::A] = (k & 2) ? a1 : a0;
        c[X::B] = (k & 4) ? b1 : b0;
        if (plane3(d, c[0], c[1], c[2]) == PL) return true;
    }
    return false;
}

std::vector<Tile3E> tile3_list(const Dims &d)
{
    static_assert(COL_NB == COL_NB_RESTRICT, "one tile list serves every 3D stencil kernel");
    std::vector<Tile3E> out;
    const bool split = d.layout == LAYOUT_TWEED3;
    auto add = [&](auto plc) {
        constexpr int PL = decltype(plc)::value;
        using X = PlaneAxes<PL>;
        const int tf = (d.n[X::F] + 16) / 16, ta = (d.n[X::A] + 4) / 4, nt = ptiles<PL, COL_NB>(d);
        for (int t = 0; t < nt; ++t) {
            if (split && !tile3_active<PL, COL_NB>(d, t)) continue;
            const int f0 = (t % tf) * 16, a0 = ((t / tf) % ta) * 4, b0 = (t / (tf * ta)) * (4 * COL_NB);
            out.push_back(Tile3E{PL | (f0 << 2), a0 | (b0 << 16)});
        }
    };
    add(PlaneC<0>());
    if (split) {
        add(PlaneC<1>());
        add(PlaneC<2>());
    }
    return out;
}

template <typename T>
hipError_t launch_residual_restrict(const Dims &fd, const Dims &cd, const Coef<T> &c, const T *u, const T *f, T *fc,
                                    T *uc, int batch, hipStream_t s, T *dscr)
{
    if (fd.dim == 2) {
        dim3 tiles(((cd.n[0] - 1 + 15) / 16) * ((cd.n[1] - 1 + 15) / 16), batch);
        hipLaunchKernelGGL((k_restrict_tile<T>), tiles, dim3(256), 0, s, fd, cd, c, u, f, fc, uc);
        return hipGetLastError();
    }
    if (fd.layout == LAYOUT_TWEED3) {
        // each fine defect once, into the scratch array (fine layout), then
        // the 27-point weighting from it
        if (!dscr) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_residual3<T>), dim3(tile3_grid<COL_NB>(fd), batch), dim3(256), 0, s, fd, c, u, f, dscr);
        hipLaunchKernelGGL((k_fw_restrict3<T>), dim3(tile3_grid<COL_NB_RESTRICT>(cd), batch), dim3(256), 0, s, fd, cd, dscr, fc, uc);
        return hipGetLastError();
    }
    dim3 grid(row_grid(cd), batch);
    hipLaunchKernelGGL((k_residual_restrict<T, 3>), grid, dim3(256), 0, s, fd, cd, c, u, f, fc, uc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused bilinear/trilinear prolongation + update (Section 4, fused step 5):
// u += P e_c in index space; e_c's boundary entries are zero.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_prolong_add(const Dims &fd, const Dims &cd, const T *ec, T *u, int batch, hipStream_t s)
{
    if (fd.dim == 2) {
        dim3 tiles(((fd.n[0] + 32) / 32) * ((fd.n[1] + 32) / 32), batch);
        hipLaunchKernelGGL((k_prolong_tile<T>), tiles, dim3(256), 0, s, fd, cd, ec, u);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_prolong3<T>), dim3(tile3_grid<COL_NB>(fd), batch), dim3(256), 0, s, fd, cd, ec, u);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Coarsest-level direct solve (Section 4 step 4): u_I = A_II^{-1}(f_I - A_IB u_B)
// with the inverse precomputed at setup; one workgroup per batch problem.
// ---------------------------------------------------------------------------
// the whole workgroup; rhs: nunk entries of workgroup scratch (LDS)
template <typename T, int DIM>
__device__ __forceinline__ void coarse_solve_wg(const Dims &d, const Coef<T> &cf, T *ub, const T *fb,
                                                const T *__restrict__ ainv, int nunk, T *rhs)
{
    const int nx = d.n[0] - 1, ny = d.n[1] - 1;
    for (int q = threadIdx.x; q < nunk; q += blockDim.x) {
        const int i = 1 + q % nx, j = 1 + (q / nx) % ny, l = (DIM == 3) ? 1 + q / (nx * ny) : 0;
        const long long p = i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0);
        T r = fb[p];
        if (i == 1) r -= cf.lo[0][i] * ub[p - 1];
        if (i == nx) r -= cf.hi[0][i] * ub[p + 1];
        if (j == 1) r -= cf.lo[1][j] * ub[p - d.st[1]];
        if (j == ny) r -= cf.hi[1][j] * ub[p + d.st[1]];
        if (DIM == 3) {
            const int nz = d.n[2] - 1;
            if (l == 1) r -= cf.lo[2][l] * ub[p - d.st[2]];
            if (l == nz) r -= cf.hi[2][l] * ub[p + d.st[2]];
        }
        rhs[q] = r;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nunk; q += blockDim.x) {
        T s = 0;
        for (int k = 0; k < nunk; ++k) s += ainv[(long long)q * nunk + k] * rhs[k];
        const int i = 1 + q % nx, j = 1 + (q / nx) % ny, l = (DIM == 3) ? 1 + q / (nx * ny) : 0;
        ub[i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0)] = s;
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_coarse_solve(Dims d, Coef<T> cf, T *__restrict__ u, const T *__restrict__ f,
                                                      const T *__restrict__ ainv, int nunk)
{
    __shared__ T rhs[1024];
    T *ub = u + (long long)blockIdx.x * d.bs;
    const T *fb = f + (long long)blockIdx.x * d.bs;
    coarse_solve_wg<T, DIM>(d, cf, ub, fb, ainv, nunk, rhs);
}

template <typename T>
hipError_t launch_coarse_solve(const Dims &d, const Coef<T> &c, T *u, const T *f, const T *ainv, int nunk, int batch,
                               hipStream_t s)
{
    if (d.dim == 2) hipLaunchKernelGGL((k_coarse_solve<T, 2>), dim3(batch), dim3(256), 0, s, d, c, u, f, ainv, nunk);
    else hipLaunchKernelGGL((k_coarse_solve<T, 3>), dim3(batch), dim3(256), 0, s, d, c, u, f, ainv, nunk);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Coarse-level sub-cycle in one workgroup per problem (Section 4 steps 1-6 on
// the levels that fit in LDS).  Everything the sub-cycle reads lives in LDS:
// the read-only image (level descriptors, coefficients, block tables and the
// operation list) is copied in first, then the first tail level's u and f.
// The operations run with barriers between them, and u is copied back.  With
// no global memory access inside the cycle, each operation costs LDS latency
// and barriers only.
// ---------------------------------------------------------------------------

// Block sweep of one workgroup descriptor with u, f, coefficients and tables
// in LDS: each lane forms its chunk's right-hand sides directly (no staging),
// phases 1-3 as in the main sweep, new values written in place.
// C: the longest chunk of the level (the code runs over C positions per lane).
// ONEWAVE: the descriptor's chunks and blocks all sit in wavefront 0, which
// runs this alone (the other wavefronts skip the operation).
template <typename T, int DIM, int C, bool ONEWAVE = false>
__device__ __forceinline__ void sweep_wg_tail(const Dims &d, const Coef<T> &cf, T *ub, const T *fb,
                                              const Chunk *chunks, const Block *blocks, const WGDesc w,
                                              const NodeFac<T> *fac, int rings, T *s_rs, T *s_rn, T *s_dl, T *s_x,
                                              T *s_a, T *s_b)
{
    const int t = threadIdx.x;
    const bool act = t < w.nchunk;
    const RedArrays<T> red{nullptr, nullptr, s_rs, nullptr, nullptr, s_rn, s_x, nullptr};
    LaneState<T, C> st;
    uint8_t nfl = 0;
    int ext = -1;
    NodeFac<T> nf{0, 0, 0, 0};
    Chunk ch = chunks[w.chunk0];
    if (act) {
        ch = chunks[w.chunk0 + t];
        nfl = ch.nflags;
        ext = ch.ext;
        nf = fac[w.chunk0 + t];
        const int L = ch.len;
        T tb, tf;
        chunk_end_terms<T, DIM>(d, cf, ub, ch, tb, tf);
        // the chunk's right-hand sides first, all reads issued together, then
        // the elimination chain
        T R[C];
        if (DIM == 2) {
            // tail levels are row-major: the lane builds its chunk's record
            const ChunkAddr a = row_chunk_addr(d, ch);
            T cm, cp;
            chunk_cross_coefs<T>(cf, ch, cm, cp);
#pragma unroll
            for (int k = 0; k < C; ++k) R[k] = point_rhs_rec<T>(d, a, cm, cp, ub, fb, k < L ? k : 0);
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) R[k] = point_rhs_across<T, DIM>(d, cf, ub, fb, ch, k < L ? k : 0);
        }
        // the last point's value, selected without indexing the array
        T rl = R[0];
#pragma unroll
        for (int k = 1; k < C; ++k) rl = (k == L - 1) ? R[k] : rl;
        const T rL = rl - tf - (L == 1 ? tb : T(0));
        sweep_phase1<T, DIM, false, true, false, C>(
            d, cf, [&](int k) { return k == 0 ? R[0] - tb : R[k]; }, rL, ch, t, red, st);
    }
    wg_sync<ONEWAVE>();
    Block bk;
    bk.type = BT_CHAIN;
    if (t < w.nblock) bk = blocks[w.block0 + t];
    reduced_solve_wg<T, ONEWAVE>(w, act, nfl, ext, nf, bk, fac, rings, s_rs, s_rn, s_dl, s_x, s_a, s_b,
                                  (T *)nullptr);
    wg_sync<ONEWAVE>();
    if (act) {
        if (DIM == 2) {
            const ChunkAddr a = row_chunk_addr(d, ch);
            sweep_phase3_each<T, C>(t, red, st, [&](int k, T v) { ub[rec_slot(d, a, k)] = v; });
        } else {
            sweep_phase3_each<T, C>(t, red, st, [&](int k, T v) { ub[point_index(d, ch, k)] = v; });
        }
    }
}

template <typename T, int DIM>
__global__ void __launch_bounds__(TAIL_NT) k_tail_cycle(TailPlan<T> P, T *__restrict__ u, const T *__restrict__ f)
{
    __shared__ __align__(16) unsigned char s_mem[TAIL_BYTES];
    __shared__ T s_rs[TAIL_NT], s_rn[TAIL_NT], s_dl[TAIL_NT], s_x[TAIL_NT];
    __shared__ T s_a[TAIL_NT / 64], s_b[TAIL_NT / 64];
    {
        // the copies issue a batch of loads per thread before storing any (a
        // plain loop waited for each load: one round trip per 16 bytes)
        const uint4 *src = reinterpret_cast<const uint4 *>(P.image);
        uint4 *dst = reinterpret_cast<uint4 *>(s_mem);
        const int n16 = P.image_bytes / 16;
        constexpr int CB = 16;
        // (positions past the end load and store the batch's first one again:
        // no branch separates the loads from each other)
        for (int q0 = threadIdx.x; q0 < n16; q0 += CB * TAIL_NT) {
            uint4 v[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const int q = q0 + k * TAIL_NT;
                v[k] = src[q < n16 ? q : q0];
            }
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const int q = q0 + k * TAIL_NT;
                dst[q < n16 ? q : q0] = v[k];
            }
        }
    }
    __syncthreads();
    const TailLevel *lev = reinterpret_cast<const TailLevel *>(s_mem + P.lev_off);
    const TailOp *ops = reinterpret_cast<const TailOp *>(s_mem + P.ops_off);
    auto arr = [&](int off) { return reinterpret_cast<T *>(s_mem + off); };
    auto coef = [&](const TailLevel &L) { return make_coef<T>(arr(L.co), L.cs); };
    const long long boff = (long long)blockIdx.x * P.nn0;
    T *ug = u + boff;
    const T *fg = f + boff;
    {
        T *u0 = arr(lev[0].uoff), *f0 = arr(lev[0].foff);
        const int nn = (int)P.nn0;
        constexpr int CB = 8;
        for (int q0 = threadIdx.x; q0 < nn; q0 += CB * TAIL_NT) {
            T uv[CB], fv[CB];
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const int q = q0 + k * TAIL_NT, qc = q < nn ? q : q0;
                uv[k] = ug[qc];
                fv[k] = fg[qc];
            }
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const int q = q0 + k * TAIL_NT, qc = q < nn ? q : q0;
                u0[qc] = uv[k];
                f0[qc] = fv[k];
            }
        }
    }
    __syncthreads();
    for (int o = 0; o < P.nops; ++o) {
        const TailOp op = ops[o];
        const TailLevel &L = lev[op.lv];
        T *us = arr(L.uoff);
        const T *fs = arr(L.foff);
        const Dims d = L.d;
        const Coef<T> cf = coef(L);
        if (op.kind == TO_SWEEP) {
            const int sl = op.slot, c = op.colour, nw = L.nwg[sl][c];
            const Chunk *chunks = reinterpret_cast<const Chunk *>(s_mem + L.chunk_off[sl][c]);
            const Block *blocks = reinterpret_cast<const Block *>(s_mem + L.block_off[sl][c]);
            const WGDesc *wgs = reinterpret_cast<const WGDesc *>(s_mem + L.wg_off[sl][c]);
            const NodeFac<T> *fac = reinterpret_cast<const NodeFac<T> *>(s_mem + L.fac_off[sl][c]);
            if (L.onewave[sl][c]) {
                // every descriptor fits wavefront 0: it alone runs the
                // sweep, with no workgroup barrier until the operation's end
                if (threadIdx.x < 64) {
                    for (int w = 0; w < nw; ++w) {
                        if (L.short_chunks)
                            sweep_wg_tail<T, DIM, TAIL_SHORT_CH, true>(d, cf, us, fs, chunks, blocks, wgs[w], fac,
                                                                       L.rings[sl][c], s_rs, s_rn, s_dl, s_x, s_a,
                                                                       s_b);
                        else
                            sweep_wg_tail<T, DIM, CH, true>(d, cf, us, fs, chunks, blocks, wgs[w], fac,
                                                            L.rings[sl][c], s_rs, s_rn, s_dl, s_x, s_a, s_b);
                        wave_sync();
                    }
                }
            } else {
                for (int w = 0; w < nw; ++w) {
                    if (L.short_chunks)
                        sweep_wg_tail<T, DIM, TAIL_SHORT_CH>(d, cf, us, fs, chunks, blocks, wgs[w], fac,
                                                             L.rings[sl][c], s_rs, s_rn, s_dl, s_x, s_a, s_b);
                    else
                        sweep_wg_tail<T, DIM, CH>(d, cf, us, fs, chunks, blocks, wgs[w], fac, L.rings[sl][c], s_rs,
                                                  s_rn, s_dl, s_x, s_a, s_b);
                    __syncthreads();
                }
            }
        } else if (op.kind == TO_CHECKER) {
            const int nx = d.n[0] - 1, ny = d.n[1] - 1, nz = DIM == 3 ? d.n[2] - 1 : 1;
            for (int q = threadIdx.x; q < nx * ny * nz; q += blockDim.x) {
                const int i = 1 + q % nx, j = 1 + (q / nx) % ny, l = DIM == 3 ? 1 + q / (nx * ny) : 0;
                if (((i + j + l) & 1) != op.colour) continue;
                us[i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0)] = point_gs<T, DIM>(d, cf, us, fs, i, j, l);
            }
        } else if (op.kind == TO_RESTRICT) {
            const TailLevel &C = lev[op.lv + 1];
            const Dims cd = C.d;
            T *uc = arr(C.uoff);
            T *fc = arr(C.foff);
            for (int q = threadIdx.x; q < (int)cd.nn; q += blockDim.x) {
                const int I = q % (cd.n[0] + 1), J = (q / (cd.n[0] + 1)) % (cd.n[1] + 1),
                          K = DIM == 3 ? q / ((cd.n[0] + 1) * (cd.n[1] + 1)) : 0;
                fc[q] = interior<DIM>(cd, I, J, K) ? restrict_at<T, DIM>(d, cf, us, fs, I, J, K) : T(0);
                uc[q] = T(0);
            }
        } else if (op.kind == TO_PROLONG) {
            const TailLevel &C = lev[op.lv + 1];
            const Dims cd = C.d;
            const T *uc = arr(C.uoff);
            const int nx = d.n[0] - 1, ny = d.n[1] - 1, nz = DIM == 3 ? d.n[2] - 1 : 1;
            for (int q = threadIdx.x; q < nx * ny * nz; q += blockDim.x) {
                const int i = 1 + q % nx, j = 1 + (q / nx) % ny, l = DIM == 3 ? 1 + q / (nx * ny) : 0;
                us[i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0)] += prolong_at<T, DIM>(cd, uc, i, j, l);
            }
        } else if (op.kind == TO_MAP) {
            // the level's sub-cycle in one step: each lane forms one unknown's
            // new value from all old values and right-hand sides, then all write
            const int nx = d.n[0] - 1, ny = d.n[1] - 1, nu = P.map_nu;
            const int i = threadIdx.x;
            T acc = 0;
            long long slot = 0;
            if (i < nu) {
                // unknown k at node (ik, jk, lk), x fastest; the map's loads
                // are independent of the sum, so unrolling keeps many in flight
                int ik = 1, jk = 1, lk = 1;
#pragma unroll 16
                for (int k = 0; k < nu; ++k) {
                    const long long pk = ik + jk * d.st[1] + (DIM == 3 ? lk * d.st[2] : 0);
                    acc += P.map[(long long)k * nu + i] * us[pk];
                    acc += P.map[(long long)(nu + k) * nu + i] * fs[pk];
                    if (++ik > nx) {
                        ik = 1;
                        if (++jk > ny) {
                            jk = 1;
                            ++lk;
                        }
                    }
                }
                const int ii = 1 + i % nx, ji = 1 + (i / nx) % ny, li = DIM == 3 ? 1 + i / (nx * ny) : 0;
                slot = ii + ji * d.st[1] + (DIM == 3 ? li * d.st[2] : 0);
            }
            __syncthreads();
            if (i < nu) us[slot] = acc;
        } else { // TO_SOLVE
            coarse_solve_wg<T, DIM>(d, cf, us, fs, P.ainv, P.nunk, arr(P.rhs_off));
        }
        __syncthreads();
    }
    {
        const T *u0 = arr(lev[0].uoff);
        for (int q = threadIdx.x; q < (int)P.nn0; q += blockDim.x) ug[q] = u0[q];
    }
}

template <typename T>
hipError_t launch_tail_cycle(const TailPlan<T> &p, T *u, const T *f, int batch, hipStream_t s)
{
    if (p.dim == 2) hipLaunchKernelGGL((k_tail_cycle<T, 2>), dim3(batch), dim3(TAIL_NT), 0, s, p, u, f);
    else hipLaunchKernelGGL((k_tail_cycle<T, 3>), dim3(batch), dim3(TAIL_NT), 0, s, p, u, f);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Infinity norm of the defect over interior nodes (Section 4 stopping rule):
// per-workgroup maxima, then one workgroup reduces them.  Maxima are order
// independent, so the result is bitwise reproducible.  Optionally writes the
// defect rounded to FP32 (iterative refinement's right-hand side).
// ---------------------------------------------------------------------------

// 2D tiled version: 32 x 32 nodes per tile, u staged with a one-node halo;
// the workgroups stride over the tiles of their problem
template <typename T, bool TO32>
__global__ void __launch_bounds__(256) k_resnorm_tile(Dims d, Coef<T> cf, const T *__restrict__ u,
                                                      const T *__restrict__ f, float *__restrict__ r32,
                                                      double *__restrict__ partial)
{
    constexpr int TS = 32, UW = TS + 2;
    __shared__ T su[UW * UW];
    __shared__ T sc[6 * TS];
    const long long boff = (long long)blockIdx.y * d.bs;
    const int tx = (d.n[0] + TS) / TS, ty = (d.n[1] + TS) / TS;
    double m = 0.0;
    bool nan = false;
    for (int it = blockIdx.x; it < tx * ty; it += gridDim.x) {
        const int tile = (int)gridDim.x == tx * ty ? xcd_tile(it, tx * ty) : it;
        const int i0 = (tile % tx) * TS, j0 = (tile / tx) * TS;
        const bool jf = in_col(d, i0 + TS / 2, j0 + TS / 2);
        __syncthreads();
        // every read of the tile issued before any is used: u with its halo,
        // the thread's f values, the coefficient strips
        constexpr int NQ = TS * TS / 256;
        T fv[NQ];
        {
            RectBuf<T, UW, UW> ru;
            ru.load(d, u + boff, i0 - 1, j0 - 1, jf);
#pragma unroll
            for (int r = 0; r < NQ; ++r) {
                const int q = threadIdx.x + 256 * r;
                const int x = jf ? q / TS : q % TS, y = jf ? q % TS : q / TS;
                fv[r] = f[boff + nidx(d, min(i0 + x, d.n[0]), min(j0 + y, d.n[1]), 0)];
            }
            const T cv = tile_coef_load<T, TS>(d, cf, i0, j0);
            __builtin_amdgcn_sched_barrier(0);
            ru.store(su, UW, jf);
            if (threadIdx.x < 6 * TS) sc[threadIdx.x] = cv;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            const int q = threadIdx.x + 256 * r;
            const int x = jf ? q / TS : q % TS, y = jf ? q % TS : q / TS;
            const int i = i0 + x, j = j0 + y;
            if (i > d.n[0] || j > d.n[1]) continue;
            T rd = 0;
            if (i > 0 && i < d.n[0] && j > 0 && j < d.n[1]) {
                const T *c = &su[(y + 1) * UW + (x + 1)];
                T sum = sc[x] * c[-1] + sc[TS + x] * c[1];
                sum += sc[3 * TS + y] * c[-UW] + sc[4 * TS + y] * c[UW];
                const T dg = sc[2 * TS + x] + sc[5 * TS + y];
                rd = fv[r] - (sum + dg * c[0]);
            }
            if (TO32) r32[boff + nidx(d, i, j, 0)] = (float)rd;
            const double a = fabs((double)rd);
            nan = nan || (a != a);
            m = fmax(m, a);
        }
    }
    if (nan) m = __builtin_inf();
    m = block_max(m);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = m;
}

// per-problem maximum: workgroup b reduces problem b's n partial maxima into
// out[b].  Each lane issues its 8 loads of a step before combining them, so a
// step costs one memory round trip (the partials hold no NaN: a NaN defect is
// recorded as +inf).
constexpr int MAXF_NT = 1024, MAXF_U = 8;
__global__ void __launch_bounds__(MAXF_NT) k_max_final(const double *__restrict__ partial, int n,
                                                       double *__restrict__ out)
{
    const double *pb = partial + (long long)blockIdx.x * n;
    double m = 0.0;
    for (int k0 = threadIdx.x; k0 < n; k0 += MAXF_NT * MAXF_U) {
        double v[MAXF_U];
#pragma unroll
        for (int q = 0; q < MAXF_U; ++q) {
            const int k = k0 + q * MAXF_NT;
            v[q] = k < n ? pb[k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < MAXF_U; ++q) m = fmax(m, v[q]);
    }
    m = block_max(m);
    if (threadIdx.x == 0) out[blockIdx.x] = m;
}

template <typename T>
hipError_t launch_resnorm(const Dims &d, const Coef<T> &c, const T *u, const T *f, double *partial, int npart,
                          double *out, int batch, hipStream_t s)
{
    int gx = npart / batch;
    if (gx < 1) return hipErrorInvalidValue;
    const int rows = lrow_grid(d);
    if (gx > rows) gx = rows;
    if (d.dim == 2) {
        const int nt = ((d.n[0] + 32) / 32) * ((d.n[1] + 32) / 32);
        if (gx > nt) gx = nt;
        hipLaunchKernelGGL((k_resnorm_tile<T, false>), dim3(gx, batch), dim3(256), 0, s, d, c, u, f, nullptr, partial);
    } else {
        if (gx >= tile3_count<COL_NB>(d)) gx = tile3_count<COL_NB>(d);
        else if (gx >= 8) gx &= ~7; // a multiple of 8: iterations stay on their XCD
        hipLaunchKernelGGL((k_resnorm3<T, false>), dim3(gx, batch), dim3(256), 0, s, d, c, u, f, nullptr, partial);
    }
    hipLaunchKernelGGL(k_max_final, dim3(batch), dim3(MAXF_NT), 0, s, partial, gx, out);
    return hipGetLastError();
}

hipError_t launch_resnorm_to_f32(const Dims &d, const Coef<double> &c, const double *u, const double *f, float *r32,
                                 double *partial, int npart, double *out, int batch, hipStream_t s)
{
    int gx = npart / batch;
    if (gx < 1) return hipErrorInvalidValue;
    const int rows = lrow_grid(d);
    if (gx > rows) gx = rows;
    if (d.dim == 2) {
        const int nt = ((d.n[0] + 32) / 32) * ((d.n[1] + 32) / 32);
        if (gx > nt) gx = nt;
        hipLaunchKernelGGL((k_resnorm_tile<double, true>), dim3(gx, batch), dim3(256), 0, s, d, c, u, f, r32,
                           partial);
    } else {
        if (gx >= tile3_count<COL_NB>(d)) gx = tile3_count<COL_NB>(d);
        else if (gx >= 8) gx &= ~7; // a multiple of 8: iterations stay on their XCD
        hipLaunchKernelGGL((k_resnorm3<double, true>), dim3(gx, batch), dim3(256), 0, s, d, c, u, f, r32, partial);
    }
    hipLaunchKernelGGL(k_max_final, dim3(batch), dim3(MAXF_NT), 0, s, partial, gx, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free defect norm: the partial maxima live in a file-scope device
// array instead of handle-owned memory.  Host code never uses the array's
// name as an address: scratch_init resolves each device's copy once, with
// that device current, and the launcher passes that address to the kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[NOALLOC_PARTS];
constexpr int SCRATCH_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[SCRATCH_MAX_DEV] = {};

hipError_t scratch_init()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
    return hipSuccess;
}

hipError_t launch_resnorm_noalloc(const Dims &d, const Coef<double> &c, const double *u, const double *f,
                                  double *out, int batch, hipStream_t s)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return hipErrorInvalidDevice;
    double *partial;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        partial = g_scratch_ptr[dev];
    }
    if (!partial) return hipErrorNotInitialized;
    int gx = NOALLOC_PARTS / batch;
    if (gx < 1) return hipErrorInvalidValue;
    const int rows = lrow_grid(d);
    if (gx > rows) gx = rows;
    // every slot the final reduction reads (gx per problem) is written by the
    // first kernel: nothing needs clearing
    if (d.dim == 2) {
        const int nt = ((d.n[0] + 32) / 32) * ((d.n[1] + 32) / 32);
        if (gx > nt) gx = nt;
        hipLaunchKernelGGL((k_resnorm_tile<double, false>), dim3(gx, batch), dim3(256), 0, s, d, c, u, f, nullptr,
                           partial);
    } else {
        if (gx >= tile3_count<COL_NB>(d)) gx = tile3_count<COL_NB>(d);
        else if (gx >= 8) gx &= ~7; // a multiple of 8: iterations stay on their XCD
        hipLaunchKernelGGL((k_resnorm3<double, false>), dim3(gx, batch), dim3(256), 0, s, d, c, u, f, nullptr,
                           partial);
    }
    // one workgroup over all problems' partial maxima: the batch's maximum
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(MAXF_NT), 0, s, partial, gx * batch, out);
    return hipGetLastError();
}

// u += e at interior nodes (FP64 update of iterative refinement)
template <int DIM> __global__ void __launch_bounds__(256) k_ir_update(Dims d, double *__restrict__ u, const float *__restrict__ e)
{
    const long long boff = (long long)blockIdx.y * d.bs;
    const int rows = lrows(d, DIM);
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int len = lrow_len(d, row);
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            int i, j, l;
            long long p;
            if (!lnode<DIM>(d, row, q, i, j, l, p) || !interior<DIM>(d, i, j, l)) continue;
            u[boff + p] += (double)e[boff + p];
        }
    }
}

hipError_t launch_ir_update(const Dims &d, double *u, const float *e, int batch, hipStream_t s)
{
    dim3 grid(row_grid(d), batch);
    if (d.dim == 2) hipLaunchKernelGGL((k_ir_update<2>), grid, dim3(256), 0, s, d, u, e);
    else hipLaunchKernelGGL(k_ir_update3, dim3(tile3_grid<COL_NB>(d), batch), dim3(256), 0, s, d, u, e);
    return hipGetLastError();
}

// boundary nodes <- bc (when given; bc is a row-major node array), interior <- 0
// (when asked); u has layout d.layout
template <int DIM>
__global__ void __launch_bounds__(256) k_set_boundary(Dims d, double *__restrict__ u, const double *__restrict__ bc,
                                                      int zero_interior)
{
    const long long boff = (long long)blockIdx.y * d.bs, bboff = (long long)blockIdx.y * d.nn;
    const int rows = lrows(d, DIM);
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int len = lrow_len(d, row);
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            int i, j, l;
            long long p;
            if (!lnode<DIM>(d, row, q, i, j, l, p)) continue;
            if (interior<DIM>(d, i, j, l)) {
                if (zero_interior) u[boff + p] = 0.0;
            } else if (bc) {
                u[boff + p] = bc[bboff + i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0)];
            }
        }
    }
}

hipError_t launch_set_boundary(const Dims &d, double *u, const double *bc, int zero_interior, int batch,
                               hipStream_t s)
{
    dim3 grid(row_grid(d), batch);
    if (d.dim == 2) hipLaunchKernelGGL((k_set_boundary<2>), grid, dim3(256), 0, s, d, u, bc, zero_interior);
    else hipLaunchKernelGGL((k_set_boundary<3>), grid, dim3(256), 0, s, d, u, bc, zero_interior);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout conversion between a row-major node array and a split layout through
// 32 x 32 LDS tiles: the row-major side and plane R are accessed along rows,
// plane C along its columns, so every access is contiguous.
// ---------------------------------------------------------------------------
template <typename T, bool TO_SPLIT>
__global__ void __launch_bounds__(256) k_convert(Dims d, const T *__restrict__ src, T *__restrict__ dst)
{
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const long long rb = (long long)blockIdx.z * d.nn, sb = (long long)blockIdx.z * d.bs;
    const long long cst = d.n[1] + 1;
    if (TO_SPLIT) {
        for (int r = ty; r < 32; r += 8) {
            const int i = i0 + tx, j = j0 + r;
            if (i <= d.n[0] && j <= d.n[1]) tile[r][tx] = src[rb + i + j * d.st[1]];
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = i0 + tx, j = j0 + r;
            if (i <= d.n[0] && j <= d.n[1] && !col_plane(d, i, j)) dst[sb + i + j * d.st[1]] = tile[r][tx];
        }
        for (int c = ty; c < 32; c += 8) {
            const int i = i0 + c, j = j0 + tx;
            if (i <= d.n[0] && j <= d.n[1] && col_plane(d, i, j)) dst[sb + d.nn + j + i * cst] = tile[tx][c];
        }
    } else {
        for (int r = ty; r < 32; r += 8) {
            const int i = i0 + tx, j = j0 + r;
            if (i <= d.n[0] && j <= d.n[1] && !col_plane(d, i, j)) tile[r][tx] = src[sb + i + j * d.st[1]];
        }
        for (int c = ty; c < 32; c += 8) {
            const int i = i0 + c, j = j0 + tx;
            if (i <= d.n[0] && j <= d.n[1] && col_plane(d, i, j)) tile[tx][c] = src[sb + d.nn + j + i * cst];
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = i0 + tx, j = j0 + r;
            if (i <= d.n[0] && j <= d.n[1]) dst[rb + i + j * d.st[1]] = tile[r][tx];
        }
    }
}

// the same for the 3D split layout, one node per thread in row-major order
// (the row-major side is contiguous; planes 1 and 2 are written or read
// along their strided axis)
template <typename T, bool TO_SPLIT>
__global__ void __launch_bounds__(256) k_convert3(Dims d, const T *__restrict__ src, T *__restrict__ dst)
{
    const long long rb = (long long)blockIdx.y * d.nn, sb = (long long)blockIdx.y * d.bs;
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < d.nn; p += (long long)gridDim.x * 256) {
        const int i = (int)(p % d.st[1]), j = (int)((p / d.st[1]) % (d.n[1] + 1)), l = (int)(p / d.st[2]);
        const long long q = nidx(d, i, j, l);
        if (TO_SPLIT) dst[sb + q] = src[rb + p];
        else dst[rb + p] = src[sb + q];
    }
}

template <typename T>
hipError_t launch_convert(const Dims &d, const T *src, T *dst, int to_split, int batch, hipStream_t s)
{
    if (d.layout == LAYOUT_ROW)
        return hipMemcpyAsync(dst, src, sizeof(T) * (size_t)d.nn * batch, hipMemcpyDeviceToDevice, s);
    if (d.layout == LAYOUT_TWEED3) {
        long long nb = (d.nn + 255) / 256;
        if (nb > 16384) nb = 16384;
        const dim3 grid((unsigned)nb, batch);
        if (to_split) hipLaunchKernelGGL((k_convert3<T, true>), grid, dim3(256), 0, s, d, src, dst);
        else hipLaunchKernelGGL((k_convert3<T, false>), grid, dim3(256), 0, s, d, src, dst);
        return hipGetLastError();
    }
    dim3 grid((d.n[0] + 32) / 32, (d.n[1] + 32) / 32, batch);
    if (to_split) hipLaunchKernelGGL((k_convert<T, true>), grid, dim3(256), 0, s, d, src, dst);
    else hipLaunchKernelGGL((k_convert<T, false>), grid, dim3(256), 0, s, d, src, dst);
    return hipGetLastError();
}

template <typename T> __global__ void __launch_bounds__(256) k_fill(T *__restrict__ p, long long n, T v)
{
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        p[k] = v;
}

template <typename T> hipError_t launch_fill(T *p, long long n, T v, hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Boundary-data gradient of L = sum(w u):  g_b = w_b - sum_{interior q ~ b} A[q,b] lam_q
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256) k_bc_grad(Dims d, Coef<double> cf, const double *__restrict__ lam,
                                                 const double *__restrict__ w, double *__restrict__ g)
{
    const long long boff = (long long)blockIdx.y * d.nn;
    const int rows = nrows(d, DIM);
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int j = row % (d.n[1] + 1), l = row / (d.n[1] + 1);
        for (int i = threadIdx.x; i <= d.n[0]; i += blockDim.x) {
            const long long p = i + j * d.st[1] + (DIM == 3 ? l * d.st[2] : 0);
            if (interior<DIM>(d, i, j, l)) {
                g[boff + p] = 0.0;
                continue;
            }
            double s = w[boff + p];
            const int c[3] = {i, j, l};
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
#pragma unroll
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    int q[3] = {c[0], c[1], c[2]};
                    q[a] += sgn;
                    if (q[a] < 0 || q[a] > d.n[a]) continue;
                    if (!interior<DIM>(d, q[0], q[1], q[2])) continue;
                    // row q's coefficient pointing back at p (direction -sgn along a)
                    const double A = (sgn > 0) ? cf.lo[a][q[a]] : cf.hi[a][q[a]];
                    s -= A * lam[boff + p + sgn * d.st[a]];
                }
            }
            g[boff + p] = s;
        }
    }
}

hipError_t launch_bc_grad(const Dims &d, const Coef<double> &fwd, const double *lam, const double *w, double *g,
                          int batch, hipStream_t s)
{
    dim3 grid(row_grid(d), batch);
    if (d.dim == 2) hipLaunchKernelGGL((k_bc_grad<2>), grid, dim3(256), 0, s, d, fwd, lam, w, g);
    else hipLaunchKernelGGL((k_bc_grad<3>), grid, dim3(256), 0, s, d, fwd, lam, w, g);
    return hipGetLastError();
}

// explicit instantiations
#define TWMG_INST(T)                                                                                                  \
    template hipError_t launch_block_sweep<T>(const Dims &, const Coef<T> &, T *, const T *, const SweepTable &, int, \
                                              int, hipStream_t, const SideStream &);                                  \
    template hipError_t launch_checker<T>(const Dims &, const Coef<T> &, T *, const T *, int, int, hipStream_t);     \
    template hipError_t launch_residual<T>(const Dims &, const Dims &, const Coef<T> &, const T *, const T *, T *,  \
                                           int, hipStream_t);                                                         \
    template hipError_t launch_convert<T>(const Dims &, const T *, T *, int, int, hipStream_t);                      \
    template hipError_t launch_residual_restrict<T>(const Dims &, const Dims &, const Coef<T> &, const T *,          \
                                                    const T *, T *, T *, int, hipStream_t, T *);                      \
    template hipError_t launch_prolong_add<T>(const Dims &, const Dims &, const T *, T *, int, hipStream_t);         \
    template hipError_t launch_coarse_solve<T>(const Dims &, const Coef<T> &, T *, const T *, const T *, int, int,   \
                                               hipStream_t);                                                          \
    template hipError_t launch_resnorm<T>(const Dims &, const Coef<T> &, const T *, const T *, double *, int,        \
                                          double *, int, hipStream_t);                                                \
    template hipError_t launch_fill<T>(T *, long long, T, hipStream_t);                                             \
    template hipError_t launch_tail_cycle<T>(const TailPlan<T> &, T *, const T *, int, hipStream_t);

TWMG_INST(double)
TWMG_INST(float)

} // namespace twmg
