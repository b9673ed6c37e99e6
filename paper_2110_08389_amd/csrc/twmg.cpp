// Host side of libtwmg: grid hierarchy, coefficients, block tables of the
// relaxation motifs, the multigrid cycle driver and the C ABI (include/twmg.h).
#include "sweep_core.h"
#include "twmg.h"
#include "twmg_debug.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace twmg;

namespace {

constexpr int MAXLEV = 24;
constexpr int MAX_COARSE_UNK = 1024;

// ---------------------------------------------------------------------------
// Geometry (Section 5: eq. tanh, eq. tanh_inv; sinh centre clustering)
// ---------------------------------------------------------------------------
int make_coords(int kind, double c, int n, double L, const double *given, std::vector<double> &x)
{
    x.assign(n + 1, 0.0);
    for (int i = 0; i <= n; ++i) {
        const double s = double(i) / double(n);
        switch (kind) {
        case MG_UNIFORM: x[i] = L * s; break;
        case MG_TANH_WALL:
            if (!(c > 0)) return MG_EINVAL;
            x[i] = 0.5 * L * (1.0 + std::tanh(c * (2.0 * s - 1.0)) / std::tanh(c));
            break;
        case MG_TANH_CENTRE:
            if (!(c > 0)) return MG_EINVAL;
            x[i] = (2 * i <= n) ? 0.5 * L * std::tanh(2.0 * c * s) / std::tanh(c)
                                : 0.5 * L * (2.0 - std::tanh(c * (2.0 - 2.0 * s)) / std::tanh(c));
            break;
        case MG_SINH_CENTRE:
            if (!(c > 0)) return MG_EINVAL;
            x[i] = L * (0.5 + std::sinh(c * (2.0 * s - 1.0)) / (2.0 * std::sinh(c)));
            break;
        case MG_EXPLICIT:
            if (!given) return MG_EINVAL;
            x[i] = given[i];
            break;
        default: return MG_EINVAL;
        }
    }
    if (kind != MG_EXPLICIT) {
        x[0] = 0.0;
        x[n] = L;
    }
    for (int i = 0; i < n; ++i)
        if (!(x[i + 1] > x[i])) return MG_EINVAL;
    return MG_OK;
}

// Section 2: W_i = 1/(dx_i dx_{i-1/2}), E_i = 1/(dx_i dx_{i+1/2}), dx_i = (x_{i+1}-x_{i-1})/2.
// With a conductivity along the axis (problem (CP) with sigma_aa = s(x_a);
// sig[k] is its value on cell k = [x_k, x_{k+1}], empty for s = 1), the
// flux form: the numerators become s_{i-1/2} and s_{i+1/2}.
void make_coefs(const std::vector<double> &x, const std::vector<double> &sig, std::vector<double> &lo,
                std::vector<double> &hi)
{
    const int n = (int)x.size() - 1;
    lo.assign(n + 1, 0.0);
    hi.assign(n + 1, 0.0);
    for (int i = 1; i < n; ++i) {
        const double hm = x[i] - x[i - 1], hp = x[i + 1] - x[i], h = 0.5 * (x[i + 1] - x[i - 1]);
        lo[i] = (sig.empty() ? 1.0 : sig[i - 1]) / (h * hm);
        hi[i] = (sig.empty() ? 1.0 : sig[i]) / (h * hp);
    }
}

// conductivity of the coarse cells: coarse cell I is fine cells 2I and 2I+1
// in series, so its conductance is theirs combined in series, length over
// the sum of length/conductivity
void coarsen_sigma(const std::vector<double> &xf, const std::vector<double> &sf, std::vector<double> &sc)
{
    sc.clear();
    if (sf.empty()) return;
    const int nc = (int)(xf.size() - 1) / 2;
    sc.resize(nc);
    for (int c = 0; c < nc; ++c) {
        const double a = xf[2 * c + 1] - xf[2 * c], b = xf[2 * c + 2] - xf[2 * c + 1];
        sc[c] = (a + b) / (a / sf[2 * c] + b / sf[2 * c + 1]);
    }
}

// ---------------------------------------------------------------------------
// Relaxation motifs (Section 3; Section 7 for 3D tweed).  A block is a
// connected set of interior points with one label; colour 0 is relaxed first.
//   tweed     : label max(i', j') (3D: the two largest of i', j', l'),
//               i' = min(i, n_x - i); red when the label (sum) is odd (even in 3D)
//               so that the corners are red.
//   wireframe : label min(i', j'); red when odd (outermost box red).
//   zebra     : lines along one axis; the first interior line is red.
// ---------------------------------------------------------------------------
enum Motif { M_TWEED = 0, M_WIREFRAME = 1, M_ZX = 3, M_ZY = 4, M_ZZ = 5 };

void motif_label(int motif, int dim, const int *n, int i, int j, int l, long long &lab, int &col)
{
    const int ip = std::min(i, n[0] - i), jp = std::min(j, n[1] - j), lp = dim == 3 ? std::min(l, n[2] - l) : 0;
    switch (motif) {
    case M_TWEED:
        if (dim == 2) {
            const int k = std::max(ip, jp);
            lab = k;
            col = (k & 1) ? 0 : 1;
        } else {
            int s[3] = {ip, jp, lp};
            std::sort(s, s + 3);
            lab = (long long)s[1] * 1000003LL + s[2];
            col = ((s[1] + s[2]) & 1) ? 1 : 0;
        }
        break;
    case M_WIREFRAME: {
        const int r = std::min(ip, jp);
        lab = r;
        col = (r & 1) ? 0 : 1;
        break;
    }
    case M_ZX:
        if (dim == 2) { lab = j; col = (j & 1) ? 0 : 1; }
        else { lab = (long long)j * 1000003LL + l; col = ((j + l) & 1) ? 1 : 0; }
        break;
    case M_ZY:
        if (dim == 2) { lab = i; col = (i & 1) ? 0 : 1; }
        else { lab = (long long)i * 1000003LL + l; col = ((i + l) & 1) ? 1 : 0; }
        break;
    case M_ZZ:
        lab = (long long)i * 1000003LL + j;
        col = ((i + j) & 1) ? 1 : 0;
        break;
    default: lab = -1; col = 0;
    }
}

struct Grid3 {
    int dim, n[3], np[3];
    long long st[3], nn;
    int layout = LAYOUT_ROW; // storage layout of the level's arrays (chunks never straddle its planes)
    // plane of node (i, j[, l]) in a split layout: as col_plane in 2D (1:
    // column-major plane), as plane3 in the 3D tweed layout
    int plane(int i, int j, int l = 0) const
    {
        if (layout == LAYOUT_ROW) return 0;
        const int ip = std::min(i, n[0] - i), jp = std::min(j, n[1] - j);
        if (layout == LAYOUT_TWEED3) {
            const int lp = std::min(l, n[2] - l);
            return (ip <= jp && ip <= lp) ? 0 : (jp <= lp ? 1 : 2);
        }
        return layout == LAYOUT_TWEED ? (ip > jp) : (layout == LAYOUT_WIREFRAME ? (ip < jp) : 1);
    }
    void coords(long long p, int &i, int &j, int &l) const
    {
        i = int(p % np[0]);
        j = int((p / np[0]) % np[1]);
        l = int(p / ((long long)np[0] * np[1]));
    }
    bool interior(int i, int j, int l) const
    {
        if (i < 1 || i > n[0] - 1 || j < 1 || j > n[1] - 1) return false;
        if (dim == 3 && (l < 1 || l > n[2] - 1)) return false;
        return true;
    }
    long long off(int d) const { return (d & 1) ? st[d >> 1] : -st[d >> 1]; }
};

struct HostBlock {
    std::vector<Chunk> ch;
    std::vector<int> succ;     // block-local successor chunk (-1 none, -2 = branch point)
    int type = BT_CHAIN, m = 0, colour = 0;
    int ends[7] = {0, 0, 0, 0, 0, 0, 0};
};

int find_root(std::vector<int> &par, int x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

// split a straight sequence of points into chunks of at most maxlen (<= CH)
// points that each lie in one plane of the level's layout and have at most
// one point per side (2D) or one point in all (3D) whose cross neighbours are
// not all kept in its plane (the addressing records hold that many
// exceptions)
void chunk_seq(const Grid3 &g, const std::vector<long long> &pts, int axdir, HostBlock &hb, int maxlen)
{
    const int n = (int)pts.size();
    const int ax = axdir >> 1, qx = ax == 0 ? 0 : 1, qy = ax == 0 ? 1 : 0;
    std::vector<int> pl(n), om(n), opp(n);
    for (int q = 0; q < n; ++q) {
        int i, j, l;
        g.coords(pts[q], i, j, l);
        pl[q] = g.plane(i, j, l);
        if (g.dim == 2) {
            om[q] = g.plane(i - qx, j - qy) != pl[q];
            opp[q] = g.plane(i + qx, j + qy) != pl[q];
        } else {
            // 3D: one count for all four cross neighbours
            int x = 0;
            for (int a = 0; a < 3; ++a) {
                if (a == ax) continue;
                for (int sg = -1; sg <= 1; sg += 2) {
                    int c[3] = {i, j, l};
                    c[a] += sg;
                    x |= g.plane(c[0], c[1], c[2]) != pl[q];
                }
            }
            om[q] = x;
            opp[q] = 0;
        }
    }
    for (int s = 0; s < n;) {
        int e = s + 1, cm = om[s], cp = opp[s];
        while (e < n && e - s < maxlen && pl[e] == pl[s] && cm + om[e] <= 1 && cp + opp[e] <= 1) {
            cm += om[e];
            cp += opp[e];
            ++e;
        }
        Chunk c;
        std::memset(&c, 0, sizeof(c));
        int i, j, l;
        g.coords(pts[s], i, j, l);
        c.c0[0] = (int16_t)i;
        c.c0[1] = (int16_t)j;
        c.c0[2] = (int16_t)l;
        c.len = (uint8_t)(e - s);
        c.axdir = (uint8_t)axdir;
        c.nextdir = (uint8_t)axdir;
        const int idx = (int)hb.ch.size();
        if (s > 0) {
            c.flags |= CF_PREV;
            c.prev = (int16_t)(idx - 1);
        }
        if (e < n) c.flags |= CF_NEXT;
        hb.ch.push_back(c);
        hb.succ.push_back(e < n ? idx + 1 : -1);
        s = e;
    }
}


// Build the block list of one motif on one level (every interior point in
// exactly one block).  Returns MG_OK or MG_EUNSUPPORTED for shapes the
// chunked solver does not handle.  maxlen: the longest chunk (CH, or less
// for the coarse-level kernel, whose lanes read their chunks' points from LDS
// directly: chunks of CH points would put the lanes of a straight run CH
// doubles apart, on the same LDS banks)
int build_blocks(const Grid3 &g, int motif, std::vector<HostBlock> &out, int maxlen = CH)
{
    const long long nn = g.nn;
    std::vector<long long> lab(nn, -1);
    std::vector<int8_t> col(nn, -1);
    for (long long p = 0; p < nn; ++p) {
        int i, j, l;
        g.coords(p, i, j, l);
        if (!g.interior(i, j, l)) continue;
        long long lb;
        int c;
        motif_label(motif, g.dim, g.n, i, j, l, lb, c);
        lab[p] = lb;
        col[p] = (int8_t)c;
    }
    std::vector<int> par(nn);
    std::iota(par.begin(), par.end(), 0);
    for (long long p = 0; p < nn; ++p) {
        if (lab[p] < 0) continue;
        for (int a = 0; a < g.dim; ++a) {
            const long long q = p + g.st[a];
            if (q < nn && lab[q] == lab[p]) {
                int i, j, l;
                g.coords(q, i, j, l);
                if (!g.interior(i, j, l)) continue;
                const int ra = find_root(par, (int)p), rb = find_root(par, (int)q);
                if (ra != rb) par[std::max(ra, rb)] = std::min(ra, rb);
            }
        }
    }
    std::vector<int> root(nn, -1);
    for (long long p = 0; p < nn; ++p)
        if (lab[p] >= 0) root[p] = find_root(par, (int)p);
    // in-block neighbour directions of every point
    std::vector<uint8_t> mask(nn, 0);
    for (long long p = 0; p < nn; ++p) {
        if (root[p] < 0) continue;
        uint8_t m = 0;
        for (int d = 0; d < 2 * g.dim; ++d) {
            const long long q = p + g.off(d);
            if (q < 0 || q >= nn || root[q] != root[p]) continue;
            int i, j, l;
            g.coords(q, i, j, l);
            if (g.interior(i, j, l)) m |= (uint8_t)(1u << d);
        }
        mask[p] = m;
    }
    // group points by component
    std::vector<int> cnt(nn + 1, 0);
    for (long long p = 0; p < nn; ++p)
        if (root[p] >= 0) cnt[root[p] + 1]++;
    for (long long p = 0; p < nn; ++p) cnt[p + 1] += cnt[p];
    std::vector<long long> pts(cnt[nn]);
    {
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (long long p = 0; p < nn; ++p)
            if (root[p] >= 0) pts[fill[root[p]]++] = p;
    }
    auto deg = [&](long long p) { return __builtin_popcount(mask[p]); };
    auto is_corner = [&](long long p) {
        const uint8_t m = mask[p];
        return __builtin_popcount(m) == 2 && !((m & 3) == 3 || (m & 12) == 12 || (m & 48) == 48);
    };
    // chunks are cut where the storage plane changes (see chunk_seq); a block
    // that would then exceed NT chunks is built without those cuts (its
    // workgroup uses the general addressing)
    Grid3 g_row = g;
    g_row.layout = LAYOUT_ROW;
    for (long long r = 0; r < nn; ++r) {
        const int b = cnt[r], e = cnt[r + 1];
        if (b == e) continue;
        const int size = e - b;
        auto build_one = [&](const Grid3 &gc, HostBlock &hb) -> int {
        hb.colour = col[pts[b]];
        long long edges2 = 0;
        int nbranch = 0;
        long long branch = -1;
        for (int k = b; k < e; ++k) {
            edges2 += deg(pts[k]);
            if (deg(pts[k]) >= 3) {
                ++nbranch;
                branch = pts[k];
            }
        }
        const long long edges = edges2 / 2;
        if (size == 1) {
            hb.type = BT_CHAIN;
            chunk_seq(gc, {pts[b]}, 1, hb, maxlen);
        } else if (edges == size - 1 && nbranch <= 1) {
            // tree: a straight line (chain), an L (spider with two legs) or a spider
            std::vector<std::vector<long long>> legs;
            std::vector<int> legdir;
            long long J = -1;
            if (nbranch == 0) {
                long long s0 = -1;
                for (int k = b; k < e; ++k)
                    if (deg(pts[k]) == 1) { s0 = pts[k]; break; }
                std::vector<long long> path{s0};
                std::vector<int> dirs;
                long long prevp = -1, cur = s0;
                while (true) {
                    long long nx = -1;
                    for (int d = 0; d < 2 * g.dim; ++d)
                        if ((mask[cur] >> d) & 1) {
                            const long long q = cur + g.off(d);
                            if (q != prevp) { nx = q; dirs.push_back(d); break; }
                        }
                    if (nx < 0) break;
                    prevp = cur;
                    cur = nx;
                    path.push_back(cur);
                }
                if ((int)path.size() != size) return MG_EUNSUPPORTED;
                std::vector<int> turns;
                for (size_t k = 1; k < dirs.size(); ++k)
                    if (dirs[k] != dirs[k - 1]) turns.push_back((int)k);
                if (turns.empty()) {
                    hb.type = BT_CHAIN;
                    chunk_seq(gc, path, dirs[0], hb, maxlen);
                } else if (turns.size() == 1) {
                    const int tj = turns[0]; // path[tj] is the turning point
                    J = path[tj];
                    legs.push_back(std::vector<long long>(path.begin(), path.begin() + tj));
                    legdir.push_back(dirs[0]);
                    std::vector<long long> other(path.rbegin(), path.rend() - tj - 1);
                    legs.push_back(other);
                    legdir.push_back(dirs.back() ^ 1);
                } else {
                    return MG_EUNSUPPORTED;
                }
            } else {
                J = branch;
                for (int d = 0; d < 2 * g.dim; ++d) {
                    if (!((mask[J] >> d) & 1)) continue;
                    std::vector<long long> walk;
                    long long cur = J + g.off(d);
                    while (true) {
                        walk.push_back(cur);
                        const uint8_t m = mask[cur];
                        if (m == (uint8_t)(1u << (d ^ 1))) break;       // tip
                        if (m != (uint8_t)((1u << d) | (1u << (d ^ 1)))) return MG_EUNSUPPORTED;
                        cur += g.off(d);
                    }
                    std::reverse(walk.begin(), walk.end());
                    legs.push_back(walk);
                    legdir.push_back(d ^ 1);
                }
            }
            if (J >= 0 && gc.layout != LAYOUT_ROW) {
                // the branch point closes leg 0's chunk sequence: take as leg 0 a
                // leg in the branch point's plane, so that no extra cut is needed
                int i, j, l;
                gc.coords(J, i, j, l);
                const int pj = gc.plane(i, j, l);
                auto leg_plane = [&](size_t lg) {
                    int a, b2, c2;
                    gc.coords(legs[lg].back(), a, b2, c2);
                    return gc.plane(a, b2, c2);
                };
                if (leg_plane(0) != pj)
                    for (size_t lg = 1; lg < legs.size(); ++lg)
                        if (leg_plane(lg) == pj) {
                            std::swap(legs[0], legs[lg]);
                            std::swap(legdir[0], legdir[lg]);
                            break;
                        }
            }
            if (J >= 0) {
                hb.type = BT_SPIDER;
                hb.m = (int)legs.size();
                if (hb.m > 7) return MG_EUNSUPPORTED;
                uint8_t jmask = 0;
                for (int lg = 1; lg < hb.m; ++lg) {
                    chunk_seq(gc, legs[lg], legdir[lg], hb, maxlen);
                    Chunk &last = hb.ch.back();
                    last.flags |= CF_NEXT | CF_NEXT_DIRECT;
                    last.nextdir = (uint8_t)legdir[lg];
                    hb.succ.back() = -2;
                    hb.ends[lg] = (int)hb.ch.size() - 1;
                    jmask |= (uint8_t)(1u << (legdir[lg] ^ 1));
                }
                std::vector<long long> l0 = legs[0];
                l0.push_back(J);
                chunk_seq(gc, l0, legdir[0], hb, maxlen);
                hb.ch.back().flags |= CF_JUNCTION;
                hb.ch.back().jmask = jmask;
            }
        } else if (edges == size && nbranch == 0) {
            // ring: split into straight sides, each ending at a corner
            long long c0 = -1;
            for (int k = b; k < e; ++k)
                if (is_corner(pts[k])) { c0 = pts[k]; break; }
            if (c0 < 0) return MG_EUNSUPPORTED;
            int d = __builtin_ctz(mask[c0]);
            std::vector<std::vector<long long>> sides;
            std::vector<int> sdir;
            std::vector<long long> cur_side;
            long long cur = c0;
            int visited = 0;
            while (true) {
                cur += g.off(d);
                cur_side.push_back(cur);
                ++visited;
                if (visited > size) return MG_EUNSUPPORTED;
                const uint8_t m = mask[cur];
                if (is_corner(cur)) {
                    sides.push_back(cur_side);
                    sdir.push_back(d);
                    cur_side.clear();
                    const int back = d ^ 1;
                    d = __builtin_ctz((uint8_t)(m & ~(1u << back)));
                    if (cur == c0) break;
                } else if (m != (uint8_t)((1u << d) | (1u << (d ^ 1)))) {
                    return MG_EUNSUPPORTED;
                }
            }
            if (visited != size) return MG_EUNSUPPORTED;
            hb.type = BT_RING;
            std::vector<int> firsts;
            for (size_t s = 0; s < sides.size(); ++s) {
                firsts.push_back((int)hb.ch.size());
                chunk_seq(gc, sides[s], sdir[s], hb, maxlen);
                Chunk &last = hb.ch.back();
                last.flags |= CF_NEXT;
                last.nextdir = (uint8_t)sdir[(s + 1) % sides.size()];
                hb.succ.back() = -3 - (int)((s + 1) % sides.size()); // patched below
            }
            const int nc = (int)hb.ch.size();
            for (size_t s = 0; s < sides.size(); ++s) {
                Chunk &f0 = hb.ch[firsts[s]];
                f0.flags |= CF_PREV;
                f0.prev = (int16_t)((firsts[s] - 1 + nc) % nc);
            }
            for (int k = 0; k < nc; ++k)
                if (hb.succ[k] <= -3) hb.succ[k] = firsts[-3 - hb.succ[k]];
        } else {
            return MG_EUNSUPPORTED;
        }
        // node roles in the reduced-system scans (block-local indices)
        {
            const int nc = (int)hb.ch.size();
            for (Chunk &c : hb.ch) {
                c.nflags = 0;
                c.ext = -1;
            }
            auto seg = [&](int a, int z) {
                hb.ch[a].nflags |= NF_HEAD;
                hb.ch[z].nflags |= NF_TAIL;
            };
            if (hb.type == BT_CHAIN) {
                seg(0, nc - 1);
            } else if (hb.type == BT_SPIDER) {
                const int J = nc - 1;
                int start = 0;
                for (int lg = 1; lg < hb.m; ++lg) {
                    seg(start, hb.ends[lg]);
                    hb.ch[hb.ends[lg]].nflags |= NF_EXTJ;
                    hb.ch[hb.ends[lg]].ext = (int16_t)J;
                    start = hb.ends[lg] + 1;
                }
                if (start < J) {
                    seg(start, J - 1);
                    hb.ch[J - 1].nflags |= NF_EXTJ;
                    hb.ch[J - 1].ext = (int16_t)J;
                }
                hb.ch[J].nflags |= NF_HEAD | NF_TAIL | NF_J;
            } else {
                const int B = nc - 1;
                seg(0, B - 1);
                for (int q = 0; q < B; ++q) {
                    hb.ch[q].nflags |= NF_RING;
                    hb.ch[q].ext = (int16_t)B;
                }
                hb.ch[B].nflags |= NF_HEAD | NF_TAIL | NF_B;
            }
        }
        // successor links: direct when the successor chunk has no interior
        for (size_t k = 0; k < hb.ch.size(); ++k) {
            const int sc = hb.succ[k];
            if (sc >= 0 && hb.ch[sc].len == 1) hb.ch[k].flags |= CF_NEXT_DIRECT;
        }
        return MG_OK;
        };
        HostBlock hb;
        int rc = build_one(g, hb);
        if (rc == MG_OK && (int)hb.ch.size() > NT && g.layout != LAYOUT_ROW) {
            hb = HostBlock();
            rc = build_one(g_row, hb);
        }
        if (rc) return rc;
        if ((int)hb.ch.size() > NT) return MG_EUNSUPPORTED;
        out.push_back(std::move(hb));
    }
    return MG_OK;
}

// Pack the blocks of one colour into workgroups (largest blocks first so the
// longest reduced solves start early).
struct HostTable {
    std::vector<Chunk> chunks;
    std::vector<ChunkAddr> addrs;   // 2D: addressing records in the level's layout
    std::vector<ChunkAddr3> addrs3; // 3D: addressing records in the level's layout
    std::vector<Block> blocks;
    std::vector<WGDesc> wgs;  // the first nbig need NT lanes, the rest nts
    int nbig = 0;
    int nts = NT / 2;         // lanes of the small workgroups (64, 128 or NT/2)
};

// Pack the blocks of one colour.  narrow: the small workgroups may be
// narrower than NT/2 lanes (64 or 128, the narrowest that holds the largest
// small block): more, shorter workgroups for levels whose sweeps are bound by
// a workgroup's latency rather than by bandwidth.
void pack(std::vector<const HostBlock *> bl, HostTable &t, bool narrow = false)
{
    std::stable_sort(bl.begin(), bl.end(),
                     [](const HostBlock *a, const HostBlock *b) { return a->ch.size() > b->ch.size(); });
    // blocks of more than NT/2 chunks get a full NT-lane workgroup each; the
    // rest are packed into NT/2-lane workgroups by best fit in decreasing
    // size: each block goes to the open workgroup with the least room that
    // still holds it, so the small blocks fill the room the large ones leave
    // (fewer, fuller workgroups: a half-empty workgroup holds a CU slot as
    // long as a full one)
    int maxsmall = 1;
    for (const HostBlock *hb : bl)
        if ((int)hb->ch.size() <= NT / 2) maxsmall = std::max(maxsmall, (int)hb->ch.size());
    t.nts = NT / 2;
    if (narrow)
        while (t.nts > 64 && maxsmall <= t.nts / 2) t.nts /= 2;
    for (int pass = 0; pass < 2; ++pass) {
        const int cap = pass == 0 ? NT : t.nts;
        const size_t w0 = t.wgs.size();
        std::vector<std::vector<const HostBlock *>> groups;
        std::multimap<int, int> room; // free chunks -> group (groups with a free block slot)
        for (const HostBlock *hb : bl) {
            const int nc = (int)hb->ch.size();
            if ((pass == 0) != (nc > NT / 2)) continue;
            int g = -1;
            if (pass == 1) {
                auto it = room.lower_bound(nc);
                if (it != room.end()) {
                    g = it->second;
                    const int left = it->first - nc;
                    room.erase(it);
                    if ((int)groups[g].size() + 1 < cap && left > 0) room.emplace(left, g);
                }
            }
            if (g < 0) {
                g = (int)groups.size();
                groups.emplace_back();
                if (pass == 1 && cap - nc > 0) room.emplace(cap - nc, g);
            }
            groups[g].push_back(hb);
        }
        for (const auto &grp : groups) {
            WGDesc cur{(int)t.chunks.size(), 0, (int)t.blocks.size(), 0};
            for (const HostBlock *hb : grp) {
                const int nc = (int)hb->ch.size();
                const int o = cur.nchunk;
                for (Chunk c : hb->ch) {
                    if (c.flags & CF_PREV) c.prev = (int16_t)(c.prev + o);
                    if (c.ext >= 0) c.ext = (int16_t)(c.ext + o);
                    t.chunks.push_back(c);
                }
                Block bk;
                std::memset(&bk, 0, sizeof(bk));
                bk.first = (int16_t)o;
                bk.count = (int16_t)nc;
                bk.type = (uint8_t)hb->type;
                bk.m = (uint8_t)hb->m;
                for (int k = 0; k < 7; ++k) bk.ends[k] = (int16_t)(hb->ends[k] + o);
                t.blocks.push_back(bk);
                cur.nchunk += nc;
                cur.nblock += 1;
            }
            t.wgs.push_back(cur);
        }
        if (pass == 0) t.nbig = (int)t.wgs.size();
        // Workgroups are handed to the 8 XCDs round-robin in index order.
        // Number them so that consecutive entries of the list (blocks of
        // neighbouring labels, which read the same cache lines) share an XCD
        // and its L2: entry w goes to XCD w/ceil(size/8), so each XCD works
        // through one contiguous eighth of the list (groups of 256 entries
        // per XCD round were 0.4% slower at 4097^2).
        {
            const int n = (int)(t.wgs.size() - w0), G = n > 0 ? n : 1;
            std::vector<WGDesc> out(n);
            for (int g0 = 0; g0 < n; g0 += G) {
                const int s = std::min(G, n - g0), q = (s + 7) / 8;
                std::vector<std::pair<int, int>> key(s);
                for (int w = 0; w < s; ++w) key[w] = {(w % q) * 8 + w / q, w};
                std::sort(key.begin(), key.end());
                for (int r = 0; r < s; ++r) out[g0 + r] = t.wgs[w0 + g0 + key[r].second];
            }
            std::copy(out.begin(), out.end(), t.wgs.begin() + w0);
        }
    }
}

// Bounds check of a table against its grid before it is uploaded: every
// chunk point and every in-block neighbour it names is an interior node, and
// every workgroup-local index stays inside its workgroup.
bool validate(const Grid3 &g, const HostTable &t)
{
    const int nc = (int)t.chunks.size(), nb = (int)t.blocks.size();
    for (size_t wi = 0; wi < t.wgs.size(); ++wi) {
        const WGDesc &w = t.wgs[wi];
        const int cap = ((int)wi < t.nbig) ? NT : t.nts;
        if (w.chunk0 < 0 || w.nchunk < 1 || w.nchunk > cap || w.chunk0 + w.nchunk > nc) return false;
        if (w.block0 < 0 || w.nblock < 1 || w.nblock > cap || w.block0 + w.nblock > nb) return false;
        for (int k = 0; k < w.nchunk; ++k) {
            const Chunk &c = t.chunks[w.chunk0 + k];
            if (c.len < 1 || c.len > CH || c.axdir >= 2 * g.dim || c.nextdir >= 2 * g.dim) return false;
            if ((c.flags & CF_PREV) && (c.prev < 0 || c.prev >= w.nchunk)) return false;
            if (c.ext < -1 || c.ext >= w.nchunk) return false;
            if ((c.nflags & (NF_EXTJ | NF_RING)) && c.ext < 0) return false;
            const int ax = c.axdir >> 1, sg = (c.axdir & 1) ? 1 : -1;
            int p[3] = {c.c0[0], c.c0[1], g.dim == 3 ? c.c0[2] : 0};
            p[ax] -= sg;
            for (int q = 0; q <= c.len; ++q) {
                // q = 0 is the predecessor position (interior, or the boundary node a tip faces)
                if (q > 0 && !g.interior(p[0], p[1], p[2])) return false;
                for (int a = 0; a < g.dim; ++a)
                    if (p[a] < 0 || p[a] > g.n[a]) return false;
                if (q < c.len) p[ax] += sg;
            }
            // p is now the last point
            if (c.flags & CF_NEXT) {
                int s[3] = {p[0], p[1], p[2]};
                s[c.nextdir >> 1] += (c.nextdir & 1) ? 1 : -1;
                if (!g.interior(s[0], s[1], s[2])) return false;
            }
            if (c.flags & CF_JUNCTION)
                for (int d = 0; d < 2 * g.dim; ++d)
                    if ((c.jmask >> d) & 1) {
                        int s[3] = {p[0], p[1], p[2]};
                        s[d >> 1] += (d & 1) ? 1 : -1;
                        if (!g.interior(s[0], s[1], s[2])) return false;
                    }
        }
        for (int k = 0; k < w.nblock; ++k) {
            const Block &b = t.blocks[w.block0 + k];
            if (b.first < 0 || b.count < 1 || b.first + b.count > w.nchunk || b.type > BT_RING || b.m > 7) return false;
            if (b.type == BT_SPIDER)
                for (int l = 1; l < b.m; ++l)
                    if (b.ends[l] < b.first || b.ends[l] >= b.first + b.count - 1) return false;
            if (b.type == BT_RING && b.count < 3) return false;
        }
    }
    return true;
}

// Factor the reduced systems of one table (geometry only).  Phase 1 of the
// sweep is run on the host without data to obtain each node's reduced row,
// then every segment is eliminated once; the kernel only substitutes.
template <int DIM>
void factor_table(const Dims &d, const Coef<double> &c, const HostTable &t, std::vector<NodeFac<double>> &fac)
{
    fac.assign(t.chunks.size(), NodeFac<double>{0, 0, 0, 0});
    std::vector<double> low(NT), ds(NT), rs(NT), dn(NT), up(NT), rn(NT), xx(NT), aux(NT);
    RedArrays<double> r{low.data(), ds.data(), rs.data(), dn.data(), up.data(), rn.data(), xx.data(), aux.data()};
    LaneState<double> st;
    for (const WGDesc &w : t.wgs) {
        std::fill(low.begin(), low.end(), 0.0);
        std::fill(ds.begin(), ds.end(), 0.0);
        std::fill(dn.begin(), dn.end(), 0.0);
        std::fill(up.begin(), up.end(), 0.0);
        std::fill(aux.begin(), aux.end(), 0.0);
        const Chunk *ch = &t.chunks[w.chunk0];
        NodeFac<double> *F = &fac[w.chunk0];
        for (int q = 0; q < w.nchunk; ++q) sweep_phase1<double, DIM, true, false>(d, c, [](int) { return 0.0; }, 0.0, ch[q], q, r, st);
        std::vector<double> dg(w.nchunk);
        for (int q = 0; q < w.nchunk; ++q) dg[q] = ds[q] + dn[q];
        auto segment = [&](int a, int z, bool open_tail) {
            double g = 0;
            for (int q = a; q <= z; ++q) {
                const double lo = (q == a) ? 0.0 : low[q];
                const double u = (q == z && open_tail) ? 0.0 : up[q];
                const double inv = 1.0 / (dg[q] - lo * g);
                F[q].alpha = -lo * inv;
                F[q].inv = inv;
                F[q].gam = u * inv;
                g = F[q].gam;
            }
        };
        for (int k = 0; k < w.nblock; ++k) {
            const Block &bk = t.blocks[w.block0 + k];
            const int s = bk.first, e = s + bk.count;
            if (bk.type == BT_CHAIN) {
                segment(s, e - 1, false);
            } else if (bk.type == BT_SPIDER) {
                const int J = e - 1;
                int start = s;
                double den = dg[J];
                for (int l = 1; l < bk.m; ++l) {
                    const int end = bk.ends[l];
                    segment(start, end, false);
                    F[end].z = aux[end];
                    den -= aux[end] * F[end].gam;
                    start = end + 1;
                }
                const bool leg0 = ch[J].flags & CF_PREV;
                if (leg0) {
                    segment(start, J - 1, false);
                    den -= low[J] * F[J - 1].gam;
                }
                F[J] = NodeFac<double>{0.0, 1.0 / den, leg0 ? low[J] : 0.0, 0.0};
            } else {
                const int B = e - 1;
                segment(s, B - 1, true);
                // border column of the open part: low at its head, up at its tail
                std::vector<double> dz(B - s), z(B - s);
                for (int q = s; q < B; ++q) {
                    const double col = (q == s ? low[s] : 0.0) + (q == B - 1 ? up[B - 1] : 0.0);
                    dz[q - s] = (q == s ? 0.0 : F[q].alpha * dz[q - s - 1]) + col * F[q].inv;
                }
                for (int q = B - 1; q >= s; --q) z[q - s] = dz[q - s] - (q == B - 1 ? 0.0 : F[q].gam * z[q - s + 1]);
                for (int q = s; q < B; ++q) F[q].z = z[q - s];
                const double inv = 1.0 / (dg[B] - low[B] * z[B - 1 - s] - up[B] * z[0]);
                F[B] = NodeFac<double>{low[B], inv, up[B], 0.0};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
struct DevPool {
    std::vector<void *> owned;
    bool host_only = false; // build host-side structures only (test hook, no device calls)
    ~DevPool()
    {
        for (void *p : owned) (void)hipFree(p);
    }
    template <typename T> T *upload(const std::vector<T> &v, int &err)
    {
        if (v.empty() || host_only) return nullptr;
        void *p = nullptr;
        if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) {
            err = MG_ENOMEM;
            return nullptr;
        }
        owned.push_back(p);
        if (hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) err = MG_EHIP;
        return (T *)p;
    }
};

struct Level {
    Dims d;
    Grid3 g;
    std::vector<double> x[3], lo[3], hi[3];
    std::vector<double> sig[3]; // conductivity per cell along each axis (empty: 1)
    Coef<double> c64[2];  // [forward, transposed]
    Coef<float> c32[2];
    SweepTable tab[MAXSLOT][2]; // [motif slot][colour]
    HostTable htab[MAXSLOT][2]; // host copies (validation and the host emulation hook)
    std::vector<NodeFac<double>> hfac[MAXSLOT][2][2]; // [slot][colour][forward/transposed]
    long long cs = 0;                 // entries per coefficient array
    std::vector<double> hblk[2];      // host coefficient blocks [forward, transposed] (layout of Coef)
    Coef<double> hc64[2];
    double *u = nullptr, *f = nullptr;   // FP64 work arrays (levels >= 1, and level 0 when its layout is split)
    float *u32 = nullptr, *f32 = nullptr; // FP32 work arrays (all levels)
};

} // namespace

struct mg_handle {
    mg_grid grid;
    mg_options opt;
    hipStream_t stream = nullptr;
    SideStream side;          // overlaps big-block launches with the rest of a half-sweep
    // One step of the solve loop (a cycle, or a refinement step, with the
    // defect norm after it) captured as a HIP graph and replayed: one launch
    // per step instead of one per kernel.  A capture is valid for its arrays,
    // direction and precision while gen is unchanged; gen moves whenever the
    // options, the workspace or the coarse-level images change.
    struct {
        bool enabled = true;
        bool broken = false; // a capture failed: the solves stay eager
        hipStream_t cap = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        const void *u = nullptr, *f = nullptr;
        int adj = -1, prec = -1;
        unsigned gen = 0;
    } step;
    unsigned gen = 1;
    int nlev = 0;
    Level lev[MAXLEV];
    int slot_motif[MAXSLOT] = {-1, -1, -1};
    bool checker = false;
    int nunk_coarse = 0;
    double *cinv64[2] = {nullptr, nullptr};
    float *cinv32[2] = {nullptr, nullptr};
    double *partial = nullptr, *normv = nullptr;
    double *h_norm = nullptr;  // pinned
    DevPool pool;
    size_t ws_bytes = 0;
    char *ws = nullptr;
    char *dscr = nullptr; // 3D split levels: defect scratch of the restriction (one fine array, FP64 or FP32)
    bool ws_owned = false;
    // coarse-level kernel: levels tail_lv .. nlev-1 run in one workgroup per
    // problem; one launch runs tail_reps visits of their sub-cycle
    int tail_lv = -1;
    int tail_reps = 1;
    void *tail_img[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}}; // [FP64, FP32][forward, transposed]
    TailPlan<double> tail64[2];
    TailPlan<float> tail32[2];
    int tail_key[4] = {-1, -1, -1, -1}; // checker, nu1, nu2, gamma the images were built for
    int tail_map_lv[2] = {-1, -1}; // [FP64, FP32] level whose sub-cycle the coarse-level kernel applies as a map
    void *tail_map[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}}; // [FP64, FP32][forward, transposed]
};

namespace {

#define HIPCHK(x)                                                                                                     \
    do {                                                                                                              \
        if ((x) != hipSuccess) return MG_EHIP;                                                                        \
    } while (0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t workspace_layout(mg_handle *h, bool assign)
{
    size_t off = 0;
    const int B = h->grid.batch;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int l = 0; l < h->nlev; ++l) {
        Level &L = h->lev[l];
        const size_t n = (size_t)L.d.bs * B;
        // level 0 works in the caller's arrays unless its layout is split
        const bool own = l > 0 || L.d.layout != LAYOUT_ROW;
        size_t ou = 0, of = 0;
        if (own) {
            ou = take(n * sizeof(double));
            of = take(n * sizeof(double));
        }
        const size_t ou32 = take(n * sizeof(float)), of32 = take(n * sizeof(float));
        if (assign) {
            L.u = own ? (double *)(h->ws + ou) : nullptr;
            L.f = own ? (double *)(h->ws + of) : nullptr;
            L.u32 = (float *)(h->ws + ou32);
            L.f32 = (float *)(h->ws + of32);
        }
    }
    // the restriction from a 3D split level runs in two passes through a
    // defect array of that level
    size_t dmax = 0;
    for (int l = 0; l + 1 < h->nlev; ++l)
        if (h->lev[l].d.layout == LAYOUT_TWEED3) dmax = std::max(dmax, (size_t)h->lev[l].d.bs * B * sizeof(double));
    if (dmax) {
        const size_t od = take(dmax);
        if (assign) h->dscr = h->ws + od;
    }
    return off;
}

int clear_workspace(mg_handle *h)
{
    // coarse arrays start at zero: their boundary entries are never written
    for (int l = 0; l < h->nlev; ++l) {
        Level &L = h->lev[l];
        const long long n = L.d.bs * h->grid.batch;
        if (L.u) {
            HIPCHK(launch_fill<double>(L.u, n, 0.0, h->stream));
            HIPCHK(launch_fill<double>(L.f, n, 0.0, h->stream));
        }
        HIPCHK(launch_fill<float>(L.u32, n, 0.0f, h->stream));
        HIPCHK(launch_fill<float>(L.f32, n, 0.0f, h->stream));
    }
    return MG_OK;
}

int ensure_workspace(mg_handle *h)
{
    if (h->ws) return MG_OK;
    void *p = nullptr;
    if (hipMalloc(&p, h->ws_bytes) != hipSuccess) return MG_ENOMEM;
    h->ws = (char *)p;
    h->ws_owned = true;
    ++h->gen;
    workspace_layout(h, true);
    return clear_workspace(h);
}

// dense inverse of the coarsest interior operator (Gauss-Jordan, partial pivoting)
bool invert(std::vector<double> &A, int n, std::vector<double> &inv)
{
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)piv * n + k])) piv = i;
        if (A[(size_t)piv * n + k] == 0.0) return false;
        if (piv != k)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
                std::swap(inv[(size_t)k * n + j], inv[(size_t)piv * n + j]);
            }
        const double dinv = 1.0 / A[(size_t)k * n + k];
        for (int j = 0; j < n; ++j) {
            A[(size_t)k * n + j] *= dinv;
            inv[(size_t)k * n + j] *= dinv;
        }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double fct = A[(size_t)i * n + k];
            if (fct == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)i * n + j] -= fct * A[(size_t)k * n + j];
                inv[(size_t)i * n + j] -= fct * inv[(size_t)k * n + j];
            }
        }
    }
    return true;
}

int motif_slots(int smoother, int dim, int *m, bool *checker)
{
    for (int s = 0; s < MAXSLOT; ++s) m[s] = -1;
    *checker = false;
    switch (smoother) {
    case MG_TWEED: m[0] = M_TWEED; break;
    case MG_WIREFRAME:
        if (dim != 2) return MG_EUNSUPPORTED;
        m[0] = M_WIREFRAME;
        break;
    case MG_CHECKERBOARD: *checker = true; break;
    case MG_ZEBRA_X: m[0] = M_ZX; break;
    case MG_ZEBRA_Y: m[0] = M_ZY; break;
    case MG_ZEBRA_Z:
        if (dim != 3) return MG_EINVAL;
        m[0] = M_ZZ;
        break;
    case MG_ADZ:
        // a zebra sweep along each axis in turn (Section 7's 3D comparison
        // scheme takes the third, along z)
        m[0] = M_ZX;
        m[1] = M_ZY;
        if (dim == 3) m[2] = M_ZZ;
        break;
    case MG_ALT_TW:
        if (dim != 2) return MG_EUNSUPPORTED;
        m[0] = M_TWEED;
        m[1] = M_WIREFRAME;
        break;
    default: return MG_EINVAL;
    }
    return MG_OK;
}

// number of sweeps (motif slots) in one relaxation
int nslots(const mg_handle *h)
{
    int ns = 0;
    while (ns < MAXSLOT && h->slot_motif[ns] >= 0) ++ns;
    return ns;
}

// ---------------------------------------------------------------------------
// coarse-level kernel set-up.  The kernel takes the longest run of coarsest
// levels (at least two) whose LDS image (level descriptors, coefficients, block
// tables, operation list) plus u, f and the coarsest solve's scratch fit in
// TAIL_BYTES, and whose blocks fit its workgroup.  The operation list depends
// on the cycle options, so the images are rebuilt when those change.
// TWMG_NO_TAIL=1 keeps every level on the per-level kernels.
// ---------------------------------------------------------------------------
void tail_ops_rec(const mg_handle *h, int lt, int lv, int adj, int map_lv, std::vector<TailOp> &ops)
{
    const uint8_t rel = (uint8_t)(lv - lt);
    if (lv == h->nlev - 1) {
        ops.push_back(TailOp{TO_SOLVE, rel, 0, 0});
        return;
    }
    if (lv == map_lv) {
        ops.push_back(TailOp{TO_MAP, rel, 0, 0});
        return;
    }
    auto relax = [&]() {
        if (h->checker) {
            for (int k = 0; k < 2; ++k) ops.push_back(TailOp{TO_CHECKER, rel, 0, (uint8_t)(adj ? 1 - k : k)});
            return;
        }
        const int ns = nslots(h);
        for (int k = 0; k < ns; ++k) {
            const int sl = adj ? ns - 1 - k : k;
            for (int q = 0; q < 2; ++q) ops.push_back(TailOp{TO_SWEEP, rel, (uint8_t)sl, (uint8_t)(adj ? 1 - q : q)});
        }
    };
    for (int k = 0; k < h->opt.nu1; ++k) relax();
    ops.push_back(TailOp{TO_RESTRICT, rel, 0, 0});
    for (int g = 0; g < h->opt.gamma; ++g) tail_ops_rec(h, lt, lv + 1, adj, map_lv, ops);
    ops.push_back(TailOp{TO_PROLONG, rel, 0, 0});
    for (int k = 0; k < h->opt.nu2; ++k) relax();
}

struct ImageBuf {
    std::vector<unsigned char> b;
    int put(const void *p, size_t n)
    {
        const size_t o = (b.size() + 15) & ~size_t(15);
        b.resize(o + n);
        if (n) std::memcpy(&b[o], p, n);
        return (int)o;
    }
};

size_t align16(size_t n) { return (n + 15) & ~size_t(15); }

// Builds the LDS image of levels lt .. nlev-1 for type T and direction adj;
// returns the LDS bytes the kernel needs (image + u, f + scratch).
template <typename T>
size_t tail_image(const mg_handle *h, int lt, int adj, std::vector<unsigned char> &img, TailPlan<T> &plan,
                  int reps = 1)
{
    const int nt = h->nlev - lt, dim = h->grid.dim;
    std::vector<TailOp> ops;
    // reps sub-cycles in a row from the same right-hand side (the gamma
    // visits of a W-cycle, in one launch)
    for (int r = 0; r < reps; ++r) tail_ops_rec(h, lt, lt, adj, h->tail_map_lv[sizeof(T) == 8 ? 0 : 1], ops);
    ImageBuf I;
    std::vector<TailLevel> tl(nt);
    std::memset(tl.data(), 0, tl.size() * sizeof(TailLevel));
    plan.lev_off = I.put(tl.data(), tl.size() * sizeof(TailLevel));
    plan.ops_off = I.put(ops.data(), ops.size() * sizeof(TailOp));
    plan.nops = (int)ops.size();
    for (int r = 0; r < nt; ++r) {
        const Level &L = h->lev[lt + r];
        TailLevel &t = tl[r];
        t.d = L.d;
        {
            const std::vector<T> vt(L.hblk[adj].begin(), L.hblk[adj].end());
            t.co = I.put(vt.data(), vt.size() * sizeof(T));
            t.cs = (int)L.cs;
        }
        if (lt + r == h->nlev - 1) continue;
        t.short_chunks = 1;
        for (int sl = 0; sl < MAXSLOT; ++sl)
            for (int c = 0; c < 2; ++c)
                if (h->slot_motif[sl] >= 0)
                    for (const Chunk &ch : L.htab[sl][c].chunks)
                        if (ch.len > TAIL_SHORT_CH) t.short_chunks = 0;
        for (int sl = 0; sl < MAXSLOT; ++sl)
            for (int c = 0; c < 2; ++c) {
                if (h->slot_motif[sl] < 0) continue;
                const HostTable &ht = L.htab[sl][c];
                const std::vector<NodeFac<double>> &f64 = L.hfac[sl][c][adj];
                std::vector<NodeFac<T>> fv(f64.size());
                for (size_t q = 0; q < f64.size(); ++q)
                    fv[q] = NodeFac<T>{(T)f64[q].alpha, (T)f64[q].inv, (T)f64[q].gam, (T)f64[q].z};
                t.chunk_off[sl][c] = I.put(ht.chunks.data(), ht.chunks.size() * sizeof(Chunk));
                t.block_off[sl][c] = I.put(ht.blocks.data(), ht.blocks.size() * sizeof(Block));
                t.wg_off[sl][c] = I.put(ht.wgs.data(), ht.wgs.size() * sizeof(WGDesc));
                t.fac_off[sl][c] = I.put(fv.data(), fv.size() * sizeof(NodeFac<T>));
                t.nwg[sl][c] = (int)ht.wgs.size();
                for (const Block &bk : ht.blocks)
                    if (bk.type == BT_RING) t.rings[sl][c] = 1;
                t.onewave[sl][c] = 1;
                for (const WGDesc &w : ht.wgs)
                    if (w.nchunk > 64 || w.nblock > 64) t.onewave[sl][c] = 0;
            }
    }
    size_t off = align16(I.b.size());
    plan.image_bytes = (int)off;
    for (int r = 0; r < nt; ++r) {
        const size_t nb = align16((size_t)h->lev[lt + r].d.nn * sizeof(T));
        tl[r].uoff = (int)off;
        off += nb;
        tl[r].foff = (int)off;
        off += nb;
    }
    plan.rhs_off = (int)off;
    off += align16((size_t)h->nunk_coarse * sizeof(T));
    std::memcpy(&I.b[plan.lev_off], tl.data(), tl.size() * sizeof(TailLevel));
    I.b.resize(plan.image_bytes, 0);
    img.swap(I.b);
    plan.nunk = h->nunk_coarse;
    plan.dim = dim;
    plan.nn0 = h->lev[lt].d.nn;
    return off;
}

void free_tail(mg_handle *h)
{
    for (auto &row : h->tail_img)
        for (void *&p : row) {
            if (p) (void)hipFree(p);
            p = nullptr;
        }
    for (auto &row : h->tail_map)
        for (void *&p : row) {
            if (p) (void)hipFree(p);
            p = nullptr;
        }
    h->tail_lv = -1;
    h->tail_reps = 1;
    ++h->gen;
    h->tail_map_lv[0] = h->tail_map_lv[1] = -1;
}

// The sub-cycle of level lm (zero boundary values, nu <= TAIL_MAP_MAX
// interior unknowns) is linear in the level's u and f: it is computed once by
// the coarse-level kernel itself, started at lm, on the 2 nu unit vectors as a
// batch, and stored input-major for TailPlan::map.  lm's operations must be
// the plain ones (tail_map_lv < 0 for T) while this runs.
template <typename T> int build_tail_map(mg_handle *h, int lm, int adj, void **out)
{
    const Level &L = h->lev[lm];
    const Dims &d = L.d;
    const int nx = d.n[0] - 1, ny = d.n[1] - 1, nz = d.dim == 3 ? d.n[2] - 1 : 1;
    const int nu = nx * ny * nz, nb = 2 * nu;
    const long long nn = d.nn;
    auto node = [&](int k) {
        return (long long)(1 + k % nx) + (long long)(1 + (k / nx) % ny) * d.st[1] +
               (d.dim == 3 ? (long long)(1 + k / (nx * ny)) * d.st[2] : 0);
    };
    std::vector<unsigned char> img;
    TailPlan<T> p;
    tail_image<T>(h, lm, adj, img, p);
    std::vector<T> hu((size_t)nb * nn, T(0)), hf((size_t)nb * nn, T(0));
    for (int k = 0; k < nu; ++k) {
        hu[(size_t)k * nn + node(k)] = T(1);
        hf[(size_t)(nu + k) * nn + node(k)] = T(1);
    }
    void *dimg = nullptr, *du = nullptr, *df = nullptr;
    int rc = MG_OK;
    if (hipMalloc(&dimg, img.size()) != hipSuccess || hipMalloc(&du, hu.size() * sizeof(T)) != hipSuccess ||
        hipMalloc(&df, hf.size() * sizeof(T)) != hipSuccess)
        rc = MG_ENOMEM;
    if (!rc && (hipMemcpy(dimg, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(du, hu.data(), hu.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(df, hf.data(), hf.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess))
        rc = MG_EHIP;
    if (!rc) {
        p.image = (const unsigned char *)dimg;
        if constexpr (sizeof(T) == 8) p.ainv = h->cinv64[adj];
        else p.ainv = h->cinv32[adj];
        if (launch_tail_cycle<T>(p, (T *)du, (const T *)df, nb, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess ||
            hipMemcpy(hu.data(), du, hu.size() * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
            rc = MG_EHIP;
    }
    if (dimg) (void)hipFree(dimg);
    if (du) (void)hipFree(du);
    if (df) (void)hipFree(df);
    if (rc) return rc;
    std::vector<T> m((size_t)nb * nu);
    for (int k = 0; k < nb; ++k)
        for (int i = 0; i < nu; ++i) m[(size_t)k * nu + i] = hu[(size_t)k * nn + node(i)];
    if (hipMalloc(out, m.size() * sizeof(T)) != hipSuccess) return MG_ENOMEM;
    if (hipMemcpy(*out, m.data(), m.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return MG_EHIP;
    return MG_OK;
}

int build_tail(mg_handle *h)
{
    if (h->pool.host_only) return MG_OK;
    const int key[4] = {h->checker ? 1 : 0, h->opt.nu1, h->opt.nu2, h->opt.gamma};
    if (std::equal(key, key + 4, h->tail_key)) return MG_OK;
    if (h->stream) HIPCHK(hipStreamSynchronize(h->stream));
    free_tail(h);
    std::copy(key, key + 4, h->tail_key);
    const char *env = std::getenv("TWMG_NO_TAIL");
    if (env && env[0] == '1') return MG_OK;
    const int nl = h->nlev;
    int lt = -1;
    for (int l = nl - 2; l >= 0; --l) {
        bool fits = h->lev[l].d.layout == LAYOUT_ROW;
        for (int sl = 0; sl < MAXSLOT; ++sl)
            for (int c = 0; c < 2; ++c)
                fits = fits && h->lev[l].tab[sl][c].nwg_big == 0 && h->lev[l].tab[sl][c].nts == NT / 2;
        std::vector<unsigned char> img;
        TailPlan<double> p;
        if (!fits || tail_image<double>(h, l, 0, img, p) > (size_t)TAIL_BYTES) break;
        lt = l;
    }
    if (lt < 0) return MG_OK;
    // the largest level below the finest (zero boundary values) and above the
    // coarsest with at most TAIL_MAP_MAX unknowns runs its sub-cycle as a map
    // (one map per precision, each computed by that precision's kernel)
    const char *envm = std::getenv("TWMG_NO_TAIL_MAP");
    auto unknowns = [&](int l) {
        long long nu = 1;
        for (int a = 0; a < h->grid.dim; ++a) nu *= h->lev[l].d.n[a] - 1;
        return nu;
    };
    int lm[2] = {-1, -1};
    for (int k = 0; k < 2; ++k) {
        if (envm && envm[0] == '1') break;
        for (int l = nl - 2; l >= std::max(lt, 1); --l) {
            if (unknowns(l) > TAIL_MAP_MAX) break;
            lm[k] = l;
        }
    }
    for (int adj = 0; adj < 2; ++adj) {
        int rc = MG_OK;
        if (lm[0] >= 0) rc = build_tail_map<double>(h, lm[0], adj, &h->tail_map[0][adj]);
        if (!rc && lm[1] >= 0) rc = build_tail_map<float>(h, lm[1], adj, &h->tail_map[1][adj]);
        if (rc) return rc;
    }
    h->tail_map_lv[0] = lm[0];
    h->tail_map_lv[1] = lm[1];
    // entered from a finer level, the kernel runs that level's gamma visits
    // of its sub-cycle in one launch (the first leaves u in LDS for the next)
    // (if the longer operation list still fits the LDS budget)
    int reps = lt > 0 ? std::max(h->opt.gamma, 1) : 1;
    if (reps > 1) {
        std::vector<unsigned char> img;
        TailPlan<double> p;
        if (tail_image<double>(h, lt, 0, img, p, reps) > (size_t)TAIL_BYTES) reps = 1;
    }
    for (int adj = 0; adj < 2; ++adj) {
        std::vector<unsigned char> i64, i32;
        tail_image<double>(h, lt, adj, i64, h->tail64[adj], reps);
        tail_image<float>(h, lt, adj, i32, h->tail32[adj], reps);
        if (lm[0] >= 0) {
            h->tail64[adj].map = (const double *)h->tail_map[0][adj];
            h->tail64[adj].map_nu = (int)unknowns(lm[0]);
        }
        if (lm[1] >= 0) {
            h->tail32[adj].map = (const float *)h->tail_map[1][adj];
            h->tail32[adj].map_nu = (int)unknowns(lm[1]);
        }
        const std::vector<unsigned char> *src[2] = {&i64, &i32};
        for (int k = 0; k < 2; ++k) {
            void *p = nullptr;
            if (hipMalloc(&p, src[k]->size()) != hipSuccess) return MG_ENOMEM;
            h->tail_img[k][adj] = p;
            HIPCHK(hipMemcpy(p, src[k]->data(), src[k]->size(), hipMemcpyHostToDevice));
        }
        h->tail64[adj].image = (const unsigned char *)h->tail_img[0][adj];
        h->tail32[adj].image = (const unsigned char *)h->tail_img[1][adj];
    }
    h->tail_lv = lt;
    h->tail_reps = reps;
    return MG_OK;
}

int setup_impl(mg_handle *h, const mg_grid *grid, const mg_stretching *st, const mg_options *opt)
{
    if (grid->dim != 2 && grid->dim != 3) return MG_EINVAL;
    if (grid->batch < 1) return MG_EINVAL;
    for (int a = 0; a < grid->dim; ++a) {
        if (grid->n[a] < 2 || grid->n[a] % 2 || grid->n[a] > 32000) return MG_EINVAL;
        if (!(grid->L[a] > 0)) return MG_EINVAL;
    }
    if (opt->nu1 < 0 || opt->nu2 < 0 || opt->gamma < 1 || opt->gamma > 2 || opt->max_cycles < 1) return MG_EINVAL;
    if (opt->precision != MG_FP64 && opt->precision != MG_FP32_IR) return MG_EINVAL;
    h->grid = *grid;
    h->opt = *opt;
    int rc = motif_slots(opt->smoother, grid->dim, h->slot_motif, &h->checker);
    if (rc) return rc;
    const int dim = grid->dim;
    // finest coordinates
    std::vector<double> x0[3];
    for (int a = 0; a < dim; ++a) {
        rc = make_coords(st->kind[a], st->param[a], grid->n[a], grid->L[a], st->coords[a], x0[a]);
        if (rc) return rc;
        if (st->sigma[a])
            for (int k = 0; k < grid->n[a]; ++k)
                if (!(st->sigma[a][k] > 0) || std::isinf(st->sigma[a][k])) return MG_EINVAL;
    }
    // hierarchy (Section 4): coarse nodes are every other fine node; stop when an
    // axis has an odd number of cells or only two
    int cur[3] = {grid->n[0], grid->n[1], dim == 3 ? grid->n[2] : 0};
    int nl = 0;
    int orient = LAYOUT_ROW;
    {
        const char *envg = std::getenv("TWMG_NO_GRAPH");
        h->step.enabled = !(envg && envg[0] == '1');
        const char *env = std::getenv("TWMG_ROW_LAYOUT");
        const bool row_only = env && env[0] == '1';
        if (dim == 2 && !row_only) {
            if (opt->smoother == MG_TWEED) orient = LAYOUT_TWEED;
            else if (opt->smoother == MG_WIREFRAME) orient = LAYOUT_WIREFRAME;
            else if (opt->smoother == MG_ZEBRA_Y) orient = LAYOUT_COLUMNS;
        }
        if (dim == 3 && !row_only && opt->smoother == MG_TWEED) orient = LAYOUT_TWEED3;
    }
    while (true) {
        Level &L = h->lev[nl];
        L.d.dim = dim;
        L.g.dim = dim;
        for (int a = 0; a < 3; ++a) {
            L.d.n[a] = a < dim ? cur[a] : 0;
            L.g.n[a] = L.d.n[a];
            L.g.np[a] = a < dim ? cur[a] + 1 : 1;
        }
        L.d.st[0] = 1;
        L.d.st[1] = L.g.np[0];
        L.d.st[2] = dim == 3 ? (long long)L.g.np[0] * L.g.np[1] : 0;
        L.d.nn = (long long)L.g.np[0] * L.g.np[1] * L.g.np[2];
        // split layout for the large 2D levels of line smoothers (lines along y
        // contiguous); small levels stay row-major (the coarse-level kernel
        // keeps them in LDS in that layout)
        // (3D tweed: three planes, one per line axis, from 65^3 nodes on)
        L.d.layout = (L.d.nn >= (dim == 3 ? SPLIT3_MIN_NODES : SPLIT_MIN_NODES)) ? orient : LAYOUT_ROW;
        L.d.bs = L.d.layout == LAYOUT_ROW ? L.d.nn : (L.d.layout == LAYOUT_TWEED3 ? 3 : 2) * L.d.nn;
        // the kernels address a problem's array with 32-bit slots (the batch
        // offset is 64-bit): one problem's array must stay below 2^31 entries
        if (L.d.bs > (long long)INT32_MAX) return MG_EUNSUPPORTED;
        // chunks are cut at the planes' borders, so that each is a run of
        // slots of one plane (3D tweed: a leg's end can be a tie node kept in
        // the other leg's plane)
        L.g.layout = L.d.layout;
        for (int a = 0; a < 3; ++a) L.g.st[a] = L.d.st[a];
        L.g.nn = L.d.nn;
        for (int a = 0; a < dim; ++a) {
            if (nl == 0) {
                L.x[a] = x0[a];
                if (st->sigma[a]) L.sig[a].assign(st->sigma[a], st->sigma[a] + cur[a]);
            } else {
                L.x[a].resize(cur[a] + 1);
                for (int i = 0; i <= cur[a]; ++i) L.x[a][i] = h->lev[nl - 1].x[a][2 * i];
                coarsen_sigma(h->lev[nl - 1].x[a], h->lev[nl - 1].sig[a], L.sig[a]);
            }
            make_coefs(L.x[a], L.sig[a], L.lo[a], L.hi[a]);
        }
        ++nl;
        bool can = true;
        for (int a = 0; a < dim; ++a)
            if (cur[a] % 2 || cur[a] < 4) can = false;
        if (!can || nl >= MAXLEV) break;
        for (int a = 0; a < dim; ++a) cur[a] /= 2;
    }
    h->nlev = nl;
    // coefficient blocks: forward and transposed, FP64 and FP32.  The
    // transposed operator's row p has the forward coefficients of its
    // neighbours toward p: lo^T_i = hi_{i-1}, hi^T_i = lo_{i+1}.
    for (int l = 0; l < nl; ++l) {
        Level &L = h->lev[l];
        // arrays of an even number of entries, so that each starts 16-byte
        // aligned in the device block (the sweep reads coefficient pairs)
        long long cs = 1;
        for (int a = 0; a < dim; ++a) cs = std::max(cs, (long long)L.d.n[a] + 1);
        cs += cs & 1;
        L.cs = cs;
        for (int o = 0; o < 2; ++o) L.hblk[o].assign(9 * cs, 0.0);
        for (int a = 0; a < dim; ++a) {
            const int n = L.d.n[a];
            const std::vector<double> &lo = L.lo[a], &hi = L.hi[a];
            for (int i = 0; i <= n; ++i) {
                const bool in = i >= 1 && i <= n - 1;
                const double dg = in ? -(lo[i] + hi[i]) : 0.0;
                L.hblk[0][(2 * a) * cs + i] = lo[i];
                L.hblk[0][(2 * a + 1) * cs + i] = hi[i];
                L.hblk[0][(6 + a) * cs + i] = dg;
                L.hblk[1][(2 * a) * cs + i] = (in && i - 1 >= 1) ? hi[i - 1] : 0.0;
                L.hblk[1][(2 * a + 1) * cs + i] = (in && i + 1 <= n - 1) ? lo[i + 1] : 0.0;
                L.hblk[1][(6 + a) * cs + i] = dg;
            }
        }
        int err = 0;
        for (int o = 0; o < 2; ++o) {
            // the device blocks carry COEF_PAD spare (zero) entries on both
            // sides: the sweep reads whole windows of CH + 2 entries around
            // a chunk, which may reach past the first or last array
            std::vector<double> b64(2 * COEF_PAD + L.hblk[o].size(), 0.0);
            std::copy(L.hblk[o].begin(), L.hblk[o].end(), b64.begin() + COEF_PAD);
            const std::vector<float> b32(b64.begin(), b64.end());
            const double *p64 = h->pool.upload(b64, err);
            const float *p32 = h->pool.upload(b32, err);
            if (err) return err;
            L.c64[o] = make_coef<double>(p64 ? p64 + COEF_PAD : nullptr, cs);
            L.c32[o] = make_coef<float>(p32 ? p32 + COEF_PAD : nullptr, cs);
            L.hc64[o] = make_coef<double>(L.hblk[o].data(), cs);
        }
        // the 3D stencil kernels visit only the tiles that hold nodes of
        // their plane
        if (dim == 3) {
            const std::vector<Tile3E> tl = tile3_list(L.d);
            L.d.tiles = h->pool.upload(tl, err);
            L.d.ntiles = (int)tl.size();
            if (err) return err;
        }
    }
    // block tables for every level that is smoothed
    for (int l = 0; l + 1 < nl; ++l) {
        Level &L = h->lev[l];
        for (int s = 0; s < MAXSLOT; ++s) {
            if (h->slot_motif[s] < 0) continue;
            // levels small enough for the coarse-level kernel: chunks of
            // CH - 1 points (its lanes read their chunks' points from LDS
            // directly, where chunks of CH points would put the lanes of a
            // straight run on the same banks)
            // (and TAIL_SHORT_CH points on the smallest of them)
            const bool tail_size = L.d.nn * 2 * (long long)sizeof(double) <= TAIL_BYTES;
            int nmax = 0;
            for (int a = 0; a < dim; ++a) nmax = std::max(nmax, L.d.n[a]);
            const bool short_main = !tail_size && nmax <= (dim == 2 ? SHORT_CH_MAXN : SHORT_CH_MAXN3);
            const int maxlen =
                !tail_size ? (short_main ? SHORT_CH : CH) : (nmax <= TAIL_SHORT_MAXN ? TAIL_SHORT_CH : CH - 1);
            std::vector<HostBlock> blocks, short_blocks;
            rc = build_blocks(L.g, h->slot_motif[s], blocks, maxlen);
            if (rc) return rc;
            // on the larger 2D levels, a colour whose blocks all still fit
            // NT/2 lanes with chunks of SHORT_CH points takes those (shorter
            // chains per lane; a colour with a larger block keeps CH)
            bool short_colour[2] = {maxlen <= SHORT_CH, maxlen <= SHORT_CH};
            if (dim == 2 && !tail_size && maxlen == CH) {
                rc = build_blocks(L.g, h->slot_motif[s], short_blocks, SHORT_CH);
                if (rc == MG_EUNSUPPORTED) short_blocks.clear(); // a block beyond NT chunks
                else if (rc) return rc;
                for (int colour = 0; colour < 2; ++colour) {
                    bool fits = !short_blocks.empty();
                    for (const HostBlock &hb : short_blocks)
                        if (hb.colour == colour && (int)hb.ch.size() > NT / 2) fits = false;
                    short_colour[colour] = fits;
                }
            }
            for (int colour = 0; colour < 2; ++colour) {
                std::vector<const HostBlock *> sel;
                for (const HostBlock &hb : short_colour[colour] && maxlen == CH ? short_blocks : blocks)
                    if (hb.colour == colour) sel.push_back(&hb);
                HostTable &t = L.htab[s][colour];
                // narrow workgroups for the levels too large for the
                // coarse-level kernel (whose sweeps use NT/2 lanes)
                const bool narrow = !tail_size;
                pack(sel, t, narrow);
                if (!validate(L.g, t)) return MG_EUNSUPPORTED;
                int err = 0;
                SweepTable &T = L.tab[s][colour];
                if (dim == 2) {
                    // records for the chunks of the small workgroups (the NT-lane
                    // ones address their points in general form)
                    t.addrs.assign(t.chunks.size(), ChunkAddr{0, 0, 0, 0});
                    for (size_t wi = (size_t)t.nbig; wi < t.wgs.size(); ++wi)
                        for (int q = t.wgs[wi].chunk0; q < t.wgs[wi].chunk0 + t.wgs[wi].nchunk; ++q)
                            if (!make_chunk_addr(L.d, t.chunks[q], t.addrs[q])) return MG_EUNSUPPORTED;
                    T.addrs = h->pool.upload(t.addrs, err);
                    for (int adj = 0; adj < 2; ++adj) {
                        std::vector<double> c64(2 * t.chunks.size());
                        for (size_t q = 0; q < t.chunks.size(); ++q)
                            chunk_cross_coefs<double>(L.hc64[adj], t.chunks[q], c64[2 * q], c64[2 * q + 1]);
                        const std::vector<float> c32(c64.begin(), c64.end());
                        T.cross64[adj] = h->pool.upload(c64, err);
                        T.cross32[adj] = h->pool.upload(c32, err);
                    }
                } else {
                    // 3D records and four cross coefficients per chunk, for
                    // the chunks of the small workgroups
                    t.addrs3.assign(t.chunks.size(), ChunkAddr3{0, 0, {0, 0}, {0, 0, 0, 0}});
                    for (size_t wi = (size_t)t.nbig; wi < t.wgs.size(); ++wi)
                        for (int q = t.wgs[wi].chunk0; q < t.wgs[wi].chunk0 + t.wgs[wi].nchunk; ++q)
                            if (!make_chunk_addr3(L.d, t.chunks[q], t.addrs3[q])) return MG_EUNSUPPORTED;
                    T.addrs3 = h->pool.upload(t.addrs3, err);
                    for (int adj = 0; adj < 2; ++adj) {
                        std::vector<double> c64(4 * t.chunks.size());
                        for (size_t q = 0; q < t.chunks.size(); ++q) {
                            double cc[4];
                            chunk_cross_coefs3<double>(L.hc64[adj], t.chunks[q], cc);
                            for (int e = 0; e < 4; ++e) c64[4 * q + e] = cc[e];
                        }
                        const std::vector<float> c32(c64.begin(), c64.end());
                        T.cross64[adj] = h->pool.upload(c64, err);
                        T.cross32[adj] = h->pool.upload(c32, err);
                    }
                }
                T.chunks = h->pool.upload(t.chunks, err);
                T.blocks = h->pool.upload(t.blocks, err);
                T.wgs = h->pool.upload(t.wgs, err);
                T.nwg = (int)t.wgs.size();
                T.nwg_big = t.nbig;
                T.nts = t.nts;
                T.cap = short_colour[colour] ? SHORT_CH : CH;
                T.nchunk = (int)t.chunks.size();
                T.nblock = (int)t.blocks.size();
                for (const Block &bk : t.blocks)
                    if (bk.type == BT_RING) T.rings = true;
                for (int adj = 0; adj < 2; ++adj) {
                    std::vector<NodeFac<double>> &f64 = L.hfac[s][colour][adj];
                    if (dim == 2) factor_table<2>(L.d, L.hc64[adj], t, f64);
                    else factor_table<3>(L.d, L.hc64[adj], t, f64);
                    std::vector<NodeFac<float>> f32(f64.size());
                    for (size_t q = 0; q < f64.size(); ++q)
                        f32[q] = NodeFac<float>{(float)f64[q].alpha, (float)f64[q].inv, (float)f64[q].gam,
                                                (float)f64[q].z};
                    T.fac64[adj] = h->pool.upload(f64, err);
                    T.fac32[adj] = h->pool.upload(f32, err);
                }
                if (err) return err;
            }
        }
    }
    // coarsest direct solve
    {
        Level &C = h->lev[nl - 1];
        const int nx = C.d.n[0] - 1, ny = C.d.n[1] - 1, nz = dim == 3 ? C.d.n[2] - 1 : 1;
        const int nu = nx * ny * nz;
        if (nu > MAX_COARSE_UNK) return MG_EUNSUPPORTED;
        h->nunk_coarse = nu;
        std::vector<double> A((size_t)nu * nu, 0.0);
        for (int q = 0; q < nu; ++q) {
            const int c[3] = {1 + q % nx, 1 + (q / nx) % ny, dim == 3 ? 1 + q / (nx * ny) : 0};
            double dg = 0;
            for (int a = 0; a < dim; ++a) dg -= C.lo[a][c[a]] + C.hi[a][c[a]];
            A[(size_t)q * nu + q] = dg;
            const int sz[3] = {1, nx, nx * ny};
            const int lim[3] = {nx, ny, nz};
            for (int a = 0; a < dim; ++a) {
                if (c[a] > 1) A[(size_t)q * nu + q - sz[a]] = C.lo[a][c[a]];
                if (c[a] < lim[a]) A[(size_t)q * nu + q + sz[a]] = C.hi[a][c[a]];
            }
        }
        std::vector<double> At((size_t)nu * nu);
        for (int i = 0; i < nu; ++i)
            for (int j = 0; j < nu; ++j) At[(size_t)i * nu + j] = A[(size_t)j * nu + i];
        std::vector<double> inv, invT;
        if (!invert(A, nu, inv) || !invert(At, nu, invT)) return MG_EINVAL;
        std::vector<float> inv32(inv.begin(), inv.end()), invT32(invT.begin(), invT.end());
        int err = 0;
        h->cinv64[0] = h->pool.upload(inv, err);
        h->cinv64[1] = h->pool.upload(invT, err);
        h->cinv32[0] = h->pool.upload(inv32, err);
        h->cinv32[1] = h->pool.upload(invT32, err);
        if (err) return err;
    }
    {
        // partial maxima, then one defect norm per problem
        std::vector<double> z(NORM_PARTS + (size_t)grid->batch, 0.0);
        int err = 0;
        h->partial = h->pool.upload(z, err);
        h->normv = h->partial + NORM_PARTS;
        if (err) return err;
        if (!h->pool.host_only) HIPCHK(hipHostMalloc((void **)&h->h_norm, sizeof(double) * grid->batch));
    }
    if ((rc = build_tail(h))) return rc;
    // the allocation-free norm's device array on this device (once per device)
    if (!h->pool.host_only) HIPCHK(scratch_init());
    if (!h->pool.host_only) {
        bool big = false;
        for (int l = 0; l + 1 < h->nlev; ++l)
            for (int sl = 0; sl < MAXSLOT; ++sl)
                for (int c = 0; c < 2; ++c) big = big || h->lev[l].tab[sl][c].nwg_big > 0;
        if (big) {
            HIPCHK(hipStreamCreateWithFlags(&h->side.aux, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&h->side.fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&h->side.join, hipEventDisableTiming));
        }
    }
    h->ws_bytes = workspace_layout(h, false);
    return MG_OK;
}

// ---------------------------------------------------------------------------
// cycle driver (Section 4, steps (1)-(6))
// ---------------------------------------------------------------------------
template <typename T> const Coef<T> &coefs(const Level &L, int adj);
template <> const Coef<double> &coefs<double>(const Level &L, int adj) { return L.c64[adj]; }
template <> const Coef<float> &coefs<float>(const Level &L, int adj) { return L.c32[adj]; }
template <typename T> T *lev_u(Level &L);
template <typename T> T *lev_f(Level &L);
template <> double *lev_u<double>(Level &L) { return L.u; }
template <> double *lev_f<double>(Level &L) { return L.f; }
template <> float *lev_u<float>(Level &L) { return L.u32; }
template <> float *lev_f<float>(Level &L) { return L.f32; }
template <typename T> const T *cinv(const mg_handle *h, int adj);
template <> const double *cinv<double>(const mg_handle *h, int adj) { return h->cinv64[adj]; }
template <> const float *cinv<float>(const mg_handle *h, int adj) { return h->cinv32[adj]; }

// one relaxation (for the alternating schemes: the group of sweeps); the
// adjoint runs sweeps and colours in reverse order
template <typename T> int relax(mg_handle *h, int lv, T *u, const T *f, int adj)
{
    Level &L = h->lev[lv];
    const Coef<T> &c = coefs<T>(L, adj);
    const int B = h->grid.batch;
    if (h->checker) {
        for (int k = 0; k < 2; ++k) HIPCHK(launch_checker<T>(L.d, c, u, f, adj ? 1 - k : k, B, h->stream));
        return MG_OK;
    }
    const int ns = nslots(h);
    for (int k = 0; k < ns; ++k) {
        const int s = adj ? ns - 1 - k : k;
        for (int q = 0; q < 2; ++q) {
            const int colour = adj ? 1 - q : q;
            HIPCHK(launch_block_sweep<T>(L.d, c, u, f, L.tab[s][colour], adj, B, h->stream, h->side));
        }
    }
    return MG_OK;
}

template <typename T> TailPlan<T> tail_plan(const mg_handle *h, int adj)
{
    TailPlan<T> p;
    if constexpr (sizeof(T) == 8) p = h->tail64[adj];
    else p = h->tail32[adj];
    p.ainv = cinv<T>(h, adj);
    return p;
}

template <typename T> int cycle(mg_handle *h, int lv, T *u, const T *f, int adj)
{
    Level &L = h->lev[lv];
    const int B = h->grid.batch;
    if (lv == h->tail_lv) {
        HIPCHK(launch_tail_cycle<T>(tail_plan<T>(h, adj), u, f, B, h->stream));
        return MG_OK;
    }
    if (lv == h->nlev - 1) {
        HIPCHK(launch_coarse_solve<T>(L.d, coefs<T>(L, adj), u, f, cinv<T>(h, adj), h->nunk_coarse, B, h->stream));
        return MG_OK;
    }
    int rc;
    for (int s = 0; s < h->opt.nu1; ++s)
        if ((rc = relax<T>(h, lv, u, f, adj))) return rc;
    Level &C = h->lev[lv + 1];
    T *uc = lev_u<T>(C), *fc = lev_f<T>(C);
    HIPCHK(launch_residual_restrict<T>(L.d, C.d, coefs<T>(L, adj), u, f, fc, uc, B, h->stream, (T *)h->dscr));
    // (the coarse-level kernel runs several of the gamma visits per launch)
    const int per = lv + 1 == h->tail_lv ? h->tail_reps : 1;
    for (int g = 0; g < h->opt.gamma; g += per)
        if ((rc = cycle<T>(h, lv + 1, uc, fc, adj))) return rc;
    HIPCHK(launch_prolong_add<T>(L.d, C.d, uc, u, B, h->stream));
    for (int s = 0; s < h->opt.nu2; ++s)
        if ((rc = relax<T>(h, lv, u, f, adj))) return rc;
    return MG_OK;
}

// the defect norm of every problem of the batch (out: batch values)
int read_norms(mg_handle *h, double *out)
{
    const int B = h->grid.batch;
    HIPCHK(hipMemcpyAsync(h->h_norm, h->normv, sizeof(double) * B, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int b = 0; b < B; ++b) out[b] = h->h_norm[b];
    return MG_OK;
}

bool finite(double v) { return v == v && !std::isinf(v); }

void drop_step_graph(mg_handle *h)
{
    if (h->step.exec) (void)hipGraphExecDestroy(h->step.exec);
    if (h->step.graph) (void)hipGraphDestroy(h->step.graph);
    h->step.exec = nullptr;
    h->step.graph = nullptr;
}

// Runs one step of the solve loop on h->stream: replays its captured graph,
// capturing it first (on a stream of the handle, with every launch of the
// step, the side stream's included) when there is none for these arrays,
// direction and precision.  A failed capture leaves the step eager for the
// rest of the handle's life.
template <typename F> int run_step(mg_handle *h, const void *u, const void *f, int adj, int prec, F &&step)
{
    auto &g = h->step;
    // only steps on the workspace's own arrays (levels in a split layout) are
    // captured: a caller's arrays may change from one solve to the next, and
    // capturing anew for each solve would cost more than it saves
    auto in_ws = [&](const void *p) {
        const char *c = static_cast<const char *>(p);
        return h->ws && c >= h->ws && c < h->ws + h->ws_bytes;
    };
    if (!g.enabled || g.broken || !in_ws(u) || !in_ws(f)) return step();
    if (!g.exec || g.u != u || g.f != f || g.adj != adj || g.prec != prec || g.gen != h->gen) {
        drop_step_graph(h);
        if (!g.cap && hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking) != hipSuccess) {
            g.broken = true;
            return step();
        }
        // (capturing runs nothing: the graph runs where it is launched)
        hipStream_t keep = h->stream;
        h->stream = g.cap;
        hipError_t e = hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal);
        int rc = e == hipSuccess ? step() : MG_EHIP;
        hipGraph_t graph = nullptr;
        if (e == hipSuccess) e = hipStreamEndCapture(g.cap, &graph);
        h->stream = keep;
        if (e == hipSuccess && rc == MG_OK) {
            g.graph = graph;
            e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        } else if (graph) {
            (void)hipGraphDestroy(graph);
        }
        if (e != hipSuccess || rc != MG_OK || !g.exec) {
            (void)hipGetLastError();
            drop_step_graph(h);
            g.broken = true;
            return step();
        }
        g.u = u;
        g.f = f;
        g.adj = adj;
        g.prec = prec;
        g.gen = h->gen;
    }
    HIPCHK(hipGraphLaunch(g.exec, h->stream));
    return MG_OK;
}

int solve_impl(mg_handle *h, double *u, const double *f, double tol, mg_stats *stats, int adj)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[0];
    const int B = h->grid.batch;
    const bool ir = h->opt.precision == MG_FP32_IR;
    // Section 4 stopping rule, per problem: each problem's defect norm is
    // measured against its own initial one, and the solve stops when the
    // largest of these ratios is below tol (a problem whose initial defect is
    // zero is already solved and takes no part)
    std::vector<double> d0(B), d(B);
    // With refinement every defect pass also leaves the defect rounded to
    // FP32 in L.f32: the right-hand side of the next step's FP32 cycle (the
    // same pass gives the norm, bitwise as launch_resnorm)
    auto defect_norm = [&]() -> hipError_t {
        return ir ? launch_resnorm_to_f32(L.d, L.c64[adj], u, f, L.f32, h->partial, NORM_PARTS, h->normv, B,
                                          h->stream)
                  : launch_resnorm<double>(L.d, L.c64[adj], u, f, h->partial, NORM_PARTS, h->normv, B, h->stream);
    };
    HIPCHK(defect_norm());
    if ((rc = read_norms(h, d0.data()))) return rc;
    int k = 0, status = MG_OK;
    double rel = 0.0, d0max = 0.0;
    bool bad0 = false, any = false;
    for (int b = 0; b < B; ++b) {
        bad0 = bad0 || !finite(d0[b]);
        any = any || d0[b] > 0.0;
        d0max = std::max(d0max, d0[b]);
    }
    if (bad0) status = MG_EDIVERGED;
    else if (any) {
        status = MG_ENOTCONV;
        // one step: a cycle (with refinement: e = FP32 cycle on A e = r from
        // 0, r = f - A u from the last defect pass rounded to FP32, then
        // u += e), then the defect pass
        auto step = [&]() -> int {
            int r;
            if (ir) {
                HIPCHK(launch_fill<float>(L.u32, L.d.bs * B, 0.0f, h->stream));
                if ((r = cycle<float>(h, 0, L.u32, L.f32, adj))) return r;
                HIPCHK(launch_ir_update(L.d, u, L.u32, B, h->stream));
            } else {
                if ((r = cycle<double>(h, 0, u, f, adj))) return r;
            }
            HIPCHK(defect_norm());
            return MG_OK;
        };
        while (k < h->opt.max_cycles) {
            if ((rc = run_step(h, u, f, adj, ir ? 1 : 0, step))) return rc;
            if ((rc = read_norms(h, d.data()))) return rc;
            rel = 0.0;
            bool bad = false;
            for (int b = 0; b < B; ++b) {
                bad = bad || !finite(d[b]);
                if (d0[b] > 0.0) rel = std::max(rel, d[b] / d0[b]);
            }
            if (bad) rel = std::numeric_limits<double>::infinity();
            if (stats && stats->history && k < stats->history_cap) stats->history[k] = rel;
            ++k;
            if (!finite(rel) || rel > 1e6) {
                status = MG_EDIVERGED;
                break;
            }
            if (rel < tol) {
                status = MG_OK;
                break;
            }
        }
    }
    if (stats) {
        stats->cycles = k;
        stats->status = status;
        stats->rel_res = rel;
        stats->res0 = d0max;
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

bool bad_level(const mg_handle *h, int lv) { return !h || lv < 0 || lv >= h->nlev; }

// does level L keep its own arrays in a split layout?
bool split(const Level &L) { return L.d.layout != LAYOUT_ROW; }

// the caller's row-major view of a level
Dims row_dims(const Dims &d)
{
    Dims r = d;
    r.layout = LAYOUT_ROW;
    r.bs = r.nn;
    r.tiles = nullptr;
    r.ntiles = 0;
    return r;
}

} // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int mg_setup(const mg_grid *grid, const mg_stretching *stretch, const mg_options *opt, void *stream, mg_handle **out)
{
    if (!grid || !stretch || !opt || !out) return MG_EINVAL;
    mg_handle *h = new (std::nothrow) mg_handle();
    if (!h) return MG_ENOMEM;
    h->stream = (hipStream_t)stream;
    int rc;
    try {
        rc = setup_impl(h, grid, stretch, opt);
    } catch (const std::bad_alloc &) {
        rc = MG_ENOMEM;
    } catch (...) {
        rc = MG_EINVAL;
    }
    if (rc) {
        mg_destroy(h);
        return rc;
    }
    *out = h;
    return MG_OK;
}

void mg_destroy(mg_handle *h)
{
    if (!h) return;
    if (h->pool.host_only) {
        delete h;
        return;
    }
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    if (h->ws_owned && h->ws) (void)hipFree(h->ws);
    if (h->h_norm) (void)hipHostFree(h->h_norm);
    drop_step_graph(h);
    if (h->step.cap) (void)hipStreamDestroy(h->step.cap);
    free_tail(h);
    if (h->side.aux) (void)hipStreamSynchronize(h->side.aux);
    if (h->side.fork) (void)hipEventDestroy(h->side.fork);
    if (h->side.join) (void)hipEventDestroy(h->side.join);
    if (h->side.aux) (void)hipStreamDestroy(h->side.aux);
    delete h;
}

int mg_set_stream(mg_handle *h, void *stream)
{
    if (!h) return MG_EINVAL;
    h->stream = (hipStream_t)stream;
    return MG_OK;
}

int mg_set_options(mg_handle *h, const mg_options *opt)
{
    if (!h || !opt) return MG_EINVAL;
    if (opt->nu1 < 0 || opt->nu2 < 0 || opt->gamma < 1 || opt->gamma > 2 || opt->max_cycles < 1) return MG_EINVAL;
    if (opt->precision != MG_FP64 && opt->precision != MG_FP32_IR) return MG_EINVAL;
    int m[MAXSLOT];
    bool ck;
    const int rc = motif_slots(opt->smoother, h->grid.dim, m, &ck);
    if (rc) return rc;
    if (!ck)
        for (int s = 0; s < MAXSLOT; ++s)
            if (m[s] != h->slot_motif[s]) return MG_EINVAL;
    h->opt = *opt;
    h->checker = ck;
    ++h->gen;
    return build_tail(h);
}

size_t mg_workspace_bytes(const mg_handle *h) { return h ? h->ws_bytes : 0; }

int mg_bind_workspace(mg_handle *h, void *dev_ptr, size_t bytes)
{
    if (!h || !dev_ptr || ((uintptr_t)dev_ptr & 255)) return MG_EINVAL;
    if (bytes < h->ws_bytes) return MG_ENOMEM;
    if (h->ws_owned && h->ws) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->ws);
    }
    h->ws = (char *)dev_ptr;
    h->ws_owned = false;
    ++h->gen;
    workspace_layout(h, true);
    return clear_workspace(h);
}

int mg_levels(const mg_handle *h, int *nlevels)
{
    if (!h || !nlevels) return MG_EINVAL;
    *nlevels = h->nlev;
    return MG_OK;
}

int mg_level_shape(const mg_handle *h, int lv, int *n)
{
    if (bad_level(h, lv) || !n) return MG_EINVAL;
    for (int a = 0; a < 3; ++a) n[a] = h->lev[lv].d.n[a];
    return MG_OK;
}

int mg_level_coefs(const mg_handle *h, int lv, int axis, double *x, double *lo, double *hi)
{
    if (bad_level(h, lv) || axis < 0 || axis >= h->grid.dim) return MG_EINVAL;
    const Level &L = h->lev[lv];
    const size_t n = L.x[axis].size();
    if (x) std::memcpy(x, L.x[axis].data(), n * sizeof(double));
    if (lo) std::memcpy(lo, L.lo[axis].data(), n * sizeof(double));
    if (hi) std::memcpy(hi, L.hi[axis].data(), n * sizeof(double));
    return MG_OK;
}

int mg_vcycle(mg_handle *h, double *u, const double *f)
{
    if (!h || !u || !f) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[0];
    if (!split(L)) return cycle<double>(h, 0, u, f, 0);
    const int B = h->grid.batch;
    HIPCHK(launch_convert<double>(L.d, u, L.u, 1, B, h->stream));
    HIPCHK(launch_convert<double>(L.d, f, L.f, 1, B, h->stream));
    if ((rc = cycle<double>(h, 0, L.u, L.f, 0))) return rc;
    HIPCHK(launch_convert<double>(L.d, L.u, u, 0, B, h->stream));
    return MG_OK;
}

int mg_solve(mg_handle *h, double *u, const double *f, const double *bc, double tol, mg_stats *stats)
{
    if (!h || !u || !f || !(tol >= 0)) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[0];
    const int B = h->grid.batch;
    const bool zero = !(h->opt.flags & MG_INITIAL_GUESS);
    if (!split(L)) {
        if (bc || zero) HIPCHK(launch_set_boundary(row_dims(L.d), u, bc, zero ? 1 : 0, B, h->stream));
        return solve_impl(h, u, f, tol, stats, 0);
    }
    if (zero) {
        // the start is the boundary data and a zero interior: written straight
        // into the level's layout (the caller's u gets every node on return)
        HIPCHK(launch_set_boundary(L.d, L.u, bc ? bc : u, 1, B, h->stream));
    } else {
        if (bc) HIPCHK(launch_set_boundary(row_dims(L.d), u, bc, 0, B, h->stream));
        HIPCHK(launch_convert<double>(L.d, u, L.u, 1, B, h->stream));
    }
    HIPCHK(launch_convert<double>(L.d, f, L.f, 1, B, h->stream));
    rc = solve_impl(h, L.u, L.f, tol, stats, 0);
    HIPCHK(launch_convert<double>(L.d, L.u, u, 0, B, h->stream));
    return rc;
}

int mg_solve_adjoint(mg_handle *h, double *lam, const double *w, double tol, mg_stats *stats)
{
    if (!h || !lam || !w || !(tol >= 0)) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[0];
    const int B = h->grid.batch;
    HIPCHK(launch_fill<double>(lam, L.d.nn * B, 0.0, h->stream));
    if (!split(L)) return solve_impl(h, lam, w, tol, stats, 1);
    HIPCHK(launch_fill<double>(L.u, L.d.bs * B, 0.0, h->stream));
    HIPCHK(launch_convert<double>(L.d, w, L.f, 1, B, h->stream));
    rc = solve_impl(h, L.u, L.f, tol, stats, 1);
    HIPCHK(launch_convert<double>(L.d, L.u, lam, 0, B, h->stream));
    return rc;
}

int mg_bc_grad(mg_handle *h, const double *lam, const double *w, double *grad_bc)
{
    if (!h || !lam || !w || !grad_bc) return MG_EINVAL;
    Level &L = h->lev[0];
    HIPCHK(launch_bc_grad(row_dims(L.d), L.c64[0], lam, w, grad_bc, h->grid.batch, h->stream));
    return MG_OK;
}

int mg_residual_norm(mg_handle *h, const double *u, const double *f, double *out_inf)
{
    if (!h || !u || !f || !out_inf) return MG_EINVAL;
    Level &L = h->lev[0];
    const int B = h->grid.batch;
    HIPCHK(launch_resnorm<double>(row_dims(L.d), L.c64[0], u, f, h->partial, NORM_PARTS, h->normv, B, h->stream));
    std::vector<double> d(B);
    const int rc = read_norms(h, d.data());
    if (rc) return rc;
    double m = 0.0;
    for (int b = 0; b < B; ++b) m = (d[b] != d[b] || m != m) ? d[b] + m : std::max(m, d[b]);
    *out_inf = m;
    return MG_OK;
}

int mg_residual_norm_noalloc(mg_handle *h, const double *u, const double *f, double *out_dev)
{
    if (!h || !u || !f || !out_dev || h->pool.host_only) return MG_EINVAL;
    if (h->grid.batch > NOALLOC_PARTS) return MG_EINVAL;
    Level &L = h->lev[0];
    HIPCHK(launch_resnorm_noalloc(row_dims(L.d), L.c64[0], u, f, out_dev, h->grid.batch, h->stream));
    return MG_OK;
}

int mg_smooth(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !u || !f || nu < 0) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[lv];
    const int B = h->grid.batch;
    double *uu = u;
    const double *ff = f;
    if (split(L)) {
        HIPCHK(launch_convert<double>(L.d, u, L.u, 1, B, h->stream));
        HIPCHK(launch_convert<double>(L.d, f, L.f, 1, B, h->stream));
        uu = L.u;
        ff = L.f;
    }
    for (int s = 0; s < nu; ++s)
        if ((rc = relax<double>(h, lv, uu, ff, adjoint ? 1 : 0))) return rc;
    if (split(L)) HIPCHK(launch_convert<double>(L.d, L.u, u, 0, B, h->stream));
    return MG_OK;
}

int mg_smooth_f32(mg_handle *h, int lv, float *u, const float *f, int nu, int adjoint)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !u || !f || nu < 0) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[lv];
    const int B = h->grid.batch;
    float *uu = u;
    const float *ff = f;
    if (split(L)) {
        HIPCHK(launch_convert<float>(L.d, u, L.u32, 1, B, h->stream));
        HIPCHK(launch_convert<float>(L.d, f, L.f32, 1, B, h->stream));
        uu = L.u32;
        ff = L.f32;
    }
    for (int s = 0; s < nu; ++s)
        if ((rc = relax<float>(h, lv, uu, ff, adjoint ? 1 : 0))) return rc;
    if (split(L)) HIPCHK(launch_convert<float>(L.d, L.u32, u, 0, B, h->stream));
    return MG_OK;
}

int mg_residual(mg_handle *h, int lv, const double *u, const double *f, double *d, int adjoint)
{
    if (bad_level(h, lv) || !u || !f || !d) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[lv];
    const int B = h->grid.batch;
    if (!split(L)) {
        HIPCHK(launch_residual<double>(L.d, L.d, L.c64[adjoint ? 1 : 0], u, f, d, B, h->stream));
        return MG_OK;
    }
    HIPCHK(launch_convert<double>(L.d, u, L.u, 1, B, h->stream));
    HIPCHK(launch_convert<double>(L.d, f, L.f, 1, B, h->stream));
    HIPCHK(launch_residual<double>(L.d, row_dims(L.d), L.c64[adjoint ? 1 : 0], L.u, L.f, d, B, h->stream));
    return MG_OK;
}

int mg_residual_restrict(mg_handle *h, int lv, const double *u, const double *f, double *fc, double *uc, int adjoint)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !u || !f || !fc || !uc) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[lv], &C = h->lev[lv + 1];
    const int B = h->grid.batch;
    const double *uu = u, *ff = f;
    double *fcc = fc, *ucc = uc;
    if (split(L)) {
        HIPCHK(launch_convert<double>(L.d, u, L.u, 1, B, h->stream));
        HIPCHK(launch_convert<double>(L.d, f, L.f, 1, B, h->stream));
        uu = L.u;
        ff = L.f;
    }
    if (split(C)) {
        // the kernel writes interior nodes only: carry the caller's boundary entries through
        HIPCHK(launch_convert<double>(C.d, fc, C.f, 1, B, h->stream));
        HIPCHK(launch_convert<double>(C.d, uc, C.u, 1, B, h->stream));
        fcc = C.f;
        ucc = C.u;
    }
    HIPCHK(launch_residual_restrict<double>(L.d, C.d, L.c64[adjoint ? 1 : 0], uu, ff, fcc, ucc, B, h->stream,
                                            (double *)h->dscr));
    if (split(C)) {
        HIPCHK(launch_convert<double>(C.d, C.f, fc, 0, B, h->stream));
        HIPCHK(launch_convert<double>(C.d, C.u, uc, 0, B, h->stream));
    }
    return MG_OK;
}

int mg_prolong_add(mg_handle *h, int lv, const double *ec, double *u)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !ec || !u) return MG_EINVAL;
    int rc = ensure_workspace(h);
    if (rc) return rc;
    Level &L = h->lev[lv], &C = h->lev[lv + 1];
    const int B = h->grid.batch;
    const double *ee = ec;
    double *uu = u;
    if (split(C)) {
        HIPCHK(launch_convert<double>(C.d, ec, C.u, 1, B, h->stream));
        ee = C.u;
    }
    if (split(L)) {
        HIPCHK(launch_convert<double>(L.d, u, L.u, 1, B, h->stream));
        uu = L.u;
    }
    HIPCHK(launch_prolong_add<double>(L.d, C.d, ee, uu, B, h->stream));
    if (split(L)) HIPCHK(launch_convert<double>(L.d, L.u, u, 0, B, h->stream));
    return MG_OK;
}

int mg_level_array_len(const mg_handle *h, int lv, long long *len)
{
    if (bad_level(h, lv) || !len) return MG_EINVAL;
    *len = h->lev[lv].d.bs;
    return MG_OK;
}

int mg_to_layout(mg_handle *h, int lv, const double *src, double *dst)
{
    if (bad_level(h, lv) || !src || !dst) return MG_EINVAL;
    HIPCHK(launch_convert<double>(h->lev[lv].d, src, dst, 1, h->grid.batch, h->stream));
    return MG_OK;
}

int mg_from_layout(mg_handle *h, int lv, const double *src, double *dst)
{
    if (bad_level(h, lv) || !src || !dst) return MG_EINVAL;
    HIPCHK(launch_convert<double>(h->lev[lv].d, src, dst, 0, h->grid.batch, h->stream));
    return MG_OK;
}

int mg_half_sweep(mg_handle *h, int lv, double *u, const double *f, int slot, int colour, int adjoint)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !u || !f || h->checker || slot < 0 || slot >= MAXSLOT || colour < 0 ||
        colour > 1 || h->slot_motif[slot] < 0)
        return MG_EINVAL;
    Level &L = h->lev[lv];
    const int adj = adjoint ? 1 : 0;
    HIPCHK(launch_block_sweep<double>(L.d, L.c64[adj], u, f, L.tab[slot][colour], adj, h->grid.batch, h->stream,
                                      h->side));
    return MG_OK;
}

const char *mg_strerror(int code)
{
    switch (code) {
    case MG_OK: return "ok";
    case MG_EINVAL: return "invalid argument";
    case MG_ENOMEM: return "out of memory (or workspace too small)";
    case MG_EHIP: return "HIP runtime error";
    case MG_ENOTCONV: return "not converged within max_cycles";
    case MG_EDIVERGED: return "diverged (NaN/Inf or defect growth)";
    case MG_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
    }
}

// ---------------------------------------------------------------------------
// Test hooks (include/twmg_debug.h).  Never called by the solver.
// ---------------------------------------------------------------------------
int mg_debug_table_info(const mg_handle *h, int lv, int slot, int colour, int *info)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || slot < 0 || slot >= MAXSLOT || colour < 0 || colour > 1 || !info)
        return MG_EINVAL;
    const HostTable &t = h->lev[lv].htab[slot][colour];
    int maxc = 0, maxb = 0;
    for (const WGDesc &w : t.wgs) {
        maxc = std::max(maxc, w.nchunk);
        maxb = std::max(maxb, w.nblock);
    }
    long long pts = 0;
    for (const Chunk &c : t.chunks) pts += c.len;
    info[0] = (int)t.wgs.size();
    info[1] = (int)t.chunks.size();
    info[2] = (int)t.blocks.size();
    info[3] = maxc;
    info[4] = maxb;
    info[5] = (int)pts;
    return MG_OK;
}

int mg_debug_setup_host(const mg_grid *grid, const mg_stretching *stretch, const mg_options *opt, mg_handle **out)
{
    if (!grid || !stretch || !opt || !out) return MG_EINVAL;
    mg_handle *h = new (std::nothrow) mg_handle();
    if (!h) return MG_ENOMEM;
    h->pool.host_only = true;
    int rc;
    try {
        rc = setup_impl(h, grid, stretch, opt);
    } catch (const std::bad_alloc &) {
        rc = MG_ENOMEM;
    }
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return MG_OK;
}

static int host_smooth(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint, const Dims &D);

int mg_debug_host_smooth(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !u || !f || nu < 0) return MG_EINVAL;
    if (h->checker) return MG_EUNSUPPORTED;
    return host_smooth(h, lv, u, f, nu, adjoint, row_dims(h->lev[lv].d));
}

int mg_debug_host_smooth_layout(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint)
{
    if (bad_level(h, lv) || lv == h->nlev - 1 || !u || !f || nu < 0) return MG_EINVAL;
    if (h->checker) return MG_EUNSUPPORTED;
    const Dims &D = h->lev[lv].d;
    const int B = h->grid.batch;
    const int nz = D.dim == 3 ? D.n[2] : 0;
    std::vector<double> us((size_t)D.bs * B, 0.0), fs((size_t)D.bs * B, 0.0);
    for (int b = 0; b < B; ++b)
        for (int l = 0; l <= nz; ++l)
            for (int j = 0; j <= D.n[1]; ++j)
                for (int i = 0; i <= D.n[0]; ++i) {
                    const long long r = (long long)b * D.nn + i + j * D.st[1] + l * D.st[2];
                    const long long q = (long long)b * D.bs + nidx(D, i, j, l);
                    us[q] = u[r];
                    fs[q] = f[r];
                }
    const int rc = host_smooth(h, lv, us.data(), fs.data(), nu, adjoint, D);
    for (int b = 0; b < B; ++b)
        for (int l = 0; l <= nz; ++l)
            for (int j = 0; j <= D.n[1]; ++j)
                for (int i = 0; i <= D.n[0]; ++i)
                    u[(long long)b * D.nn + i + j * D.st[1] + l * D.st[2]] = us[(long long)b * D.bs + nidx(D, i, j, l)];
    return rc;
}

} // extern "C"

// the kernel's per-lane steps run sequentially on the host, on arrays of layout D
static int host_smooth(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint, const Dims &D)
{
    Level &L = h->lev[lv];
    const int adj = adjoint ? 1 : 0;
    const Coef<double> &c = L.hc64[adj];
    std::vector<double> red(8 * NT);
    RedArrays<double> r{&red[0], &red[NT], &red[2 * NT], &red[3 * NT], &red[4 * NT], &red[5 * NT], &red[6 * NT],
                        &red[7 * NT]};
    std::vector<LaneState<double>> st(NT);
    std::vector<double> rhs(NT), dl(NT), pt((size_t)NT * CH);
    const int ns = nslots(h);
    for (int it = 0; it < nu; ++it)
        for (int k = 0; k < ns; ++k) {
            const int s = adj ? ns - 1 - k : k;
            for (int q = 0; q < 2; ++q) {
                const int colour = adj ? 1 - q : q;
                const HostTable &t = L.htab[s][colour];
                for (int b = 0; b < h->grid.batch; ++b) {
                    double *ub = u + (long long)b * D.bs;
                    const double *fb = f + (long long)b * D.bs;
                    const std::vector<NodeFac<double>> &fac = L.hfac[s][colour][adj];
                    for (const WGDesc &w : t.wgs) {
                        std::fill(red.begin(), red.end(), 0.0);
                        const Chunk *chs = &t.chunks[w.chunk0];
                        // the kernel's gather (cross-axis couplings per point), then
                        // per chunk the along-axis couplings of its end points
                        // as the kernel: 2D workgroups of NT/2 lanes use the chunk
                        // records (valid in the level's own layout only)
                        const bool rec = D.layout == L.d.layout && (&w - &t.wgs[0]) >= t.nbig;
                        for (int ln = 0; ln < w.nchunk; ++ln) {
                            double cm = 0, cp = 0, cc[4] = {0, 0, 0, 0};
                            if (rec && D.dim == 2) chunk_cross_coefs<double>(c, chs[ln], cm, cp);
                            if (rec && D.dim == 3) chunk_cross_coefs3<double>(c, chs[ln], cc);
                            for (int k = 0; k < chs[ln].len; ++k)
                                pt[ln * CH + k] =
                                    rec ? (D.dim == 2 ? point_rhs_rec<double>(D, t.addrs[w.chunk0 + ln], cm, cp, ub, fb, k)
                                                      : point_rhs_rec3<double>(D, t.addrs3[w.chunk0 + ln], cc, ub, fb, k))
                                        : (D.dim == 2 ? point_rhs_across<double, 2>(D, c, ub, fb, chs[ln], k)
                                                      : point_rhs_across<double, 3>(D, c, ub, fb, chs[ln], k));
                        }
                        for (int ln = 0; ln < w.nchunk; ++ln) {
                            double tb, tf;
                            if (D.dim == 2) chunk_end_terms<double, 2>(D, c, ub, chs[ln], tb, tf);
                            else chunk_end_terms<double, 3>(D, c, ub, chs[ln], tb, tf);
                            const double *rp = &pt[ln * CH];
                            const int Lc = chs[ln].len;
                            const double rL = rp[Lc - 1] - tf - (Lc == 1 ? tb : 0.0);
                            auto rr = [&](int k) { return k == 0 ? rp[0] - tb : rp[k]; };
                            if (D.dim == 2) sweep_phase1<double, 2, false, true>(D, c, rr, rL, chs[ln], ln, r, st[ln]);
                            else sweep_phase1<double, 3, false, true>(D, c, rr, rL, chs[ln], ln, r, st[ln]);
                        }
                        for (int ln = 0; ln < w.nchunk; ++ln) rhs[ln] = r.rs[ln] + r.rn[ln];
                        reduced_solve_seq<double>(w.nchunk, &t.chunks[w.chunk0], &fac[w.chunk0], rhs.data(),
                                                  dl.data(), r.x);
                        for (int ln = 0; ln < w.nchunk; ++ln) sweep_phase3<double>(&pt[ln * CH], ln, r, st[ln]);
                        for (int ln = 0; ln < w.nchunk; ++ln)
                            for (int k = 0; k < chs[ln].len; ++k)
                                ub[rec ? (D.dim == 2 ? rec_slot(D, t.addrs[w.chunk0 + ln], k)
                                                     : rec3_slot(D, t.addrs3[w.chunk0 + ln], k))
                                       : point_index(D, chs[ln], k)] = pt[ln * CH + k];
                    }
                }
            }
        }
    return MG_OK;
}

