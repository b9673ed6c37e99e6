// Internal data layout shared by the host driver (twmg.cpp) and the device
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace twmg {

// Lanes per block-relaxation workgroup and maximum points per chunk.  A block
// (one tweed spider, wireframe ring or zebra line) must fit in one workgroup:
// at most NT chunks of at most CH points each.
constexpr int NT = 512;
constexpr int CH = 16;
// spare entries on each side of a device coefficient block (a multiple of 2,
// at least the CH + 2 entries of a chunk's coefficient window)
constexpr int COEF_PAD = CH + 2;
// chunk capacity on the levels whose sweeps are bound by one workgroup's
// latency (the lane's serial chains and its gather batches are half as long)
constexpr int SHORT_CH = 8;
constexpr int SHORT_CH_MAXN = 1024; // 2D levels with at most this many cells per axis
constexpr int SHORT_CH_MAXN3 = 128; // 3D levels with at most this many cells per axis
// motif slots: the sweeps of one relaxation (three for 3D alternating-direction
// zebra: lines along x, then y, then z)
constexpr int MAXSLOT = 3;

// Direction codes: d = 2*axis + (positive ? 1 : 0); the reverse is d ^ 1.
__host__ __device__ inline int dir_axis(int d) { return d >> 1; }
__host__ __device__ inline int dir_sign(int d) { return (d & 1) ? 1 : -1; }

enum ChunkFlags : uint8_t {
    CF_PREV = 1,        // the first point's predecessor (reverse axis direction) is a node of this block
    CF_NEXT = 2,        // the last point has an in-block successor in direction nextdir
    CF_NEXT_DIRECT = 4, // ... and that successor is itself a reduced node (not a chunk interior point)
    CF_JUNCTION = 8,    // the last point is the branch point of a spider (extra in-block directions jmask)
};

// A chunk: up to CH consecutive collinear points of one leg/line/side.  Its
// last point is a node of the block's reduced system; the others are
// eliminated inside the lane that owns the chunk.
struct Chunk {
    int16_t c0[3];   // coordinates of the first point
    uint8_t len;     // 1..CH
    uint8_t axdir;   // direction of travel along the chunk
    uint8_t nextdir; // direction from the last point to its successor (CF_NEXT)
    uint8_t flags;   // ChunkFlags
    uint8_t jmask;   // CF_JUNCTION: bit d set if direction d from the last point is in-block
    uint8_t nflags;  // NodeFlags of the chunk's node in its block's reduced system
    int16_t prev;    // workgroup-local index of the predecessor node (CF_PREV)
    int16_t ext;     // workgroup-local index of the branch point (leg ends) or ring border node
};

// Precomputed addressing of a 2D chunk in its level's layout.  A chunk lies
// in one plane; along the chunk the slot moves by dp = +-1 when the chunk runs
// along its plane's fast axis, else by +-S (S: the plane's row length), and
// the neighbours across the chunk sit at -reg / +reg (reg = S or 1, the other
// one).  Near the diagonal of a split layout one point per side may have its
// cross neighbour in the other plane: point km (k_p) then reads slot irr_m
// (irr_p).  meta bits: 0-4 len, 5-9 km, 10-14 kp (31: none), 15/16 the last
// point's - / + cross neighbour is in the block, 17 plane (1: column-major),
// 18 chunk axis, 19 direction (1: increasing coordinate).
struct ChunkAddr {
    int p0;
    int irr_m, irr_p;
    uint32_t meta;
};
static_assert(sizeof(ChunkAddr) == 16, "chunk address record is 16 bytes");

// Addressing record of a 3D chunk.  Point k's slot is p0 + k step, step the
// chunk axis's stride in the chunk's plane (1 in the 3D tweed layout, whose
// lines run along their plane's fast axis), signed by the direction.  Its
// four neighbours across the chunk axis (the two other axes in increasing
// order, each toward - then +) sit at -/+ s[0] and -/+ s[1], except at one
// point (kx), whose neighbours flagged in xmask lie in other planes and are
// read from irr.  Along a line of the 3D tweed layout only the point nearest
// the centre can have such neighbours.  meta bits: 0-4 len, 5-9 kx (31:
// none), 10-13 xmask, 14-17 the last point's four cross neighbours are in the
// block, 18-19 chunk axis, 20 direction (1: increasing coordinate).
struct ChunkAddr3 {
    int p0;
    uint32_t meta;
    int s[2];
    int irr[4];
};
static_assert(sizeof(ChunkAddr3) == 32, "3D chunk address record is 32 bytes");

// Role of a node in the reduced-system solve.  Nodes are solved by two affine
// scans over the workgroup: forward elimination along each segment (a leg, a
// chain, or a ring opened at its border node), then back substitution.
enum NodeFlags : uint8_t {
    NF_HEAD = 1,  // first node of a segment
    NF_TAIL = 2,  // last node of a segment
    NF_J = 4,     // branch point of a spider (solved from the leg ends)
    NF_B = 8,     // border node of a ring (solved last)
    NF_RING = 16, // node of a ring's open part (corrected by the border value)
    NF_EXTJ = 32, // segment tail coupled to the branch point ext
};

// Setup-time factorisation of a node's reduced row (geometry only).
//  ordinary node: alpha = -lower*inv (0 at a head), inv = 1/pivot, gam = upper*inv,
//                 z = ring: border-column solution; leg end: branch row's coupling to it
//  branch point : inv = 1/(branch pivot), gam = its coupling to the node before it
//  ring border  : alpha = its lower coupling, inv = 1/(closing pivot), gam = its upper coupling
template <typename T> struct NodeFac {
    T alpha, inv, gam, z;
};
static_assert(sizeof(Chunk) == 16, "chunk descriptor is 16 bytes");

enum BlockType : uint8_t { BT_CHAIN = 0, BT_SPIDER = 1, BT_RING = 2 };

// A block's reduced system: nodes first .. first+count-1 (workgroup-local).
//  chain : nodes in order, node k couples to k-1 and k+1.
//  spider: legs 1..m-1 occupy consecutive node ranges ending at ends[l]; leg 0
//          follows and ends with the branch point (the last node).
//  ring  : nodes in cyclic order.
struct Block {
    int16_t first;
    int16_t count;
    uint8_t type;
    uint8_t m;
    int16_t ends[7];
};
static_assert(sizeof(Block) == 20, "block descriptor is 20 bytes");

struct WGDesc {
    int chunk0;   // first chunk of this workgroup in the colour's chunk array
    int nchunk;   // <= NT
    int block0;   // first block in the colour's block array
    int nblock;   // <= NT
};

// Node array layouts.  LAYOUT_ROW: row-major, x fastest (the caller's layout).
// The split layouts (2D only) keep two planes of nn slots each: plane R,
// row-major, holds the points whose block lines run along x; plane C, column-
// major (y fastest), holds those whose lines run along y.  Every line of a
// block is then contiguous in memory.  With i' = min(i, nx-i), j' = min(j, ny-j):
//   LAYOUT_TWEED     : plane C iff i' > j'  (tweed legs along y)
//   LAYOUT_WIREFRAME : plane C iff i' < j'  (wireframe sides along y)
//   LAYOUT_COLUMNS   : plane C for every node (lines along y everywhere)
// LAYOUT_TWEED3 (3D tweed): three planes of nn slots.  A node is kept in the
// plane of the axis its tweed line runs along, the axis of the smallest of
// i', j', l' (ties to the lower axis; boundary nodes alike), and each plane
// stores that axis fastest:
//   plane 0: i + (nx+1)(j + (ny+1) l)         (x-lines, row-major)
//   plane 1: nn + j + (ny+1)(i + (nx+1) l)    (y-lines)
//   plane 2: 2 nn + l + (nz+1)(i + (nx+1) j)  (z-lines)
enum Layout : int { LAYOUT_ROW = 0, LAYOUT_TWEED = 1, LAYOUT_WIREFRAME = 2, LAYOUT_COLUMNS = 3, LAYOUT_TWEED3 = 4 };

// levels with at least this many nodes use the split layout of their smoother
constexpr long long SPLIT_MIN_NODES = 129 * 129;
constexpr long long SPLIT3_MIN_NODES = 65LL * 65 * 65;

struct Dims {
    int dim;
    int n[3];          // cells per axis (0 beyond dim)
    long long st[3];   // row-major node strides: 1, nx+1, (nx+1)(ny+1)
    long long nn;      // nodes per problem
    int layout;        // Layout
    long long bs;      // array length per problem (batch stride): nn, 2 nn (2D split), 3 nn (3D split)
    // 3D levels: the tiles the 3D stencil kernels visit (device list of
    // ntiles entries, Tile3E; on the split layout only the tiles that hold
    // nodes of their plane); null: every tile of the row-major layout
    const struct Tile3E *tiles = nullptr;
    int ntiles = 0;
};
// A tile of the 3D stencil kernels: x = plane | (first F coordinate << 2),
// y = first A coordinate | (first B coordinate << 16)
struct Tile3E {
    int x, y;
};

// split layouts: is node (i, j) stored in plane C?
__host__ __device__ inline bool col_plane(const Dims &d, int i, int j)
{
    const int ip = i < d.n[0] - i ? i : d.n[0] - i, jp = j < d.n[1] - j ? j : d.n[1] - j;
    return d.layout == LAYOUT_TWEED ? ip > jp : (d.layout == LAYOUT_WIREFRAME ? ip < jp : true);
}

// 3D tweed split layout: the plane (axis) of node (i, j, l)
__host__ __device__ inline int plane3(const Dims &d, int i, int j, int l)
{
    const int ip = i < d.n[0] - i ? i : d.n[0] - i, jp = j < d.n[1] - j ? j : d.n[1] - j,
              lp = l < d.n[2] - l ? l : d.n[2] - l;
    if (ip <= jp && ip <= lp) return 0;
    return jp <= lp ? 1 : 2;
}

// slot of node (i, j, l) in plane pl of the 3D tweed split layout
__host__ __device__ inline long long plane3_slot(const Dims &d, int pl, int i, int j, int l)
{
    const long long S0 = d.n[0] + 1, S1 = d.n[1] + 1, S2 = d.n[2] + 1;
    if (pl == 0) return i + S0 * (j + S1 * l);
    if (pl == 1) return d.nn + j + S1 * (i + S0 * l);
    return 2 * d.nn + l + S2 * (i + S0 * j);
}

// slot of node (i, j, l) in an array of layout d.layout
__host__ __device__ inline long long nidx(const Dims &d, int i, int j, int l)
{
    if (d.layout == LAYOUT_ROW) return i + j * d.st[1] + l * d.st[2];
    if (d.layout == LAYOUT_TWEED3) return plane3_slot(d, plane3(d, i, j, l), i, j, l);
    return col_plane(d, i, j) ? d.nn + j + (long long)i * (d.n[1] + 1) : i + j * d.st[1];
}

// Coefficients of one level (one direction of the operator), stored as nine
// arrays of cs entries in one block: lo_x, hi_x, lo_y, hi_y, lo_z, hi_z, dg_x,
// dg_y, dg_z, each indexed by the node coordinate along its axis.  The array of
// direction d (= 2*axis + positive) starts at base + d*cs, so picking one for a
// per-lane direction is address arithmetic, not a choice between pointers.
template <typename T> struct Coef {
    const T *lo[3];    // coefficient toward the -1 neighbour
    const T *hi[3];    // toward the +1 neighbour
    const T *dg[3];    // contribution of the axis to the diagonal
    const T *base;     // start of the block (== lo[0])
    long long cs;      // entries per array
};

template <typename T> __host__ __device__ inline Coef<T> make_coef(const T *base, long long cs)
{
    Coef<T> c;
    for (int a = 0; a < 3; ++a) {
        c.lo[a] = base + (2 * a) * cs;
        c.hi[a] = base + (2 * a + 1) * cs;
        c.dg[a] = base + (6 + a) * cs;
    }
    c.base = base;
    c.cs = cs;
    return c;
}

struct SweepTable {
    Chunk *chunks = nullptr;
    ChunkAddr *addrs = nullptr;   // 2D: per-chunk addressing records
    ChunkAddr3 *addrs3 = nullptr; // 3D: per-chunk addressing records
    // per-chunk cross coefficients [fwd, transposed]: 2D toward -, +; 3D
    // toward -, + along each of the two other axes
    double *cross64[2] = {nullptr, nullptr};
    float *cross32[2] = {nullptr, nullptr};
    Block *blocks = nullptr;
    WGDesc *wgs = nullptr;
    NodeFac<double> *fac64[2] = {nullptr, nullptr}; // [forward, transposed operator]
    NodeFac<float> *fac32[2] = {nullptr, nullptr};
    int nwg = 0, nchunk = 0, nblock = 0;
    int nwg_big = 0; // the first nwg_big workgroups need NT lanes, the others nts
    int nts = NT / 2; // lanes of the small workgroups: 64, 128 or NT/2
    int cap = CH;     // longest chunk: CH, or SHORT_CH (levels bound by a workgroup's latency)
    bool rings = false;
};

// ---- coarse-level cycle in one workgroup ---------------------------------
// The coarsest levels of the hierarchy are small enough to live in LDS: one
// workgroup per problem runs their whole sub-cycle (smoothing, defect
// restriction, coarsest solve, prolongation) from a host-built list of
// operations, with workgroup barriers between them.  Its read-only data (level
// descriptors, coefficients, block tables, operations) form one image that the
// kernel copies into LDS; all offsets below are byte offsets into LDS.
constexpr int TAIL_BYTES = 147456; // LDS bytes for the image plus the levels' u, f and solve scratch
constexpr int TAIL_NT = NT / 2;    // lanes of the coarse-level workgroup
// chunk length on the smallest levels of the coarse-level kernel: its sweeps
// are bound by one workgroup's instruction issue, which a lane's chunk length
// sets (code for C positions runs whatever the actual length)
constexpr int TAIL_SHORT_CH = 4;
constexpr int TAIL_SHORT_MAXN = 32; // levels with at most this many cells per axis

// TO_MAP: the whole sub-cycle of a level applied as its precomputed affine
// map (TailPlan::map), in place of the operations it stands for
enum TailOpKind : uint8_t { TO_SWEEP = 0, TO_CHECKER = 1, TO_RESTRICT = 2, TO_PROLONG = 3, TO_SOLVE = 4, TO_MAP = 5 };
// largest number of unknowns of a level whose sub-cycle is applied as a map
constexpr int TAIL_MAP_MAX = 256;
static_assert(TAIL_MAP_MAX <= TAIL_NT, "one lane per unknown of a mapped level");
struct TailOp {
    uint8_t kind;   // TailOpKind
    uint8_t lv;     // level, counted from the first level of the tail
    uint8_t slot;   // TO_SWEEP: motif slot
    uint8_t colour; // TO_SWEEP / TO_CHECKER
};

struct TailLevel {
    Dims d;
    int co;            // coefficient block (nine arrays of cs entries, as in Coef)
    int cs;
    int uoff, foff;    // the level's u and f (whole node arrays)
    int chunk_off[MAXSLOT][2], block_off[MAXSLOT][2], wg_off[MAXSLOT][2], fac_off[MAXSLOT][2]; // [slot][colour]
    int nwg[MAXSLOT][2];
    int rings[MAXSLOT][2];
    int short_chunks;        // every chunk of the level has at most TAIL_SHORT_CH points
    int onewave[MAXSLOT][2]; // every descriptor of the table has at most 64 chunks and 64 blocks
};

template <typename T> struct TailPlan {
    const unsigned char *image = nullptr; // device copy of the read-only image (16-byte multiple)
    int image_bytes = 0;
    int lev_off = 0;                      // TailLevel array
    int ops_off = 0;                      // TailOp array
    int nops = 0;
    int rhs_off = 0;                      // coarsest solve scratch (nunk values)
    int nunk = 0;                         // unknowns of the coarsest level
    int dim = 2;
    long long nn0 = 0;                    // nodes of the first tail level (batch stride)
    const T *ainv = nullptr;              // coarsest-level inverse (global memory)
    // TO_MAP: the sub-cycle of one level (map_nu <= TAIL_MAP_MAX interior
    // unknowns, numbered x fastest) as u_out = U u_in + F f, stored input
    // major: map[k * map_nu + i] is U[i][k] for k < map_nu and F[i][k - map_nu]
    // above (global memory)
    const T *map = nullptr;
    int map_nu = 0;
};

// ---- launchers (kernels.hip) -------------------------------------------
// Side stream for the NT-lane workgroups of a half-sweep: blocks of one colour
// are independent, so the big-block launch runs beside the NT/2-lane one
// (fork and join through the two events).  aux == nullptr: one stream.
struct SideStream {
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

template <typename T>
hipError_t launch_block_sweep(const Dims &d, const Coef<T> &c, T *u, const T *f, const SweepTable &tab, int adj,
                              int batch, hipStream_t s, const SideStream &side = SideStream());
template <typename T>
hipError_t launch_checker(const Dims &d, const Coef<T> &c, T *u, const T *f, int colour, int batch, hipStream_t s);
template <typename T>
hipError_t launch_residual(const Dims &d, const Dims &dout, const Coef<T> &c, const T *u, const T *f, T *r, int batch,
                           hipStream_t s);
// row-major <-> layout d.layout (a plain copy for LAYOUT_ROW)
template <typename T>
hipError_t launch_convert(const Dims &d, const T *src, T *dst, int to_split, int batch, hipStream_t s);
template <typename T>
// dscr: scratch of one fine-level array (layout fd, batch included) for the
// 3D split layout, whose restriction runs in two passes (defect, weighting)
hipError_t launch_residual_restrict(const Dims &fd, const Dims &cd, const Coef<T> &c, const T *u, const T *f, T *fc,
                                    T *uc, int batch, hipStream_t s, T *dscr = nullptr);
template <typename T>
hipError_t launch_prolong_add(const Dims &fd, const Dims &cd, const T *ec, T *u, int batch, hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve(const Dims &d, const Coef<T> &c, T *u, const T *f, const T *ainv, int nunk, int batch,
                               hipStream_t s);
// ||f - L u||_inf over the interior of each problem b into out[b] (b < batch);
// partial holds npart slots of per-workgroup maxima
template <typename T>
hipError_t launch_resnorm(const Dims &d, const Coef<T> &c, const T *u, const T *f, double *partial, int npart,
                          double *out, int batch, hipStream_t s);
hipError_t launch_resnorm_to_f32(const Dims &d, const Coef<double> &c, const double *u, const double *f, float *r32,
                                 double *partial, int npart, double *out, int batch, hipStream_t s);
hipError_t launch_ir_update(const Dims &d, double *u, const float *e, int batch, hipStream_t s);
// the tiles of the 3D stencil kernels on a 3D level (for Dims::tiles): on the
// split layout those that hold nodes of their plane
std::vector<Tile3E> tile3_list(const Dims &d);
hipError_t launch_set_boundary(const Dims &d, double *u, const double *bc, int zero_interior, int batch,
                               hipStream_t s);
template <typename T> hipError_t launch_fill(T *p, long long n, T v, hipStream_t s);
hipError_t launch_bc_grad(const Dims &d, const Coef<double> &fwd, const double *lam, const double *w, double *g,
                          int batch, hipStream_t s);

template <typename T>
hipError_t launch_tail_cycle(const TailPlan<T> &p, T *u, const T *f, int batch, hipStream_t s);

constexpr int NORM_PARTS = 65536; // partial-maximum slots used by launch_resnorm

// Allocation-free defect norm (mg_residual_norm_noalloc): partial maxima in a
// file-scope device array of NOALLOC_PARTS doubles (128 KiB per device, held
// until the process ends).  scratch_init resolves the current device's copy
// (call once per device, that device current); launch_resnorm_noalloc writes
// the maximum over the batch of ||f - L u||_inf to out[0] (device memory).
constexpr int NOALLOC_PARTS = 16384;
hipError_t scratch_init();
hipError_t launch_resnorm_noalloc(const Dims &d, const Coef<double> &c, const double *u, const double *f,
                                  double *out, int batch, hipStream_t s);

} // namespace twmg
