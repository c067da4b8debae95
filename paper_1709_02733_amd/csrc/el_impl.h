// Internal declarations of the elastic operator library (device parameter
// block, workspace layout, kernel launchers).  Not part of the public ABI.
//
// Volume layout.  Every wavefield and material array is stored padded:
// row pitch px >= nx + 2 (a multiple of 32 elements), py = ny + 2 rows per
// plane, and nz + 4 planes of which the first and last two are guards.
// Cell (i, j, k) sits at element (k + 2) * px * py + j * px + i.  The
// padding of a wavefield is zero and is never written, so a stencil tap that
// leaves the grid (by at most two cells along one axis) reads zero -- the
// zero extension of the fields -- without a bounds check: a tap at i = -1 or
// -2 lands in the padding columns at the end of the previous row, a tap at
// j = -1, -2 in the padding rows at the end of the previous plane, and taps
// beyond the upper faces in the padding of the same row or plane.  Material
// maps hold, in their +x, +y, +z padding, the value of the nearest cell, so
// the staggered averages at the last index replicate it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include "el.h"

namespace el {

// Wavefield array ids (same order as el_plan_field).
enum Field { U1 = 0, U2, U3, S11, S22, S33, S23, S13, S12, NFIELD };

// Padded volume geometry (elements).
struct Vol {
    int nx, ny, nz;
    int px, py;              // row pitch, rows per plane
    long long plane;         // px * py
    long long total;         // plane * (nz + 4)
    long long origin;        // element of cell (0,0,0): 2 * plane
};
Vol make_vol(int nx, int ny, int nz);

// Record the detail of a failure for el_last_error() and return the status.
el_status set_error(el_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Everything a stencil kernel needs, passed by value.
template <typename T>
struct Dev {
    int nx, ny, nz;
    unsigned sy, sz;         // byte strides of +y and +z (the +x stride is sizeof(T))
    unsigned origin;         // byte offset of cell (0,0,0)
    int px;                  // row pitch (elements)
    long long plane;         // plane size (elements)
    T dt, inv_dx;
    T *f[NFIELD];            // u1, u2, u3, s11, s22, s33, s23, s13, s12 (padded)
    const T *lam, *mu, *rho, *alpha;   // cell maps (padded, edge-replicated)
    int P;                   // C-PML cells per face, 0 = none
    int hi[3];               // first index of the high boundary slab per axis: n - 1 - P
    int W;                   // slab planes per axis: 2 (P + 7)
    const T *pa[3][2];       // PML a per axis, [0] integer / [1] half positions
    const T *pb[3][2];       // PML b
    T *mem[3][6];            // boundary-slab memory variables of axis j:
                             //   mem[j][i]     = phi^{ij} (u^i point),
                             //   mem[j][3 + i] = psi^{ij} (sigma^{ij} point)
    const T *med;            // per tile: lambda, rho, alpha, 0 of a uniform fluid tile
};

// Boundary-slab storage of the C-PML memory variables.  Along each axis the variables live on
// two extended ranges of planes: the low range covers coordinates -2 .. P+4 and the high
// range hi-4 .. n+1 (hi = n-1-P), stored at slab coordinates 0 .. P+6 and P+7 .. 2P+13, so
// W = 2 (P + 7) planes in all.  Cells of the layer (c <= P or c >= hi) own their value; the
// extra planes let a 4-tap difference centred on any cell within two planes of a layer read
// its taps without tests, and hold zeros (the adjoint keeps its memory variables multiplied
// by the layer coefficient a, which vanishes outside the layer).  When both ranges cover a
// layer cell (fewer than ten planes between the layers) the cell writes both copies.
__host__ __device__ inline int slab_lo(int c) { return c + 2; }
__host__ __device__ inline int slab_hi(int c, int P, int hi) { return c - (hi - 4) + P + 7; }
// primary slab coordinate of a layer cell, -1 outside the layer
__host__ __device__ inline int slab_own(int c, int P, int hi) {
    return c <= P ? slab_lo(c) : (c >= hi ? slab_hi(c, P, hi) : -1);
}
// second copy of a layer cell covered by both ranges, -1 otherwise
__host__ __device__ inline int slab_twin(int c, int P, int hi) {
    return (c <= P && c >= hi - 4) ? slab_hi(c, P, hi) : ((c >= hi && c <= P + 4) ? slab_lo(c) : -1);
}
// slab coordinate of a cell whose 4-tap stencil along the axis reaches a layer, -1 otherwise
__host__ __device__ inline int slab_near(int c, int P, int hi) {
    return c <= P + 2 ? slab_lo(c) : (c >= hi - 2 ? slab_hi(c, P, hi) : -1);
}
// Element order: axis x as [side][k][j][s'] with s' the coordinate within the side's
// P + 7 planes (a tile's rows of one side are contiguous; the two sides are touched by
// different tiles), axis y as [k][s][i], axis z as [s][j][i].
template <typename T>
__device__ inline unsigned slab_byte(const Dev<T> &d, int axis, int s, int i, int j, int k) {
    unsigned e;
    if (axis == 0) {
        const int hw = d.W >> 1;
        const int side = s >= hw ? 1 : 0;
        e = (((unsigned)side * d.nz + k) * d.ny + j) * hw + (s - side * hw);
    } else {
        e = axis == 1 ? ((unsigned)k * d.W + s) * d.nx + i : ((unsigned)s * d.ny + j) * d.nx + i;
    }
    return e * (unsigned)sizeof(T);
}
// byte stride between neighbouring slab coordinates of an axis
template <typename T>
__device__ inline unsigned slab_stride(const Dev<T> &d, int axis) {
    return (unsigned)sizeof(T) * (axis == 0 ? 1u : (axis == 1 ? (unsigned)d.nx : (unsigned)d.nx * d.ny));
}

// Column tiles of the stencil passes: kTileX x kTileY cells in x-y, a chunk of zc planes in z.
constexpr int kTileX = 64;
constexpr int kTileY = 4;
struct Tiles {
    int ntx, nty, nzc, zc;   // tiles along x and y, z chunks, planes per chunk
    int ntiles;              // ntx * nty * nzc
    int per;                 // tiles per XCD: the grid has 8 * per blocks
    const int *order;        // device: tile of each block (-1 for a padding block)
    const unsigned long long *lanes;   // device: per tile and row, its fluid columns; then, per tile
                                       // and row, those of the tile's reference medium (k_classify)
};
Tiles make_tiles(int nx, int ny, int nz);
// XCD (0..7) that processes tile q; blocks run on XCD blockIdx % 8.
int tile_xcd(const Tiles &t, int q);
// Tile of each block (8 * per entries, -1 for padding blocks): the tiles of XCD x in z-major
// order at entries x, x + 8, x + 16, ...  An entry holds the tile number in its low
// kEdgeShift bits and carries kFastTile when fast[q] is set (fast may be null): the block
// then runs the fluid update of the tile.  The four bits from kEdgeShift up mark which face
// neighbours of a fluid tile along y (y-, y+) and z (z-, z+) take the general update.  The
// general loop differences s22 only along y and s33 only along z, with taps reaching two
// cells into a neighbouring tile, so the fluid update stores s22 only on two-row bands
// along such y faces and s33 only on two-plane bands along such z faces.
// kUniformTile marks a fluid tile whose lambda, rho and alpha are constant over the cells
// its loops read (k_classify): they come from a per-tile table instead of the maps.
// kColumnTile marks a tile that is not fluid but has fluid columns (Tiles::lanes): the
// lanes of those columns run the fluid update.
constexpr int kFastTile = 1 << 30;
constexpr int kUniformTile = 1 << 29;
constexpr int kColumnTile = 1 << 28;
constexpr int kEdgeShift = 24;
constexpr int kTileMask = (1 << kEdgeShift) - 1;
std::vector<int> tile_order(const Tiles &t, const unsigned char *fast, const unsigned char *uni,
                            const unsigned char *cols);
// Bits kEdgeShift.. of tile q's entry (0 unless q is a fluid tile).
int tile_edges(const Tiles &t, const unsigned char *fast, int q);

// Relaxation mechanisms of the frequency-dependent absorption (el_relaxation): after every
// velocity pass the tiles holding a velocity point with beta > 0 apply the pointwise
// sub-update R (forward) or R^T (adjoint) to u and the memory variables zeta_l.
template <typename T>
struct Relax {
    int L;                   // mechanisms (0: none)
    T w[EL_MAX_MECH];        // weights
    T c[EL_MAX_MECH];        // exp(-omega_l dt)
    const T *ar;             // strength alpha_r, a padded cell map (edge-replicated like the others)
    const unsigned char *flag;   // per tile: 1 if some velocity point of it has beta > 0 (set-up)
    int *count;              // per tile: its (cell, component) velocity points with beta > 0 (set-up)
    long long *off;          // per tile: index of its first point in pts (set-up)
    // the velocity points with beta > 0, tile by tile, within a tile by component, then plane,
    // row, column: the padded element index with the component in bits 30-31, beta, and the
    // memory variables [l][point]
    unsigned *pts;
    T *beta;
    T *zeta;
    long long npts;
};

constexpr unsigned kRelaxElemMask = (1u << 30) - 1;

// Receiver tables (cell offsets are padded element indices).
struct Rec {
    int nrec;
    const long long *idx;    // [L][8] corner elements
    const double *w;         // [L][8] trilinear weights
    const unsigned char *fl; // [L][8] 1 where the corner lies in a fluid tile: trace is 3 s11
    // grid-point-major transpose for the deterministic scatter
    int npts;
    const long long *pt;     // [npts] touched elements
    const int *ptc;          // [npts][3] their i, j, k
    const int *row;          // [npts + 1] offsets into ent_rec / ent_w
    const int *ent_rec;      // receiver of each entry
    const double *ent_w;     // weight of each entry
    // scatter points by stencil tile and column: tslot[t] is -1 for a tile without points,
    // else s, and the points of column (c, r) of the tile (key c + kTileX r) are
    // tpts[loff[s (kTileX kTileY + 1) + key] .. loff[... + key + 1])
    const int *tslot;        // [ntiles]
    const int *loff;         // [slots][kTileX kTileY + 1]
    const int *tpts;         // [npts] point numbers sorted by (tile, key)
};

// Receiver gather: p_hat_m[l] = -sum_c w_lc (s11 + s22 + s33)[c]  (Sec. 3, eq. interpgrid), in
// double.  One wavefront serves 8 receivers; lane = 8 * receiver + corner, reduced over 8
// lanes.  On a fluid tile s22 = s33 = s11 (the lean stress loop stores s11 alone there), and
// the trace is taken as 3 s11, the same double as the sum of the three equal terms.
template <typename T>
__device__ __forceinline__ double trace_at(const Dev<T> &d, const Rec &r, int e) {
    const long long q = r.idx[e];
    const double s11 = (double)d.f[S11][q];
    return r.fl[e] ? 3.0 * s11 : s11 + (double)d.f[S22][q] + (double)d.f[S33][q];
}
// The receivers of gather block gb (256 threads: 4 wavefronts, 32 receivers) into out[].
template <typename T>
__device__ __forceinline__ void gather_block(const Dev<T> &d, const Rec &r, double *out, int gb) {
    const int lane = threadIdx.x & 63;
    const int wave = (gb * 256 + (int)threadIdx.x) >> 6;
    const int l = wave * 8 + (lane >> 3);
    const int c = lane & 7;
    double v = 0.0;
    if (l < r.nrec) v = r.w[8 * l + c] * trace_at(d, r, 8 * l + c);
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (l < r.nrec && c == 0) out[l] = -v;
}
inline int gather_blocks(int nrec) { return ((nrec + 7) / 8 + 3) / 4; }

// s_kk += Theta^T y_m at point t of the grid-point-major table (entries summed in a fixed
// order).  With the adjoint stress kept as w = C s this adds (3 lambda + 2 mu) delta to w11,
// w22, w33, and the normal adjoint memory variables, which hold a (b psi~ + dt w) for the
// coming step, receive a dt times the same increment.
template <typename T>
__device__ __forceinline__ void scatter_point(const Dev<T> &d, const Rec &r, const double *y, int t) {
    double acc = 0.0;
    for (int e = r.row[t]; e < r.row[t + 1]; ++e) acc += r.ent_w[e] * y[r.ent_rec[e]];
    const long long q = r.pt[t];
    const T dw = T(-acc) * (T(3) * d.lam[q] + T(2) * d.mu[q]);
    d.f[S11][q] += dw;
    d.f[S22][q] += dw;
    d.f[S33][q] += dw;
    if (d.P > 0) {
        const int crd[3] = {r.ptc[3 * t], r.ptc[3 * t + 1], r.ptc[3 * t + 2]};
        for (int a = 0; a < 3; ++a) {
            const int s = slab_own(crd[a], d.P, d.hi[a]);
            if (s < 0) continue;
            const T inc = d.pa[a][0][crd[a]] * d.dt * dw;
            T *g = d.mem[a][3 + a];
            g[slab_byte(d, a, s, crd[0], crd[1], crd[2]) / sizeof(T)] += inc;
            const int tw = slab_twin(crd[a], d.P, d.hi[a]);
            if (tw >= 0) g[slab_byte(d, a, tw, crd[0], crd[1], crd[2]) / sizeof(T)] += inc;
        }
    }
}

// Arguments of a stencil launch over the tiles of G plans of one precision (G = 1: a plan's
// own forward passes; G = kGroupMax: the grouped passes of el_group, and a plan's own
// adjoint passes as one member).  Member q owns blocks first[q] .. first[q+1]-1; each
// first[q] is a multiple of 8, so that the member's block b - first[q] runs on XCD
// (b - first[q]) % 8 as its tile order assumes.  Entries past the last member repeat the
// total block count (or lie beyond every block).  row[q]: the trace row that member's gather
// blocks write (forward velocity launch) or its adjoint stress launch scatters, or null.
constexpr int kGroupMax = 4;
template <typename T, int G>
struct Grp {
    Dev<T> d[G];
    Tiles tl[G];
    Rec r[G];
    double *row[G];
    int first[G + 1];
    int n;
};
template <typename T, int G>
__device__ __forceinline__ int member_of(const Grp<T, G> &g) {
    int q = 0;
#pragma unroll
    for (int k = 1; k < G; ++k) q += (int)blockIdx.x >= g.first[k] ? 1 : 0;
    return q;
}

// Workspace layout (byte offsets), computed identically for sizing and binding.
struct Layout {
    size_t field[NFIELD];
    size_t map[4];           // lam, mu, rho, alpha
    size_t mem[3][6];
    size_t pa[3][2], pb[3][2];
    size_t rec_idx, rec_w, rec_fl, csr_pt, csr_ptc, csr_row, csr_rec, csr_w, csr_tslot, csr_loff, csr_tpts;
    size_t stats;            // media statistics (16 doubles)
    size_t counter;          // device step counter of captured step graphs
    size_t tile_order;       // tile of each stencil block
    size_t tile_flags;       // per tile: 1 if the fluid update applies; then per tile: 1 if uniform
    size_t tile_media;       // per tile: lambda, rho, alpha, 0 (elements of the plan's precision)
    size_t tile_lanes;       // per tile and row: 64-bit masks of fluid columns, then of uniform ones
    size_t partial;          // reduction partials
    size_t energy;           // modified energy: kinetic part of each thread of the tile blocks, then
                             // kinetic and potential part of each tile block
    size_t relax_map;        // alpha_r (padded cell map), with relaxation mechanisms only
    size_t relax_flag;       // per tile: relaxation applies
    size_t relax_count;      // per tile: velocity points with beta > 0 (int)
    size_t relax_off;        // per tile: first point of the tile in the point list (long long)
    size_t relax_pts;        // point list: element index and component (unsigned), at most 3 per cell
    size_t relax_beta;       // beta of each point
    size_t relax_zeta;       // memory variables of the relaxation mechanisms (Relax::zeta)
    size_t total;
};

constexpr int kDotBlocks = 1024;
constexpr int kStats = 8;   // media statistics (launch_media_stats)

bool layout(const el_grid &g, int nrec, Layout *L);

// Launchers (return hipError_t of the launch).
template <typename T> hipError_t launch_convert_maps(const Dev<T> &d, const float *lam, const float *mu,
                                                     const float *rho, const float *alpha, hipStream_t s);
hipError_t launch_media_stats(const float *lam, const float *mu, const float *rho, const float *alpha,
                              long long n, double dt, double *stats, double *partial, hipStream_t s);
template <typename T> hipError_t launch_zero_state(const Dev<T> &d, hipStream_t s);
template <typename T> hipError_t launch_classify(const Dev<T> &d, const Tiles &tl, unsigned char *fast,
                                                 unsigned char *uni, T *med, unsigned long long *lanes,
                                                 hipStream_t s);
template <typename T> hipError_t launch_inject(const Dev<T> &d, const T *p0, hipStream_t s);
// The forward velocity launch can also gather a trace row (grow != null) from the stresses it
// reads and does not write: extra blocks after the tiles' run gather_block.
// epart != null: the launch also writes the kinetic part of the modified energy, one double per
// thread of every tile block (8 * per * kTileX * kTileY doubles); launch_energy_pot writes the
// potential part, one double per tile block; launch_energy_final sums the threads' parts per
// block into kin_block, then everything into *out.
// ctr != null (captured step graphs): a device step counter.  The velocity launch gathers row
// *ctr of the traces at grow and the stress launch then advances the counter; the adjoint
// velocity launch steps it back by one and the scatter then reads row *ctr of the traces at y.
template <typename T> hipError_t launch_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s,
                                                 const Rec *r = nullptr, double *grow = nullptr,
                                                 double *epart = nullptr, int *ctr = nullptr);
template <typename T> hipError_t launch_energy_pot(const Dev<T> &d, const Tiles &tl, double *epart, hipStream_t s);
hipError_t launch_energy_final(const double *kin_thread, double *kin_block, const double *pot, int nb, double *out,
                               hipStream_t s);
template <typename T> hipError_t launch_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s, int *ctr = nullptr);
template <typename T> hipError_t launch_gather(const Dev<T> &d, const Rec &r, double *trace_row, hipStream_t s);
template <typename T> hipError_t launch_adj_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s,
                                                     int *ctr = nullptr);
// The adjoint stress launch also applies the scatter of trace row y (r and y non-null): each
// lane, after its column's update, adds Theta^T y at the scatter points of its own cells (the
// values it has just written), in the order and arithmetic of launch_scatter.  ctr != null:
// y is the whole trace array and the row is *ctr (stepped back by the adjoint velocity launch).
template <typename T> hipError_t launch_adj_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s,
                                                   const Rec *r = nullptr, const double *y = nullptr,
                                                   int *ctr = nullptr);
template <typename T> hipError_t launch_scatter(const Dev<T> &d, const Rec &r, const double *y, hipStream_t s,
                                                const int *ctr = nullptr);
// Grouped passes (el_group): pass 0 velocity (with the gather blocks of members whose row is
// set), 1 stress, 2 adjoint velocity, 3 adjoint stress (with the scatter of members whose row
// is set); g.first from the members' 8 * per blocks (plus gather blocks for pass 0).
template <typename T> hipError_t launch_group_pass(const Grp<T, kGroupMax> &g, int pass, hipStream_t s);
template <typename T> hipError_t launch_extract(const Dev<T> &d, T *p, hipStream_t s);
template <typename T> hipError_t launch_fluid_fill(const Dev<T> &d, const Tiles &tl, hipStream_t s);
hipError_t launch_eir(const double *h, int nh, const double *in, double *out, int M, int L, int transpose,
                      hipStream_t s);
template <typename T> hipError_t launch_dot(const T *a, const T *b, long long n, double *partial, double *out,
                                            hipStream_t s);
hipError_t launch_set_counter(int *ctr, int v, hipStream_t s);
// Relaxation: statistics of the strength map (stats[0] min, [1] non-finite count, [2] max
// over the cells within `margin` of a face), its padded copy, the per-tile flags, the
// memory variables' reset, and the pointwise sub-update (ADJ: its transpose).
hipError_t launch_relax_stats(const float *ar, int nx, int ny, int nz, int margin, double *stats, double *partial,
                              hipStream_t s);
template <typename T> hipError_t launch_relax_setup(const Dev<T> &d, const Tiles &tl, const float *ar_cells,
                                                    const Relax<T> &r, hipStream_t s);
template <typename T> hipError_t launch_relax_compact(const Dev<T> &d, const Tiles &tl, const Relax<T> &r,
                                                      hipStream_t s);
template <typename T> hipError_t launch_relax_zero(const Tiles &tl, const Relax<T> &r, hipStream_t s);
template <typename T> hipError_t launch_relax(const Dev<T> &d, const Tiles &tl, const Relax<T> &r, bool adjoint,
                                              hipStream_t s);

}  // namespace el

// Host state of a plan (the opaque el_plan of the ABI).
struct el_plan_ {
    el_grid g;
    int nrec;
    long long N;
    el::Layout L;
    char *ws;
    int device;
    el::Dev<float> df;
    el::Dev<double> dd;
    el::Relax<float> rf;               // relaxation mechanisms (L = 0: none)
    el::Relax<double> rd;
    long long relax_tiles = 0;         // tiles the relaxation sub-update visits
    long long relax_cells = 0;         // and their cells
    long long relax_points = 0;        // (cell, component) velocity points with beta > 0
    el::Rec rec;
    el::Tiles tiles;
    std::vector<unsigned char> fast;   // per tile: the fluid update applies (host copy)
    std::vector<unsigned char> uni;    // per tile: fluid with uniform lambda, rho, alpha (host copy)
    std::vector<unsigned char> cols;   // per tile: not fluid, with fluid columns (host)
    long long column_cells = 0;        // cells of fluid columns in such tiles
    long long uniform_cells = 0;       // cells of uniform fluid tiles
    long long fast_tiles = 0, fast_cells = 0;
    long long fast_layer_cells = 0;    // sum over axes of fluid-tile cells in that axis's C-PML layers
    long long fast_skipped = 0;        // s22 and s33 stores a fluid stress pass leaves out
    std::vector<int> rec_tile;         // [L][8] tile of each receiver corner (host)
    bool fluid_path = true;            // use the fluid update where it applies
    hipEvent_t done;
    double cmax;
    // benchmark instrumentation: per kernel kind, event pairs and how many are in use
    int timing_every = 0;              // bracket the launches of steps m with m % timing_every == 0
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[EL_K_COUNT];
    size_t used[EL_K_COUNT] = {};
};

// The plan's relaxation parameters in the plan's precision.
template <typename T> inline el::Relax<T> &plan_relax(el_plan_ *p);
template <> inline el::Relax<float> &plan_relax<float>(el_plan_ *p) { return p->rf; }
template <> inline el::Relax<double> &plan_relax<double>(el_plan_ *p) { return p->rd; }
