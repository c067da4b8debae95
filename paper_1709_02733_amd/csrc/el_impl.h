// Internal declarations of the elastic operator library (device parameter
// block, workspace layout, kernel launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "el.h"

namespace el {

// Wavefield array ids (same order as el_plan_field).
enum Field { U1 = 0, U2, U3, S11, S22, S33, S23, S13, S12, NFIELD };

// Everything a stencil kernel needs, passed by value.
template <typename T>
struct Dev {
    int nx, ny, nz;
    long long nxy;           // nx * ny
    T dt, inv_dx;
    T *f[NFIELD];            // u1, u2, u3, s11, s22, s33, s23, s13, s12
    const T *lam, *mu, *rho, *alpha;   // cell maps
    int P;                   // C-PML cells per face, 0 = none
    int hi[3];               // first index of the high boundary slab per axis: n - 1 - P
    int W;                   // slab planes per axis: 2 (P + 1)
    const T *pa[3][2];       // PML a per axis, [0] integer / [1] half positions
    const T *pb[3][2];       // PML b
    T *mem[3][6];            // boundary-slab memory variables of axis j:
                             //   mem[j][i]     = phi^{ij} (u^i point),
                             //   mem[j][3 + i] = psi^{ij} (sigma^{ij} point)
};

// Column tiles of the stencil passes: kTileX x kTileY cells in x-y, a chunk of zc planes in z.
constexpr int kTileX = 64;
constexpr int kTileY = 8;
struct Tiles {
    int ntx, nty, nzc, zc;   // tiles along x and y, z chunks, planes per chunk
    int ntiles;              // ntx * nty * nzc
    int per;                 // tiles per XCD: the grid has 8 * per blocks
};
Tiles make_tiles(int nx, int ny, int nz);

// Receiver tables.
struct Rec {
    int nrec;
    const long long *idx;    // [L][8] corner cell indices
    const double *w;         // [L][8] trilinear weights
    // grid-point-major transpose for the deterministic scatter
    int npts;
    const long long *pt;     // [npts] touched cells
    const int *row;          // [npts + 1] offsets into ent_rec / ent_w
    const int *ent_rec;      // receiver of each entry
    const double *ent_w;     // weight of each entry
};

// Workspace layout (byte offsets), computed identically for sizing and binding.
struct Layout {
    size_t field[NFIELD];
    size_t map[4];           // lam, mu, rho, alpha
    size_t mem[3][6];
    size_t pa[3][2], pb[3][2];
    size_t rec_idx, rec_w, csr_pt, csr_row, csr_rec, csr_w;
    size_t stats;            // media statistics (16 doubles)
    size_t partial;          // reduction partials
    size_t total;
};

constexpr int kDotBlocks = 1024;

bool layout(const el_grid &g, int nrec, Layout *L);

// Launchers (return hipError_t of the launch).
template <typename T> hipError_t launch_convert_maps(const Dev<T> &d, const float *lam, const float *mu,
                                                     const float *rho, const float *alpha, hipStream_t s);
hipError_t launch_media_stats(const float *lam, const float *mu, const float *rho, const float *alpha,
                              long long n, double dt, double *stats, double *partial, hipStream_t s);
template <typename T> hipError_t launch_zero_state(const Dev<T> &d, hipStream_t s);
template <typename T> hipError_t launch_inject(const Dev<T> &d, const T *p0, hipStream_t s);
template <typename T> hipError_t launch_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s);
template <typename T> hipError_t launch_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s);
template <typename T> hipError_t launch_gather(const Dev<T> &d, const Rec &r, double *trace_row, hipStream_t s);
template <typename T> hipError_t launch_adj_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s);
template <typename T> hipError_t launch_adj_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s);
template <typename T> hipError_t launch_scatter(const Dev<T> &d, const Rec &r, const double *y_row, hipStream_t s);
template <typename T> hipError_t launch_extract(const Dev<T> &d, T *p, hipStream_t s);
template <typename T> hipError_t launch_dot(const T *a, const T *b, long long n, double *partial, double *out,
                                            hipStream_t s);

}  // namespace el
