// Host side of the C ABI declared in include/el.h: validation, workspace
// layout, C-PML profiles, receiver tables and the time loops of H and H^T.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "el_impl.h"

using namespace el;

namespace {

thread_local std::string g_err;

#define fail el::set_error

el_status hip_fail(hipError_t e, const char *what) {
    return fail(EL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                        \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// 4th-order staggered 3-D stability bound: c dt/dx <= 1 / (sqrt(3) (9/8 + 1/24)).
const double kCflMax = 6.0 / (7.0 * std::sqrt(3.0));

// Receivers may sit up to this many cells outside [0, n-1] (rounding of x/dx); they are clamped onto the box.
const double kRecSlack = 1e-9;

}  // namespace

namespace el {

el_status set_error(el_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

Vol make_vol(int nx, int ny, int nz) {
    Vol v;
    v.nx = nx;
    v.ny = ny;
    v.nz = nz;
    v.px = (nx + 2 + 31) / 32 * 32;
    v.py = ny + 2;
    v.plane = (long long)v.px * v.py;
    v.total = v.plane * (nz + 4);
    v.origin = 2 * v.plane;
    return v;
}

bool layout(const el_grid &g, int nrec, Layout *L) {
    const size_t es = g.precision == EL_F64 ? 8 : 4;
    const size_t N = (size_t)make_vol(g.nx, g.ny, g.nz).total;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int f = 0; f < NFIELD; ++f) L->field[f] = take(N * es);
    for (int m = 0; m < 4; ++m) L->map[m] = take(N * es);
    const int P = g.npml;
    const size_t W = P > 0 ? 2 * (size_t)(P + 7) : 0;
    const size_t ns[3] = {W * g.ny * g.nz, (size_t)g.nx * W * g.nz, (size_t)g.nx * g.ny * W};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 6; ++q) L->mem[a][q] = P > 0 ? take(ns[a] * es) : 0;
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h) {
            L->pa[a][h] = P > 0 ? take(n[a] * es) : 0;
            L->pb[a][h] = P > 0 ? take(n[a] * es) : 0;
        }
    const size_t E = 8 * (size_t)std::max(nrec, 1);
    L->rec_idx = take(E * 8);
    L->rec_w = take(E * 8);
    L->rec_fl = take(E);
    L->csr_pt = take(E * 8);
    L->csr_ptc = take(E * 3 * 4);
    L->csr_row = take((E + 1) * 4);
    L->csr_rec = take(E * 4);
    L->csr_w = take(E * 8);
    L->stats = take(16 * 8);
    L->counter = take(256);
    {
        const Tiles t = make_tiles(g.nx, g.ny, g.nz);
        L->csr_tslot = take((size_t)t.ntiles * 4);
        L->csr_loff = take(std::min((size_t)t.ntiles, E) * (kTileX * kTileY + 1) * 4);
        L->csr_tpts = take(E * 4);
        L->tile_order = take((size_t)8 * t.per * sizeof(int));
        L->tile_flags = take(2 * (size_t)t.ntiles);
        L->tile_media = take((size_t)4 * t.ntiles * es);
        L->tile_lanes = take((size_t)2 * kTileY * t.ntiles * 8);
        L->energy = take((size_t)(kTileX * kTileY + 2) * 8 * t.per * sizeof(double));
        const int nm = g.relax.nmech;
        L->relax_map = nm > 0 ? take(N * es) : 0;
        L->relax_flag = nm > 0 ? take((size_t)t.ntiles) : 0;
        L->relax_count = nm > 0 ? take((size_t)t.ntiles * sizeof(int)) : 0;
        const size_t cap = (size_t)t.ntiles * 3 * t.zc * kTileX * kTileY;   // points at most
        L->relax_off = nm > 0 ? take((size_t)t.ntiles * sizeof(long long)) : 0;
        L->relax_pts = nm > 0 ? take(cap * sizeof(unsigned)) : 0;
        L->relax_beta = nm > 0 ? take(cap * es) : 0;
        L->relax_zeta = nm > 0 ? take(cap * nm * es) : 0;
    }
    L->partial = take(kStats * kDotBlocks * 8);
    L->total = off;
    return true;
}

// Tiles of kTileX x kTileY columns by chunks of chunk_planes() planes.  Chunks of kZChunk
// planes where the grid has enough columns (measured at 384^3 with the fluid update and its
// pipelined loops: 6 planes beat 4 by 1.2%, 8 by 0.5% and 12 by 1.7%; short blocks keep the
// XCDs evenly loaded, long ones re-read fewer halo planes).  A small grid takes shorter
// chunks until it has kMinTiles tiles (16 blocks per compute unit): at 96^3 chunks of 2
// planes make the adjoint passes 1.5x and the forward passes 1.15x faster than chunks of 6
// (768 blocks, under three per compute unit), at 128^3 1.2x and 1.1x.
// The grid has 8 * per blocks; tile_order() says which tile each block processes.
constexpr int kZChunk = 6;
constexpr long long kMinTiles = 4096;
int chunk_planes(int nx, int ny, int nz) {
    const long long cols = (long long)((nx + kTileX - 1) / kTileX) * ((ny + kTileY - 1) / kTileY);
    int zc = kZChunk;
    while (zc > 2 && cols * ((nz + zc - 1) / zc) < kMinTiles) --zc;
    return std::min(zc, nz);
}
Tiles make_tiles(int nx, int ny, int nz) {
    Tiles t;
    t.ntx = (nx + kTileX - 1) / kTileX;
    t.nty = (ny + kTileY - 1) / kTileY;
    t.zc = chunk_planes(nx, ny, nz);
    t.nzc = (nz + t.zc - 1) / t.zc;
    t.ntiles = t.ntx * t.nty * t.nzc;
    t.order = nullptr;
    t.lanes = nullptr;
    t.per = 0;
    std::vector<int> cnt(8, 0);
    for (int q = 0; q < t.ntiles; ++q) ++cnt[tile_xcd(t, q)];
    for (int x = 0; x < 8; ++x) t.per = std::max(t.per, cnt[x]);
    return t;
}

// XCD of a tile.  With at least eight tile rows and eight z chunks, the rows and chunks are
// cut into eight bands each and region (y band, z band) goes to XCD (y band + z band) mod 8:
// a Latin square, so every XCD holds one region of every y band and of every z band (the
// same share of the C-PML layers of y and z; every region spans the x extent) and a
// region's tiles share one L2.  Smaller grids deal runs of about ntiles / 512 tiles in
// z-major order round-robin.
int tile_xcd(const Tiles &t, int q) {
    const int bx = q % t.ntx, r = q / t.ntx, by = r % t.nty, bz = r / t.nty;
    (void)bx;
    if (t.nty >= 8 && t.nzc >= 8) return (by * 8 / t.nty + bz * 8 / t.nzc) % 8;
    const int run = std::max(1, (t.ntiles + 511) / 512);
    return (q / run) % 8;
}

int tile_edges(const Tiles &t, const unsigned char *fast, int q) {
    if (!fast || !fast[q]) return 0;
    const int b[2] = {(q / t.ntx) % t.nty, q / t.ntx / t.nty};
    const int nb[2] = {t.nty, t.nzc};
    const int step[2] = {t.ntx, t.ntx * t.nty};
    int edges = 0;
    for (int a = 0; a < 2; ++a) {   // y, z
        if (b[a] > 0 && !fast[q - step[a]]) edges |= 1 << (kEdgeShift + 2 * a);
        if (b[a] + 1 < nb[a] && !fast[q + step[a]]) edges |= 1 << (kEdgeShift + 2 * a + 1);
    }
    return edges;
}

std::vector<int> tile_order(const Tiles &t, const unsigned char *fast, const unsigned char *uni,
                            const unsigned char *cols) {
    std::vector<int> order((size_t)8 * t.per, -1);
    std::vector<int> fill(8, 0);
    // tiles of an XCD in z-major order: a region's tiles are consecutive
    for (int q = 0; q < t.ntiles; ++q) {
        const int x = tile_xcd(t, q);
        const bool f = fast && fast[q];
        const int flags = f ? kFastTile | tile_edges(t, fast, q) | (uni && uni[q] ? kUniformTile : 0)
                            : (fast && cols && cols[q] ? kColumnTile : 0);
        order[(size_t)fill[x]++ * 8 + x] = q | flags;
    }
    return order;
}

}  // namespace el

extern "C" {

const char *el_version(void) { return "elastic-pact-mi355x 0.1.0 (gfx950)"; }

const char *el_status_string(el_status s) {
    switch (s) {
        case EL_OK: return "EL_OK";
        case EL_EINVAL: return "EL_EINVAL";
        case EL_EUNSTABLE: return "EL_EUNSTABLE";
        case EL_ERANGE: return "EL_ERANGE";
        case EL_ENOMEM: return "EL_ENOMEM";
        case EL_EDEVICE: return "EL_EDEVICE";
        case EL_EBUSY: return "EL_EBUSY";
        default: return "EL_UNKNOWN";
    }
}

const char *el_last_error(void) { return g_err.c_str(); }

el_status el_grid_check(const el_grid *g, const double *rec, int32_t nrec) {
    if (!g) return fail(EL_EINVAL, "grid is NULL");
    if (g->nx < 4 || g->ny < 4 || g->nz < 4)
        return fail(EL_EINVAL, "grid %dx%dx%d: every axis needs at least 4 cells", g->nx, g->ny, g->nz);
    if (!(g->dx > 0) || !std::isfinite(g->dx)) return fail(EL_EINVAL, "dx must be positive and finite");
    if (!(g->dt > 0) || !std::isfinite(g->dt)) return fail(EL_EINVAL, "dt must be positive and finite");
    if (g->nsteps < 1) return fail(EL_EINVAL, "nsteps must be >= 1");
    if (g->npml < 0) return fail(EL_EINVAL, "npml must be >= 0");
    const int n[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a)
        if (g->npml > 0 && n[a] < 2 * g->npml + 2)
            return fail(EL_EINVAL, "axis %d has %d cells, fewer than 2*npml+2 = %d", a, n[a], 2 * g->npml + 2);
    if (g->precision != EL_F32 && g->precision != EL_F64) return fail(EL_EINVAL, "precision must be EL_F32 or EL_F64");
    {
        const long long es = g->precision == EL_F64 ? 8 : 4;
        const long long bytes = make_vol(g->nx, g->ny, g->nz).total * es;
        if (bytes >= (1LL << 32))
            return fail(EL_EINVAL, "grid %dx%dx%d: one padded volume array needs %lld bytes; the kernels address at most 4 GiB per array",
                        g->nx, g->ny, g->nz, bytes);
        // the C-PML memory variables of axis a live on W = 2 (P + 7) planes of that axis
        // (slab_byte forms 32-bit byte offsets into them as well)
        if (g->npml > 0) {
            const long long W = 2LL * (g->npml + 7);
            const long long slab[3] = {W * g->ny * g->nz, W * g->nx * g->nz, W * g->nx * g->ny};
            for (int a = 0; a < 3; ++a)
                if (slab[a] * es >= (1LL << 32))
                    return fail(EL_EINVAL,
                                "grid %dx%dx%d, npml %d: a C-PML memory-variable array of axis %d needs %lld bytes; "
                                "the kernels address at most 4 GiB per array",
                                g->nx, g->ny, g->nz, g->npml, a, slab[a] * es);
        }
        const int zc = chunk_planes(g->nx, g->ny, g->nz);
        const long long tiles = (long long)((g->nx + kTileX - 1) / kTileX) * ((g->ny + kTileY - 1) / kTileY) *
                                ((g->nz + zc - 1) / zc);
        if (tiles > kTileMask)
            return fail(EL_EINVAL, "grid %dx%dx%d: %lld stencil tiles, at most %d", g->nx, g->ny, g->nz, tiles, kTileMask);
    }
    {
        const el_relaxation &rx = g->relax;
        if (rx.nmech < 0 || rx.nmech > EL_MAX_MECH)
            return fail(EL_EINVAL, "relax.nmech = %d outside 0..%d", rx.nmech, EL_MAX_MECH);
        for (int l = 0; l < rx.nmech; ++l)
            if (!(rx.omega[l] > 0) || !std::isfinite(rx.omega[l]) || !(rx.weight[l] >= 0) || !std::isfinite(rx.weight[l]))
                return fail(EL_EINVAL, "relaxation mechanism %d: omega must be > 0 and weight >= 0, both finite", l);
    }
    if (nrec < 0) return fail(EL_EINVAL, "nrec must be >= 0");
    if (nrec > (1 << 26)) return fail(EL_EINVAL, "too many receivers");
    if (nrec > 0 && !rec) return fail(EL_EINVAL, "rec_xyz is NULL");
    for (int l = 0; l < nrec; ++l)
        for (int a = 0; a < 3; ++a) {
            const double x = rec[3 * l + a] / g->dx;
            if (!(x >= -kRecSlack && x <= (double)(n[a] - 1) + kRecSlack))
                return fail(EL_ERANGE, "receiver %d axis %d at %.6g cells is outside [0, %d]", l, a, x, n[a] - 1);
        }
    return EL_OK;
}

el_status el_plan_bytes(const el_grid *g, int32_t nrec, size_t *bytes) {
    el_status st = el_grid_check(g, nullptr, 0);
    if (st != EL_OK) return st;
    if (nrec < 0) return fail(EL_EINVAL, "nrec must be >= 0");
    if (!bytes) return fail(EL_EINVAL, "bytes is NULL");
    Layout L;
    layout(*g, nrec, &L);
    *bytes = L.total;
    return EL_OK;
}

}  // extern "C"

namespace {

// C-PML profile of one axis (Appendix A.1-A.2, kappa = 1): with xi the depth into
// the layer over its thickness, measured from planes P and n-1-P and clamped to
// [0, 1], d = d0 xi^npow, beta = pi f0 (1 - xi), b = exp(-(d + beta) dt),
// a = d / (d + beta) (b - 1); a = 0 where xi = 0.
void pml_axis(const el_grid &g, int n, double d0, double f0, double npow, int half, std::vector<double> &a,
              std::vector<double> &b) {
    a.assign(n, 0.0);
    b.assign(n, 1.0);
    const int P = g.npml;
    for (int i = 0; i < n; ++i) {
        const double x = i + 0.5 * half;
        double depth = 0.0;
        if (x < P) depth = P - x;
        if (x > n - 1 - P) depth = x - (n - 1 - P);
        double xi = depth / P;
        if (xi > 1.0) xi = 1.0;
        if (xi > 0.0) {
            const double d = d0 * std::pow(xi, npow);
            const double beta = M_PI * f0 * (1.0 - xi);
            b[i] = std::exp(-(d + beta) * g.dt);
            a[i] = d / (d + beta) * (b[i] - 1.0);
        } else {
            b[i] = std::exp(-(M_PI * f0) * g.dt);
        }
    }
}

template <typename T>
void bind(Dev<T> &d, el_plan_ *p) {
    const el_grid &g = p->g;
    char *ws = p->ws;
    const Vol v = make_vol(g.nx, g.ny, g.nz);
    d.nx = g.nx;
    d.ny = g.ny;
    d.nz = g.nz;
    d.px = v.px;
    d.plane = v.plane;
    d.sy = (unsigned)(v.px * sizeof(T));
    d.sz = (unsigned)(v.plane * sizeof(T));
    d.origin = (unsigned)(v.origin * sizeof(T));
    d.dt = T(g.dt);
    d.inv_dx = T(1.0 / g.dx);
    for (int f = 0; f < NFIELD; ++f) d.f[f] = reinterpret_cast<T *>(ws + p->L.field[f]);
    d.lam = reinterpret_cast<T *>(ws + p->L.map[0]);
    d.mu = reinterpret_cast<T *>(ws + p->L.map[1]);
    d.rho = reinterpret_cast<T *>(ws + p->L.map[2]);
    d.alpha = reinterpret_cast<T *>(ws + p->L.map[3]);
    d.med = reinterpret_cast<T *>(ws + p->L.tile_media);
    d.P = g.npml;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) d.hi[a] = n[a] - 1 - g.npml;
    d.W = g.npml > 0 ? 2 * (g.npml + 7) : 0;
    for (int a = 0; a < 3; ++a) {
        for (int h = 0; h < 2; ++h) {
            d.pa[a][h] = g.npml > 0 ? reinterpret_cast<T *>(ws + p->L.pa[a][h]) : nullptr;
            d.pb[a][h] = g.npml > 0 ? reinterpret_cast<T *>(ws + p->L.pb[a][h]) : nullptr;
        }
        for (int q = 0; q < 6; ++q) d.mem[a][q] = g.npml > 0 ? reinterpret_cast<T *>(ws + p->L.mem[a][q]) : nullptr;
    }
}

// Relaxation parameters in the plan's precision: weights, c_l = exp(-omega_l dt), buffers.
template <typename T>
void bind_relax(Relax<T> &r, el_plan_ *p) {
    const el_relaxation &rx = p->g.relax;
    r = Relax<T>{};
    r.L = rx.nmech;
    for (int l = 0; l < rx.nmech; ++l) {
        r.w[l] = T(rx.weight[l]);
        r.c[l] = T(std::exp(-rx.omega[l] * p->g.dt));
    }
    if (rx.nmech > 0) {
        r.ar = reinterpret_cast<T *>(p->ws + p->L.relax_map);
        r.flag = reinterpret_cast<unsigned char *>(p->ws + p->L.relax_flag);
        r.count = reinterpret_cast<int *>(p->ws + p->L.relax_count);
        r.off = reinterpret_cast<long long *>(p->ws + p->L.relax_off);
        r.pts = reinterpret_cast<unsigned *>(p->ws + p->L.relax_pts);
        r.beta = reinterpret_cast<T *>(p->ws + p->L.relax_beta);
        r.zeta = reinterpret_cast<T *>(p->ws + p->L.relax_zeta);
    }
}

template <typename T>
el_status upload_pml(el_plan_ *p, Dev<T> &d, hipStream_t s) {
    const el_grid &g = p->g;
    if (g.npml <= 0) return EL_OK;
    const double R = g.pml_R > 0 ? g.pml_R : 1e-3;
    const double npow = g.pml_npower > 0 ? g.pml_npower : 2.0;
    const double f0 = g.pml_f0 > 0 ? g.pml_f0 : 1500.0 / (8.0 * g.dx);
    const double d0 = -(npow + 1.0) * p->cmax * std::log(R) / (2.0 * g.npml * g.dx);
    const int n[3] = {g.nx, g.ny, g.nz};
    std::vector<double> a, b;
    for (int ax = 0; ax < 3; ++ax)
        for (int h = 0; h < 2; ++h) {
            pml_axis(g, n[ax], d0, f0, npow, h, a, b);
            std::vector<T> at(a.begin(), a.end()), bt(b.begin(), b.end());
            HIP_TRY(hipMemcpyAsync(const_cast<T *>(d.pa[ax][h]), at.data(), n[ax] * sizeof(T), hipMemcpyHostToDevice, s),
                    "copy PML a");
            HIP_TRY(hipMemcpyAsync(const_cast<T *>(d.pb[ax][h]), bt.data(), n[ax] * sizeof(T), hipMemcpyHostToDevice, s),
                    "copy PML b");
            HIP_TRY(hipStreamSynchronize(s), "PML upload");
        }
    return EL_OK;
}

// Trilinear weights on the normal-stress grid (Sec. 3, eq. interpgrid): base index
// floor(x/dx) clamped to n-2, fraction x/dx - base; corner c = (c&1, c>>1&1, c>>2&1).
el_status upload_receivers(el_plan_ *p, const double *rec, hipStream_t s) {
    const el_grid &g = p->g;
    const int L = p->nrec;
    const int n[3] = {g.nx, g.ny, g.nz};
    const Vol v = make_vol(g.nx, g.ny, g.nz);
    std::vector<long long> idx(8 * (size_t)L);
    std::vector<int> cidx(3 * 8 * (size_t)L);
    std::vector<double> w(8 * (size_t)L);
    p->rec_tile.assign(8 * (size_t)L, 0);
    for (int l = 0; l < L; ++l) {
        int b[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
            const double x = std::min(std::max(rec[3 * l + a] / g.dx, 0.0), (double)(n[a] - 1));
            int bb = (int)std::floor(x);
            if (bb > n[a] - 2) bb = n[a] - 2;
            b[a] = bb;
            f[a] = x - bb;
        }
        for (int c = 0; c < 8; ++c) {
            const int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
            idx[8 * l + c] = v.origin + (long long)(b[2] + oz) * v.plane + (long long)(b[1] + oy) * v.px + (b[0] + ox);
            cidx[3 * (8 * l + c) + 0] = b[0] + ox;
            cidx[3 * (8 * l + c) + 1] = b[1] + oy;
            cidx[3 * (8 * l + c) + 2] = b[2] + oz;
            w[8 * l + c] = (ox ? f[0] : 1 - f[0]) * (oy ? f[1] : 1 - f[1]) * (oz ? f[2] : 1 - f[2]);
            const Tiles &t = p->tiles;
            p->rec_tile[8 * l + c] = ((b[2] + oz) / t.zc * t.nty + (b[1] + oy) / kTileY) * t.ntx + (b[0] + ox) / kTileX;
        }
    }
    // grid-point-major transpose: entries sorted by (cell, receiver, corner)
    std::vector<int> order(8 * (size_t)L);
    for (size_t e = 0; e < order.size(); ++e) order[e] = (int)e;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return idx[x] != idx[y] ? idx[x] < idx[y] : x < y; });
    std::vector<long long> pt;
    std::vector<int> ptc, row, erec;
    std::vector<double> ew;
    for (size_t e = 0; e < order.size(); ++e) {
        const int o = order[e];
        if (pt.empty() || pt.back() != idx[o]) {
            pt.push_back(idx[o]);
            for (int a = 0; a < 3; ++a) ptc.push_back(cidx[3 * o + a]);
            row.push_back((int)e);
        }
        erec.push_back(o / 8);
        ew.push_back(w[o]);
    }
    row.push_back((int)order.size());
    // the points of each stencil tile and column (the adjoint stress launch adds Theta^T y at
    // the cells its lanes own): sorted by (tile, column key), a slot per tile with points
    const Tiles &tt = p->tiles;
    constexpr int kKeys = kTileX * kTileY;
    std::vector<long long> tkey(pt.size());
    std::vector<int> tpts(pt.size()), tslot(tt.ntiles, -1), loff;
    for (size_t q = 0; q < pt.size(); ++q) {
        const int i = ptc[3 * q], j = ptc[3 * q + 1], k = ptc[3 * q + 2];
        const long long t = ((long long)(k / tt.zc) * tt.nty + j / kTileY) * tt.ntx + i / kTileX;
        tkey[q] = t * kKeys + (i % kTileX) + kTileX * (j % kTileY);
        tpts[q] = (int)q;
    }
    std::stable_sort(tpts.begin(), tpts.end(), [&](int a, int b) { return tkey[a] < tkey[b]; });
    for (size_t e = 0; e < tpts.size();) {
        const int t = (int)(tkey[tpts[e]] / kKeys);
        const int slot = (int)(loff.size() / (kKeys + 1));
        tslot[t] = slot;
        loff.resize(loff.size() + kKeys + 1);
        int *lo = loff.data() + (size_t)slot * (kKeys + 1);
        size_t f = e;
        for (int key = 0; key <= kKeys; ++key) {
            while (f < tpts.size() && tkey[tpts[f]] < (long long)t * kKeys + key) ++f;
            lo[key] = (int)f;
        }
        while (f < tpts.size() && tkey[tpts[f]] / kKeys == t) ++f;
        e = f;
    }
    char *ws = p->ws;
    Rec &r = p->rec;
    r.nrec = L;
    r.idx = reinterpret_cast<long long *>(ws + p->L.rec_idx);
    r.w = reinterpret_cast<double *>(ws + p->L.rec_w);
    r.fl = reinterpret_cast<unsigned char *>(ws + p->L.rec_fl);
    r.npts = (int)pt.size();
    r.pt = reinterpret_cast<long long *>(ws + p->L.csr_pt);
    r.ptc = reinterpret_cast<int *>(ws + p->L.csr_ptc);
    r.row = reinterpret_cast<int *>(ws + p->L.csr_row);
    r.ent_rec = reinterpret_cast<int *>(ws + p->L.csr_rec);
    r.ent_w = reinterpret_cast<double *>(ws + p->L.csr_w);
    r.tslot = reinterpret_cast<int *>(ws + p->L.csr_tslot);
    r.loff = reinterpret_cast<int *>(ws + p->L.csr_loff);
    r.tpts = reinterpret_cast<int *>(ws + p->L.csr_tpts);
    HIP_TRY(hipMemcpyAsync((void *)r.tslot, tslot.data(), tslot.size() * 4, hipMemcpyHostToDevice, s),
            "copy receivers");
    if (L > 0) {
        HIP_TRY(hipMemcpyAsync((void *)r.loff, loff.data(), loff.size() * 4, hipMemcpyHostToDevice, s),
                "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.tpts, tpts.data(), tpts.size() * 4, hipMemcpyHostToDevice, s),
                "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.idx, idx.data(), idx.size() * 8, hipMemcpyHostToDevice, s), "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.w, w.data(), w.size() * 8, hipMemcpyHostToDevice, s), "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.pt, pt.data(), pt.size() * 8, hipMemcpyHostToDevice, s), "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.ptc, ptc.data(), ptc.size() * 4, hipMemcpyHostToDevice, s), "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.row, row.data(), row.size() * 4, hipMemcpyHostToDevice, s), "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.ent_rec, erec.data(), erec.size() * 4, hipMemcpyHostToDevice, s),
                "copy receivers");
        HIP_TRY(hipMemcpyAsync((void *)r.ent_w, ew.data(), ew.size() * 8, hipMemcpyHostToDevice, s), "copy receivers");
    }
    HIP_TRY(hipStreamSynchronize(s), "receiver upload");
    return EL_OK;
}

// Upload the tile order table and the receiver corners' fluid flags, both with the fluid
// tiles when the fluid update is enabled and without them otherwise.
el_status upload_order(el_plan p, hipStream_t s) {
    const unsigned char *fast = p->fluid_path ? p->fast.data() : nullptr;
    const std::vector<int> order = tile_order(p->tiles, fast, p->uni.data(), p->cols.data());
    int *dst = reinterpret_cast<int *>(p->ws + p->L.tile_order);
    HIP_TRY(hipMemcpyAsync(dst, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, s), "tile order");
    std::vector<unsigned char> fl(p->rec_tile.size(), 0);
    for (size_t e = 0; e < fl.size(); ++e) fl[e] = fast && fast[p->rec_tile[e]] ? 1 : 0;
    if (!fl.empty())
        HIP_TRY(hipMemcpyAsync((void *)p->rec.fl, fl.data(), fl.size(), hipMemcpyHostToDevice, s), "receiver flags");
    HIP_TRY(hipStreamSynchronize(s), "tile order");
    p->tiles.order = dst;
    return EL_OK;
}

el_status check_plan(el_plan p) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) return fail(EL_EINVAL, "current device %d is not the plan's device %d", dev, p->device);
    return EL_OK;
}

// Launch one kernel of time step m, bracketed by an event pair when timing samples that step.
template <typename F>
hipError_t timed(el_plan p, int kind, int m, hipStream_t s, F launch) {
    if (p->timing_every <= 0 || m % p->timing_every != 0) return launch();
    auto &v = p->ev[kind];
    if (p->used[kind] == v.size()) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        v.emplace_back(a, b);
    }
    auto &pr = v[p->used[kind]++];
    hipError_t e = hipEventRecord(pr.first, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    return hipEventRecord(pr.second, s);
}

// energy != null: also the modified energy E_{m-1} = (kinetic + potential) / 2 of every
// `every`-th level m - 1, formed during update m (the velocity pass, which turns u_{m-3/2}
// into u_{m-1/2} while sigma_{m-1} stays in place) into energy[(m - 1) / every].
template <typename T>
el_status run_forward(el_plan p, Dev<T> &d, const T *p0, double *traces, hipStream_t s, int every = 0,
                      double *energy = nullptr) {
    const int M = p->g.nsteps, L = p->nrec;
    const int nb = 8 * p->tiles.per;
    double *ekin = reinterpret_cast<double *>(p->ws + p->L.energy);   // per thread
    double *ekb = ekin + (size_t)nb * kTileX * kTileY;                 // per block
    double *epot = ekb + nb;
    const Relax<T> &rx = plan_relax<T>(p);
    HIP_TRY(launch_zero_state(d, s), "zero state");
    HIP_TRY(launch_relax_zero(p->tiles, rx, s), "relaxation state");
    HIP_TRY(launch_inject(d, p0, s), "inject");
    // trace row m-1 is gathered by extra blocks of velocity pass m (which reads those stresses
    // and writes none); the last row by a gather launch of its own
    for (int m = 1; m < M; ++m) {
        double *row = traces + (size_t)(m - 1) * L;
        const bool en = energy && (m - 1) % every == 0;
        if (en) HIP_TRY(launch_energy_pot(d, p->tiles, epot, s), "potential energy");
        HIP_TRY(timed(p, EL_K_VELOCITY, m, s,
                      [&] { return launch_velocity(d, p->tiles, s, &p->rec, row, en ? ekin : nullptr); }),
                "velocity pass");
        if (en) HIP_TRY(launch_energy_final(ekin, ekb, epot, nb, energy + (m - 1) / every, s), "energy");
        if (rx.L > 0)
            HIP_TRY(timed(p, EL_K_RELAX, m, s, [&] { return launch_relax(d, p->tiles, rx, false, s); }), "relaxation");
        HIP_TRY(timed(p, EL_K_STRESS, m, s, [&] { return launch_stress(d, p->tiles, s); }), "stress pass");
    }
    HIP_TRY(timed(p, EL_K_GATHER, M - 1, s, [&] { return launch_gather(d, p->rec, traces + (size_t)(M - 1) * L, s); }),
            "gather");
    if (p->fluid_path && p->fast_tiles > 0) HIP_TRY(launch_fluid_fill(d, p->tiles, s), "fluid fill");
    return EL_OK;
}

template <typename T>
el_status run_adjoint(el_plan p, Dev<T> &d, const double *y, T *out, hipStream_t s) {
    const int M = p->g.nsteps, L = p->nrec;
    const Relax<T> &rx = plan_relax<T>(p);
    HIP_TRY(launch_zero_state(d, s), "zero state");
    HIP_TRY(launch_relax_zero(p->tiles, rx, s), "relaxation state");
    HIP_TRY(timed(p, EL_K_SCATTER, M - 1, s, [&] { return launch_scatter(d, p->rec, y + (size_t)(M - 1) * L, s); }),
            "scatter");
    for (int m = M - 1; m >= 1; --m) {
        HIP_TRY(timed(p, EL_K_ADJ_VELOCITY, m, s, [&] { return launch_adj_velocity(d, p->tiles, s); }),
                "adjoint velocity pass");
        // the transposed relaxation sits between the transposed stress and velocity updates of
        // the step (the forward applies R between its velocity and stress updates)
        if (rx.L > 0)
            HIP_TRY(timed(p, EL_K_RELAX, m, s, [&] { return launch_relax(d, p->tiles, rx, true, s); }), "relaxation");
        // the adjoint stress launch also adds Theta^T y of row m-1 (launch_adj_stress)
        HIP_TRY(timed(p, EL_K_ADJ_STRESS, m, s,
                      [&] { return launch_adj_stress(d, p->tiles, s, &p->rec, y + (size_t)(m - 1) * L); }),
                "adjoint stress pass");
    }
    if (p->fluid_path && p->fast_tiles > 0) HIP_TRY(launch_fluid_fill(d, p->tiles, s), "fluid fill");
    HIP_TRY(launch_extract(d, out, s), "extract");
    return EL_OK;
}

}  // namespace

extern "C" {

el_status el_plan_create(el_plan *out, const el_grid *grid, const float *lam, const float *mu, const float *rho,
                         const float *alpha, const float *alpha_r, const double *rec, int32_t nrec, void *workspace,
                         size_t workspace_bytes, void *stream) {
    if (!out) return fail(EL_EINVAL, "out is NULL");
    *out = nullptr;
    el_status st = el_grid_check(grid, rec, nrec);
    if (st != EL_OK) return st;
    if (!lam || !mu || !rho || !alpha) return fail(EL_EINVAL, "a material map is NULL");
    if (grid->relax.nmech > 0 && !alpha_r) return fail(EL_EINVAL, "alpha_r is NULL with relaxation mechanisms");
    if (!workspace) return fail(EL_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(EL_EINVAL, "workspace is not 256-byte aligned");
    Layout L;
    layout(*grid, nrec, &L);
    if (workspace_bytes < L.total)
        return fail(EL_ENOMEM, "workspace has %zu bytes, the plan needs %zu", workspace_bytes, L.total);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");

    el_plan_ *p = new el_plan_();
    p->g = *grid;
    p->nrec = nrec;
    p->N = (long long)grid->nx * grid->ny * grid->nz;
    p->L = L;
    p->ws = static_cast<char *>(workspace);
    p->device = dev;
    p->tiles = make_tiles(grid->nx, grid->ny, grid->nz);
    auto bail = [&](el_status e) {
        if (p->done) (void)hipEventDestroy(p->done);
        delete p;
        return e;
    };

    // media checks on the device, in double
    double *stats = reinterpret_cast<double *>(p->ws + L.stats);
    double *partial = reinterpret_cast<double *>(p->ws + L.partial);
    hipError_t e = launch_media_stats(lam, mu, rho, alpha, p->N, grid->dt, stats, partial, s);
    if (e != hipSuccess) return bail(hip_fail(e, "media statistics"));
    double hs[kStats];
    e = hipMemcpyAsync(hs, stats, sizeof hs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "media statistics"));
    if (hs[6] > 0) return bail(fail(EL_EINVAL, "%.0f non-finite material values", hs[6]));
    if (!(hs[1] > 0)) return bail(fail(EL_EINVAL, "rho must be > 0 (min %.6g)", hs[1]));
    if (hs[2] < 0) return bail(fail(EL_EINVAL, "mu must be >= 0 (min %.6g)", hs[2]));
    if (!(hs[3] > 0)) return bail(fail(EL_EINVAL, "lambda + 2 mu must be > 0 (min %.6g)", hs[3]));
    // a positive bulk modulus (Sec. 2.1): the adjoint state w = C s divides by 3 lambda + 2 mu
    if (!(hs[7] > 0)) return bail(fail(EL_EINVAL, "3 lambda + 2 mu must be > 0 (min %.6g)", hs[7]));
    if (hs[5] < 0 || hs[4] >= 1.0)
        return bail(fail(EL_EUNSTABLE, "dt*alpha must lie in [0, 1) (range %.6g .. %.6g)", hs[5], hs[4]));
    p->cmax = std::sqrt(hs[0]);
    const double cfl = p->cmax * grid->dt / grid->dx;
    if (cfl > kCflMax)
        return bail(fail(EL_EUNSTABLE, "CFL c_max dt/dx = %.6g exceeds the 4th-order staggered limit %.6g", cfl, kCflMax));
    if (grid->relax.nmech > 0) {
        // alpha_r: finite, >= 0, and zero within npml + 2 cells of a face
        const int margin = grid->npml > 0 ? grid->npml + 2 : 0;
        e = launch_relax_stats(alpha_r, grid->nx, grid->ny, grid->nz, margin, stats + 8, partial, s);
        double rs[3] = {0, 0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(rs, stats + 8, sizeof rs, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(hip_fail(e, "relaxation strength statistics"));
        if (rs[1] > 0) return bail(fail(EL_EINVAL, "%.0f non-finite alpha_r values", rs[1]));
        if (rs[0] < 0) return bail(fail(EL_EINVAL, "alpha_r must be >= 0 (min %.6g)", rs[0]));
        if (rs[2] > 0)
            return bail(fail(EL_EINVAL, "alpha_r must be 0 within npml + 2 = %d cells of a face (max there %.6g)",
                             margin, rs[2]));
    }

    e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) return bail(hip_fail(e, "event"));
    if (grid->precision == EL_F64) {
        bind(p->dd, p);
        bind_relax(p->rd, p);
        e = launch_convert_maps(p->dd, lam, mu, rho, alpha, s);
        if (e == hipSuccess && p->rd.L > 0) e = launch_relax_setup(p->dd, p->tiles, alpha_r, p->rd, s);
        if (e != hipSuccess) return bail(hip_fail(e, "copy maps"));
        st = upload_pml(p, p->dd, s);
    } else {
        bind(p->df, p);
        bind_relax(p->rf, p);
        e = launch_convert_maps(p->df, lam, mu, rho, alpha, s);
        if (e == hipSuccess && p->rf.L > 0) e = launch_relax_setup(p->df, p->tiles, alpha_r, p->rf, s);
        if (e != hipSuccess) return bail(hip_fail(e, "copy maps"));
        st = upload_pml(p, p->df, s);
    }
    if (st != EL_OK) return bail(st);
    if (grid->relax.nmech > 0 && p->tiles.ntiles > 0) {
        std::vector<unsigned char> rflag(p->tiles.ntiles, 0);
        std::vector<int> rcount(p->tiles.ntiles, 0);
        e = hipMemcpyAsync(rflag.data(), p->ws + L.relax_flag, rflag.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rcount.data(), p->ws + L.relax_count, rcount.size() * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(hip_fail(e, "relaxation tiles"));
        const Tiles &t = p->tiles;
        // the point list: the points of tile q start at roff[q] (tiles in index order)
        std::vector<long long> roff(t.ntiles, 0);
        long long npts = 0;
        for (int q = 0; q < t.ntiles; ++q) {
            roff[q] = npts;
            if (!rflag[q]) continue;
            const int bx = q % t.ntx, r = q / t.ntx, by = r % t.nty, bz = r / t.nty;
            p->relax_tiles += 1;
            p->relax_points += rcount[q];
            npts += rcount[q];
            p->relax_cells += (long long)std::min(kTileX, grid->nx - bx * kTileX) * std::min(kTileY, grid->ny - by * kTileY) *
                              std::min(t.zc, grid->nz - bz * t.zc);
        }
        // a point keeps its element index in 30 bits
        const long long elements = (long long)(grid->precision == EL_F64 ? p->dd.plane : p->df.plane) * (grid->nz + 4);
        if (elements > (long long)kRelaxElemMask + 1)
            return bail(fail(EL_EINVAL, "relaxation needs a padded grid of at most 2^30 elements (%lld)", elements));
        e = hipMemcpyAsync(p->ws + L.relax_off, roff.data(), roff.size() * sizeof(long long), hipMemcpyHostToDevice, s);
        p->rf.npts = p->rd.npts = npts;
        if (e == hipSuccess)
            e = grid->precision == EL_F64 ? launch_relax_compact(p->dd, t, p->rd, s) : launch_relax_compact(p->df, t, p->rf, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(hip_fail(e, "relaxation point list"));
    }
    st = upload_receivers(p, rec, s);
    if (st != EL_OK) return bail(st);
    {
        // fluid tiles (el_kernels.hip, k_classify), then the order table
        unsigned char *flags = reinterpret_cast<unsigned char *>(p->ws + L.tile_flags);
        unsigned char *uflags = flags + p->tiles.ntiles;
        unsigned long long *lanes = reinterpret_cast<unsigned long long *>(p->ws + L.tile_lanes);
        p->tiles.lanes = lanes;
        e = grid->precision == EL_F64
                ? launch_classify(p->dd, p->tiles, flags, uflags, const_cast<double *>(p->dd.med), lanes, s)
                : launch_classify(p->df, p->tiles, flags, uflags, const_cast<float *>(p->df.med), lanes, s);
        p->fast.assign(p->tiles.ntiles, 0);
        p->uni.assign(p->tiles.ntiles, 0);
        p->cols.assign(p->tiles.ntiles, 0);
        std::vector<unsigned long long> hl((size_t)2 * kTileY * p->tiles.ntiles, 0);
        if (e == hipSuccess && p->tiles.ntiles > 0)
            e = hipMemcpyAsync(hl.data(), lanes, hl.size() * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && p->tiles.ntiles > 0)
            e = hipMemcpyAsync(p->fast.data(), flags, p->fast.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && p->tiles.ntiles > 0)
            e = hipMemcpyAsync(p->uni.data(), uflags, p->uni.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bail(hip_fail(e, "fluid tiles"));
        const Tiles &t = p->tiles;
        const int P = grid->npml;
        const int n[3] = {grid->nx, grid->ny, grid->nz};
        // cells c of [c0, c1) in the layers of an axis of n cells (depth > 0: c < P or c > n-1-P)
        auto in_layers = [P](int c0, int c1, int nn) {
            if (P <= 0) return 0;
            const int lo = std::max(0, std::min(c1, P) - c0);
            const int hi = std::max(0, c1 - std::max(c0, nn - P));
            return lo + hi;
        };
        for (int q = 0; q < t.ntiles; ++q) {
            if (!p->fast[q]) {
                // fluid columns of a general tile: all their cells take the fluid update
                const int bx = q % t.ntx, r = q / t.ntx, by = r % t.nty, bz = r / t.nty;
                const int z0 = bz * t.zc, dep = std::min(t.zc, n[2] - z0);
                for (int row = 0; row < kTileY; ++row) {
                    const unsigned long long m = hl[(size_t)kTileY * q + row];
                    if (!m) continue;
                    p->cols[q] = 1;
                    const unsigned long long um = hl[(size_t)kTileY * ((size_t)t.ntiles + q) + row];
                    p->uniform_cells += (long long)__builtin_popcountll(um) * dep;
                    for (int b = 0; b < 64; ++b) {
                        if (!((m >> b) & 1ull)) continue;
                        const int i = bx * kTileX + b, j = by * kTileY + row;
                        p->column_cells += dep;
                        p->fast_layer_cells += (long long)in_layers(i, i + 1, n[0]) * dep +
                                               (long long)in_layers(j, j + 1, n[1]) * dep + in_layers(z0, z0 + dep, n[2]);
                    }
                }
                continue;
            }
            const int bx = q % t.ntx, r = q / t.ntx, by = r % t.nty, bz = r / t.nty;
            const int c0[3] = {bx * kTileX, by * kTileY, bz * t.zc};
            const int w[3] = {std::min(kTileX, n[0] - c0[0]), std::min(kTileY, n[1] - c0[1]), std::min(t.zc, n[2] - c0[2])};
            p->fast_tiles += 1;
            p->fast_cells += (long long)w[0] * w[1] * w[2];
            if (p->uni[q]) p->uniform_cells += (long long)w[0] * w[1] * w[2];
            for (int a = 0; a < 3; ++a)
                p->fast_layer_cells += (long long)in_layers(c0[a], c0[a] + w[a], n[a]) * w[(a + 1) % 3] * w[(a + 2) % 3];
            // s22 (s33) is stored only on two-cell bands along y (z) faces next to general tiles
            const int edges = tile_edges(t, p->fast.data(), q) >> kEdgeShift;
            for (int a = 1; a < 3; ++a) {
                const int lo = (edges >> (2 * (a - 1))) & 1, hi = (edges >> (2 * (a - 1) + 1)) & 1;
                p->fast_skipped += (long long)std::max(0, w[a] - 2 * lo - 2 * hi) * w[(a + 1) % 3] * w[(a + 2) % 3];
            }
        }
        st = upload_order(p, s);
        if (st != EL_OK) return bail(st);
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "plan set-up"));
    e = hipEventRecord(p->done, s);
    if (e != hipSuccess) return bail(hip_fail(e, "event"));
    *out = p;
    return EL_OK;
}

el_status el_plan_destroy(el_plan p) {
    if (!p) return EL_OK;
    if (p->done) (void)hipEventDestroy(p->done);
    for (auto &v : p->ev)
        for (auto &pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete p;
    return EL_OK;
}

el_status el_plan_timing(el_plan p, int32_t every) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    if (every < 0) return fail(EL_EINVAL, "every must be >= 0");
    p->timing_every = every;
    return EL_OK;
}

el_status el_plan_kernel_time(el_plan p, int32_t kind, int64_t *launches, double *total_ms) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    if (kind < 0 || kind >= EL_K_COUNT) return fail(EL_EINVAL, "kernel kind %d outside 0..%d", kind, EL_K_COUNT - 1);
    double ms = 0.0;
    const size_t n = p->used[kind];
    for (size_t q = 0; q < n; ++q) {
        auto &pr = p->ev[kind][q];
        HIP_TRY(hipEventSynchronize(pr.second), "wait for timing event");
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second), "elapsed time");
        ms += t;
    }
    p->used[kind] = 0;
    if (launches) *launches = (int64_t)n;
    if (total_ms) *total_ms = ms;
    return EL_OK;
}

el_status el_forward(el_plan p, const void *p0, double *traces, void *stream) {
    el_status st = check_plan(p);
    if (st != EL_OK) return st;
    if (!p0 || (!traces && p->nrec > 0)) return fail(EL_EINVAL, "p0 or traces is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamWaitEvent(s, p->done, 0), "order after the previous operation");
    st = p->g.precision == EL_F64 ? run_forward(p, p->dd, static_cast<const double *>(p0), traces, s)
                                  : run_forward(p, p->df, static_cast<const float *>(p0), traces, s);
    if (st != EL_OK) return st;
    HIP_TRY(hipEventRecord(p->done, s), "record completion");
    return EL_OK;
}

el_status el_forward_energy(el_plan p, const void *p0, double *traces, int32_t every, double *energy, void *stream) {
    el_status st = check_plan(p);
    if (st != EL_OK) return st;
    if (!p0 || (!traces && p->nrec > 0)) return fail(EL_EINVAL, "p0 or traces is NULL");
    if (every < 1) return fail(EL_EINVAL, "every must be >= 1");
    if (!energy && p->g.nsteps > 1) return fail(EL_EINVAL, "energy is NULL");
    if (p->g.relax.nmech > 0)
        return fail(EL_EINVAL, "the modified energy is not defined with relaxation mechanisms (their memory variables "
                               "hold energy it does not count)");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamWaitEvent(s, p->done, 0), "order after the previous operation");
    st = p->g.precision == EL_F64
             ? run_forward(p, p->dd, static_cast<const double *>(p0), traces, s, every, energy)
             : run_forward(p, p->df, static_cast<const float *>(p0), traces, s, every, energy);
    if (st != EL_OK) return st;
    HIP_TRY(hipEventRecord(p->done, s), "record completion");
    return EL_OK;
}

el_status el_adjoint(el_plan p, const double *y, void *p_adj, void *stream) {
    el_status st = check_plan(p);
    if (st != EL_OK) return st;
    if ((!y && p->nrec > 0) || !p_adj) return fail(EL_EINVAL, "y or p_adj is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamWaitEvent(s, p->done, 0), "order after the previous operation");
    st = p->g.precision == EL_F64 ? run_adjoint(p, p->dd, y, static_cast<double *>(p_adj), s)
                                  : run_adjoint(p, p->df, y, static_cast<float *>(p_adj), s);
    if (st != EL_OK) return st;
    HIP_TRY(hipEventRecord(p->done, s), "record completion");
    return EL_OK;
}

el_status el_eir_apply(const double *h, int32_t nh, const double *in, double *out, int32_t nsteps, int32_t nrec,
                       int32_t transpose, void *stream) {
    if (!h || !in || !out) return fail(EL_EINVAL, "h, in or out is NULL");
    if (nh < 1) return fail(EL_EINVAL, "nh must be >= 1");
    if (nsteps < 1 || nrec < 0) return fail(EL_EINVAL, "nsteps must be >= 1 and nrec >= 0");
    if (transpose != 0 && transpose != 1) return fail(EL_EINVAL, "transpose must be 0 or 1");
    const char *a0 = reinterpret_cast<const char *>(in), *b0 = reinterpret_cast<const char *>(out);
    const size_t bytes = (size_t)nsteps * nrec * sizeof(double);
    if (bytes > 0 && a0 < b0 + bytes && b0 < a0 + bytes) return fail(EL_EINVAL, "in and out overlap");
    if ((size_t)nsteps * (size_t)nrec > (size_t)INT32_MAX * 64) return fail(EL_EINVAL, "traces too large");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_eir(h, nh, in, out, nsteps, nrec, transpose, s), "transducer response");
    return EL_OK;
}

el_status el_dot_f64(el_plan p, int32_t space, const void *a, const void *b, double *out, void *stream) {
    el_status st = check_plan(p);
    if (st != EL_OK) return st;
    if (!a || !b || !out) return fail(EL_EINVAL, "a, b or out is NULL");
    if (space != 0 && space != 1) return fail(EL_EINVAL, "space must be 0 (N) or 1 (LM)");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamWaitEvent(s, p->done, 0), "order after the previous operation");
    double *partial = reinterpret_cast<double *>(p->ws + p->L.partial);
    hipError_t e;
    if (space == 1)
        e = launch_dot(static_cast<const double *>(a), static_cast<const double *>(b),
                       (long long)p->g.nsteps * p->nrec, partial, out, s);
    else if (p->g.precision == EL_F64)
        e = launch_dot(static_cast<const double *>(a), static_cast<const double *>(b), p->N, partial, out, s);
    else
        e = launch_dot(static_cast<const float *>(a), static_cast<const float *>(b), p->N, partial, out, s);
    if (e != hipSuccess) return hip_fail(e, "dot");
    HIP_TRY(hipEventRecord(p->done, s), "record completion");
    return EL_OK;
}

el_status el_plan_field(el_plan p, int32_t id, void **ptr, size_t *count) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    if (id < 0 || id >= NFIELD) return fail(EL_EINVAL, "field id %d outside 0..8", id);
    if (!ptr || !count) return fail(EL_EINVAL, "ptr or count is NULL");
    *ptr = p->ws + p->L.field[id];
    *count = (size_t)make_vol(p->g.nx, p->g.ny, p->g.nz).total;
    return EL_OK;
}

el_status el_plan_layout(el_plan p, int64_t *row_pitch, int64_t *plane_pitch, int64_t *origin) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    const Vol v = make_vol(p->g.nx, p->g.ny, p->g.nz);
    if (row_pitch) *row_pitch = v.px;
    if (plane_pitch) *plane_pitch = v.plane;
    if (origin) *origin = v.origin;
    return EL_OK;
}

el_status el_plan_fluid_path(el_plan p, int32_t enable, el_fluid_stats *stats) {
    el_status st = check_plan(p);
    if (st != EL_OK) return st;
    if (enable != -1 && enable != 0 && enable != 1) return fail(EL_EINVAL, "enable must be -1, 0 or 1");
    if (enable >= 0 && (enable != 0) != p->fluid_path) {
        HIP_TRY(hipEventSynchronize(p->done), "wait for the plan's previous operation");
        p->fluid_path = enable != 0;
        st = upload_order(p, nullptr);
        if (st != EL_OK) return st;
    }
    if (stats) {
        *stats = el_fluid_stats{};
        if (p->fluid_path) {
            stats->tiles = p->fast_tiles;
            stats->cells = p->fast_cells + p->column_cells;
            stats->column_cells = p->column_cells;
            stats->layer_cells = p->fast_layer_cells;
            stats->skipped_stores = p->fast_skipped;
            stats->uniform_cells = p->uniform_cells;
        }
    }
    return EL_OK;
}

el_status el_plan_relaxation(el_plan p, int64_t *tiles, int64_t *cells, int64_t *points) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    if (tiles) *tiles = p->relax_tiles;
    if (cells) *cells = p->relax_cells;
    if (points) *points = p->relax_points;
    return EL_OK;
}

el_status el_plan_sizes(el_plan p, int64_t *ncells, int32_t *nrec, int32_t *nsteps) {
    if (!p) return fail(EL_EINVAL, "plan is NULL");
    if (ncells) *ncells = p->N;
    if (nrec) *nrec = p->nrec;
    if (nsteps) *nsteps = p->g.nsteps;
    return EL_OK;
}

}  // extern "C"
