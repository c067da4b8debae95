// Stencil passes of the forward operator H and of its adjoint H^T (gfx950).
//
// One time step is two passes.  Both operators use the same two shapes:
//
//  velocity-shaped  out^c = J_c out^c + k_c sum_a D_a[In_ca]          (c = component, a = axis)
//  stress-shaped    out   = out + C Eps[In]                          (C = Voigt stiffness)
//
// Forward (Appendix, Discrete formulation; Sec. 2.2 eq. it):
//   velocity: In_ca = sigma^{ca}, k_c = dt / rho_c; the C-PML memory variable
//             phi^{ca} <- b_a phi^{ca} + a_a D_a sigma^{ca} is formed at the output
//             point and added to the sum.
//   stress:   In_ca = u^c, C scaled by dt; psi^{ca} <- b_a psi^{ca} + a_a D_a u^c
//             is added to each strain term.
// Adjoint, in the variables r = Q^{-1} q (velocity adjoint over the staggered
// density) and w = C s (stiffness times stress adjoint).  One adjoint step
// applies the transposes of the four forward sub-updates in reverse order,
// with the diagonal factors J, B, B~ of each step deferred to the next one:
//   velocity: In_ca = dt w_(ca) + a_a psi~^{ca}, k_c = -1 / rho_c, then
//             phi~^{ca} <- b_a phi~^{ca} + dt chi_a r^c at the output point;
//   stress:   In_ca = dt r^c + a_a phi~^{ca}, C scaled by -1, then
//             psi~^{ca} <- b_a psi~^{ca} + dt w_(ca) at the output point.
// The adjoint stores its memory variables multiplied by the layer coefficient,
// g = a psi~ and g = a phi~ (b and a are diagonal, so g <- b g + a dt w).
// These follow from Psi^T = -dt Div C, Phi^T = -dt Eps Q^{-1} and the
// zero-extended identity Dp^T = -Dm between the two difference types.  The
// difference of In is evaluated as dt D[w] (or dt D[r]) plus, only where a
// tap reaches a C-PML slab of that axis, D[g] on the extended slab planes.
//
// Tiling: a block owns a 64 x 4 column tile (four wavefronts of 32 x 2 cells) and each
// thread marches along z through a chunk of planes of its own column.
// Inputs differentiated along z sit in four-deep register queues; taps along
// x and y are read from memory, where the neighbouring rows of the tile and
// the tiles processed next to it keep them in L1/L2.  There is no LDS and no
// barrier.  The padded volume layout (see el_impl.h) makes every tap a plain
// load: addresses are a 32-bit byte offset, shared by all fields, from the
// field's base pointer.  Each block reads its tile from an order table (built
// by tile_order on the host) that gives every XCD (block id mod 8) contiguous
// regions of tiles spread over the volume, so every XCD holds the same share of
// the C-PML layers and a region's neighbouring tiles share one L2.
//
// Fluid tiles (marked in the order table, see k_classify): where mu = 0 on the
// tile and within two cells of it, s22 = s33 = s11 and the shear stresses are
// zero on every tap, so both passes run a lean loop that differences s11
// alone and carries only the diagonal memory variables.  s22 and s33 are read
// only by the general loop, which differences s22 along y and s33 along z with
// taps reaching two cells into a neighbouring tile, so the lean stress loop
// stores s22 only on two-row bands along y faces shared with general tiles and
// s33 only on two-plane bands along such z faces (edge bits of the order
// entry), s11 everywhere; k_fluid_fill restores s22 = s33 = s11 on fluid tiles
// at the end of an operation.  Fluid tiles of uniform media take lambda, rho
// and alpha from a per-tile table.  Inside the other tiles, fluid columns are
// marked per lane: a wavefront of fluid columns runs the lean loop, and the
// fluid lanes of a mixed wavefront run the general loop with the loads they do
// not need masked off.  The results are those of the general loop.
#include "el_impl.h"

namespace el {

constexpr int TX = kTileX;
constexpr int TY = kTileY;
constexpr int NT = TX * TY;

template <typename T>
__device__ __forceinline__ T ldb(const T *base, unsigned off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T>
__device__ __forceinline__ void stb(T *base, unsigned off, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

// Load unless off (then zero): the load is issued under the lane mask, so lanes that do not
// need the value move no bytes.
template <typename T>
__device__ __forceinline__ T ld_if(bool on, const T *base, unsigned off) {
    T v = T(0);
    if (on) v = ldb(base, off);
    return v;
}
// Load unless off (then alt), under the lane mask likewise.
template <typename T>
__device__ __forceinline__ T ld_or(bool on, const T *base, unsigned off, T alt) {
    T v = alt;
    if (on) v = ldb(base, off);
    return v;
}

// Cells of a wavefront.  A tile's four wavefronts each cover kWaveX columns of kWaveY rows
// (32 x 2): one 128-byte line of each of two rows per load, as coalesced as a 64 x 1 row,
// while a wavefront that meets a solid region holds half as many fluid columns that must run
// the general loop with it (the shell of the skull medium crosses most 64-wide rows of the
// tiles it touches).
constexpr int kWaveX = 32;
constexpr int kWaveY = 64 / kWaveX;
static_assert(TX % kWaveX == 0 && TY % kWaveY == 0 && (TX / kWaveX) * (TY / kWaveY) == NT / 64,
              "a tile is covered by its wavefronts");
// Column (i - x0) and row (j - y0) of this thread's cell within its tile.
__device__ __forceinline__ int tile_col() {
    return ((int)threadIdx.x >> 6) % (TX / kWaveX) * kWaveX + ((int)threadIdx.x & 63) % kWaveX;
}
__device__ __forceinline__ int tile_row() {
    return ((int)threadIdx.x >> 6) / (TX / kWaveX) * kWaveY + ((int)threadIdx.x & 63) / kWaveX;
}

// Fluid columns of a general tile (Tiles::lanes).  fl: this lane's column is fluid; ul: its
// lambda, rho and alpha are the tile's reference medium (in the per-tile table).  Returns
// true for a wavefront whose columns inside the grid are all fluid, which runs the fluid loop
// (uniform when every such column is, rowuni); in a mixed wavefront the fluid lanes run the
// general loop with the loads they do not need masked off (their shear taps are zero, and
// s22 = s33 = s11 on their taps).
__device__ __forceinline__ bool fluid_row(const Tiles &tl, int t, int x0, int y0, int nx, int ny, bool cols, bool &fl,
                                          bool &ul, bool &rowuni) {
    fl = ul = rowuni = false;
    if (!cols) return false;
    const int col = tile_col(), row = tile_row();
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);   // uniform: scalar mask loads
    const int wx = wave % (TX / kWaveX), wy = wave / (TX / kWaveX);
    const int nv = min(TX, nx - x0);
    const unsigned long long inx = nv >= 64 ? ~0ull : ((1ull << nv) - 1ull);
    const unsigned long long seg = (kWaveX == 64 ? ~0ull : ((1ull << kWaveX) - 1ull)) << (wx * kWaveX);
    bool all = true, alluni = true;
#pragma unroll
    for (int r = wy * kWaveY; r < (wy + 1) * kWaveY; ++r) {
        const unsigned long long m = tl.lanes[kTileY * t + r];
        const unsigned long long um = tl.lanes[kTileY * ((size_t)tl.ntiles + t) + r];
        const unsigned long long valid = y0 + r < ny ? (inx & seg) : 0ull;
        all = all && (m & valid) == valid;
        alluni = alluni && (um & valid) == valid;
        if (r == row) {
            fl = ((m >> col) & 1ull) != 0;
            ul = ((um >> col) & 1ull) != 0;
        }
    }
    rowuni = alluni;
    return all;
}

// 4th-order staggered differences (Sec. 2.2, eq. derivative):
//   Dp: value at i + 1/2 from samples i-1, i, i+1, i+2;  Dm: value at i from samples i-2 .. i+1.
template <typename T>
__device__ __forceinline__ T dplus(T fm1, T f0, T f1, T f2, T h) {
    return (T(9) / T(8) * (f1 - f0) + T(-1) / T(24) * (f2 - fm1)) * h;
}
template <typename T>
__device__ __forceinline__ T dminus(T fm2, T fm1, T f0, T f1, T h) {
    return (T(9) / T(8) * (f0 - fm1) + T(-1) / T(24) * (f1 - fm2)) * h;
}
template <typename T>
__device__ __forceinline__ T dp_at(const T *f, unsigned o, unsigned s, T h) {
    return dplus(ldb(f, o - s), ldb(f, o), ldb(f, o + s), ldb(f, o + 2 * s), h);
}
template <typename T>
__device__ __forceinline__ T dm_at(const T *f, unsigned o, unsigned s, T h) {
    return dminus(ldb(f, o - 2 * s), ldb(f, o - s), ldb(f, o), ldb(f, o + s), h);
}

// Memory-variable parts of the nine adjoint stencil inputs along axis A, for a cell whose
// stencil reaches a layer of that axis (slab coordinate sn): the premultiplied variables
// g = a m are differenced with the same tap type as the main input.  VEL selects the
// velocity-shaped pass (g = a psi~, Dp where c == A) or the stress-shaped pass (g = a phi~,
// Dm where c == A).
template <typename T, bool VEL, int A>
__device__ __forceinline__ void add_pml_axis(const Dev<T> &d, T (&dd)[3][3], int sn, int i, int j, int k, T h) {
    const unsigned off = slab_byte(d, A, sn, i, j, k), st = slab_stride(d, A);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T *g = VEL ? d.mem[A][3 + c] : d.mem[A][c];
        dd[c][A] += (VEL == (c == A)) ? dp_at(g, off, st, h) : dm_at(g, off, st, h);
    }
}

// Reciprocal: the hardware v_rcp_f32 (within 1 ulp) in single precision, the correctly
// rounded quotient in double precision.  Both give +inf for +0 and 0 for +inf.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ float rcp<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double rcp<double>(double x) {
    return 1.0 / x;
}

// Harmonic mean of four non-negative moduli given their reciprocals (Sec. 2.2: the shear
// modulus at an edge point); zero when any modulus is zero, whose reciprocal is +inf.
template <typename T>
__device__ __forceinline__ T harmonic4r(T r0, T r1, T r2, T r3) {
    return T(4) * rcp(r0 + r1 + r2 + r3);
}

// Tile t of this block from the XCD-balanced order table; false for padding blocks.  fast is
// set for a fluid tile (see k_classify), uni for a fluid tile of uniform media, cols for a
// general tile with fluid columns, edges to the face neighbours of a fluid tile that take
// the general update (bits 0, 1: lower and upper side along y; bits 2, 3: along z).
__device__ __forceinline__ bool tile_of(const Tiles &tl, int nz, int &x0, int &y0, int &z0, int &z1, int &t,
                                        bool &fast, bool &uni, bool &cols, int &edges, int bid = -1) {
    const int ent = tl.order[bid < 0 ? (int)blockIdx.x : bid];
    if (ent < 0) return false;
    fast = (ent & kFastTile) != 0;
    uni = (ent & kUniformTile) != 0;
    cols = (ent & kColumnTile) != 0;
    edges = (ent >> kEdgeShift) & 15;
    t = ent & kTileMask;
    const int bx = t % tl.ntx;
    const int r = t / tl.ntx;
    const int by = r % tl.nty;
    const int bz = r / tl.nty;
    x0 = bx * TX;
    y0 = by * TY;
    z0 = bz * tl.zc;
    z1 = min(z0 + tl.zc, nz);
    return true;
}

// Each plane of a column is processed as: every load of the plane's main inputs, one
// scheduling fence (so they are in flight together: one memory round trip per plane), the
// arithmetic and the stores.  Where the cell lies in a C-PML layer, the memory variables of
// each layer axis are loaded as one batch ahead of their update and store.

// ------------------------------------------------------------------------
// velocity-shaped pass.  In_ca lives in field sigma^{ca} (forward) or w_(ca) (adjoint):
//   axis x: c=0 s11 (Dp), c=1 s12 (Dm), c=2 s13 (Dm)
//   axis y: c=0 s12 (Dm), c=1 s22 (Dp), c=2 s23 (Dm)
//   axis z: c=0 s13 (Dm), c=1 s23 (Dm), c=2 s33 (Dp)
// ------------------------------------------------------------------------
// Fluid-tile loop of the velocity-shaped pass.  UNI: a uniform tile, whose rho and alpha
// come from the per-tile table instead of the maps (the same values, so the same results).
//
// fluid tile: s22 = s33 = s11 and the shear stresses are zero on every tap, so the three
// nonzero differences are those of s11 along x, y and z.  Of the C-PML memory variables
// only the diagonal ones (phi^{cc}; in the adjoint a psi~^{cc} and a phi~^{cc}) act on
// fluid cells: the others stay zero or meet only zero moduli.
//
// Every input of plane k + 1, the own-point memory variable included, is loaded before
// plane k is computed (two planes of loads in flight per wavefront).  None of them is
// written by this pass except that memory variable, which only this lane reads and writes.
// The adjoint's taps of a psi~ are loaded with the plane's arithmetic, in one batch ahead
// of its first store (prefetching them too costs more registers than it saves).
//
// EN (forward only): also accumulate into kin the kinetic part sum_c rho_c u_old^c u_new^c of
// the modified energy (Sec. 2.2), with the staggered density of the update itself.
template <typename T, bool ADJ, bool UNI, bool EN>
__device__ __forceinline__ void fluid_vel(const Dev<T> &d, int i, int j, int z0, int z1, unsigned o, int t,
                                          int snx, int sny, int sox, int soy, double &kin) {
    const T h = d.inv_dx, dt = d.dt;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    const T *s11 = d.f[S11];
    const bool pml = d.P > 0;
    T qs[4];   // s11 at planes k-1..k+2
    qs[0] = T(0);
    qs[1] = ldb(s11, o - sz);
    qs[2] = ldb(s11, o);
    qs[3] = ldb(s11, o + sz);
    const T rho_t = UNI ? d.med[4 * t + 1] : T(0), alp_t = UNI ? d.med[4 * t + 2] : T(0);
    T rho_k = UNI ? rho_t : ldb(d.rho, o), alp_k = UNI ? alp_t : ldb(d.alpha, o);
    // layer coefficients of the column's x and y positions (half points)
    const T pa_x = sox >= 0 ? d.pa[0][1][i] : T(0), pb_x = sox >= 0 ? d.pb[0][1][i] : T(0);
    const T pa_y = soy >= 0 ? d.pa[1][1][j] : T(0), pb_y = soy >= 0 ? d.pb[1][1][j] : T(0);
    struct Plane {
        T qn, a11[4], b11[4], uold[3], rho_n[3], alp_n[3];
        T own[3];       // forward phi^{aa}, adjoint a phi~^{aa}, at the own slab point
        T pa_z, pb_z;
        int so_z;
    };
    auto load = [&](Plane &p, unsigned oo, int kk) {
        p.qn = ldb(s11, oo + 2 * sz);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            p.a11[q] = ldb(s11, oo + (unsigned)(q - 1) * sx);
            p.b11[q] = ldb(s11, oo + (unsigned)(q - 1) * sy);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) p.uold[c] = ldb(d.f[U1 + c], oo);
        p.rho_n[0] = UNI ? rho_t : ldb(d.rho, oo + sx);
        p.rho_n[1] = UNI ? rho_t : ldb(d.rho, oo + sy);
        p.rho_n[2] = UNI ? rho_t : ldb(d.rho, oo + sz);
        p.alp_n[0] = UNI ? alp_t : ldb(d.alpha, oo + sx);
        p.alp_n[1] = UNI ? alp_t : ldb(d.alpha, oo + sy);
        p.alp_n[2] = UNI ? alp_t : ldb(d.alpha, oo + sz);
        p.so_z = pml ? slab_own(kk, d.P, d.hi[2]) : -1;
        p.pa_z = p.so_z >= 0 ? d.pa[2][1][kk] : T(0);
        p.pb_z = p.so_z >= 0 ? d.pb[2][1][kk] : T(0);
        const int so[3] = {sox, soy, p.so_z};
#pragma unroll
        for (int a = 0; a < 3; ++a)
            p.own[a] = so[a] >= 0 ? ldb(d.mem[a][a], slab_byte(d, a, so[a], i, j, kk)) : T(0);
    };
    Plane cur{}, nxt{};
    load(cur, o, z0);
    for (int k = z0; k < z1; ++k, o += sz) {
        if (k + 1 < z1) load(nxt, o + sz, k + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int n = 0; n < 3; ++n) qs[n] = qs[n + 1];
        qs[3] = cur.qn;
        const T *a11 = cur.a11, *b11 = cur.b11, *uold = cur.uold, *rho_n = cur.rho_n, *alp_n = cur.alp_n;
        T acc[3];
        acc[0] = dplus(a11[0], a11[1], a11[2], a11[3], h);
        acc[1] = dplus(b11[0], b11[1], b11[2], b11[3], h);
        acc[2] = dplus(qs[0], qs[1], qs[2], qs[3], h);
        const int crd[3] = {i, j, k};
        const int slab[3] = {sox, soy, cur.so_z};
        const T pa[3] = {pa_x, pa_y, cur.pa_z}, pb[3] = {pb_x, pb_y, cur.pb_z};
        if (ADJ) {
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] *= dt;
            const int near[3] = {snx, sny, pml ? slab_near(k, d.P, d.hi[2]) : -1};
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (near[a] >= 0)
                    acc[a] += dp_at(d.mem[a][3 + a], slab_byte(d, a, near[a], i, j, k), slab_stride(d, a), h);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const T phi = pb[a] * cur.own[a] + pa[a] * acc[a];
                stb(d.mem[a][a], slab_byte(d, a, slab[a], i, j, k), phi);
                acc[a] += phi;
            }
        }
        T out[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T rho_c = T(0.5) * (rho_k + rho_n[c]);
            const T alp_c = T(0.5) * (alp_k + alp_n[c]);
            const T irho = rcp(rho_c);
            out[c] = ADJ ? (T(1) - dt * alp_c) * uold[c] - acc[c] * irho
                         : (T(1) - dt * alp_c) * uold[c] + dt * irho * acc[c];
            stb(d.f[U1 + c], o, out[c]);
            if (EN) kin += (double)rho_c * (double)uold[c] * (double)out[c];
        }
        rho_k = rho_n[2];
        alp_k = alp_n[2];
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                // g' = a phi~^{aa} <- b g' + a dt r^a
                const int tw = slab_twin(crd[a], d.P, d.hi[a]);
                const T g = pb[a] * cur.own[a] + pa[a] * dt * out[a];
                stb(d.mem[a][a], slab_byte(d, a, slab[a], i, j, k), g);
                if (tw >= 0) stb(d.mem[a][a], slab_byte(d, a, tw, i, j, k), g);
            }
        }
        cur = nxt;
    }
}

// Sum of v over the block's 256 threads in a fixed order (wavefront butterflies, then the four
// wavefronts in turn): the same double for the same inputs.  Every thread of the block calls it.
__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    __shared__ double part[NT / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += part[w];
    return s;
}

// EN (forward only): each thread also writes its part of the kinetic energy sum (fluid_vel) to
// epart[blockIdx.x * NT + threadIdx.x], once on every path, padding blocks and lanes outside
// the grid included (a block reduction would need every lane at a barrier, and the early exits
// of the plain pass are kept as they are).
//
// ctr (captured step graphs, el_exec): a device step counter.  The forward's gather blocks
// write trace row *ctr of the traces at grow (the stress pass that follows advances it); the
// adjoint pass steps it back by one, for the scatter that follows.
//
// G > 1 (grouped launch): the blocks of member q of the group are first[q] .. first[q+1]-1.
template <typename T, bool ADJ, bool EN, int G>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) void k_vel(
    Grp<T, G> g, double *epart, int *ctr) {
    static_assert(NT == 256, "gather_block works on blocks of 256 threads");
    static_assert(!(ADJ && EN), "the energy belongs to the forward recursion");
    static_assert(G == 1 || !EN, "the energy is a single plan's");
    const int q = member_of(g);
    const int bid = G > 1 ? (int)blockIdx.x - g.first[q] : (int)blockIdx.x;
    const Dev<T> &d = g.d[q];
    const Tiles &tl = g.tl[q];
    const Rec &r = g.r[q];
    double *grow = g.row[q];
    if (ADJ && ctr && bid == 0 && threadIdx.x == 0) *ctr -= 1;
    if (!ADJ && grow && bid >= 8 * tl.per) {
        // the trace row of the stresses this pass reads (the previous step's), see launch_velocity
        gather_block(d, r, ctr ? grow + (size_t)(*ctr) * r.nrec : grow, bid - 8 * tl.per);
        return;
    }
    int x0, y0, z0, z1, t = 0, edges = 0;
    bool fast = false, uni = false, cols = false;
    double kin = 0.0;
    double *ekin = EN ? epart + (size_t)blockIdx.x * NT + threadIdx.x : nullptr;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1, t, fast, uni, cols, edges, G > 1 ? bid : -1)) {
        if (EN) *ekin = kin;
        return;
    }
    const int i = x0 + tile_col(), j = y0 + tile_row();
    if (i >= d.nx || j >= d.ny) {
        if (EN) *ekin = kin;
        return;
    }
    const T h = d.inv_dx, dt = d.dt;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    const T *s11 = d.f[S11], *s22 = d.f[S22], *s33 = d.f[S33], *s23 = d.f[S23], *s13 = d.f[S13], *s12 = d.f[S12];
    unsigned o = d.origin + (unsigned)z0 * sz + (unsigned)j * sy + (unsigned)i * sx;
    const bool pml = d.P > 0;
    const int snx = pml ? slab_near(i, d.P, d.hi[0]) : -1, sny = pml ? slab_near(j, d.P, d.hi[1]) : -1;
    const int sox = pml ? slab_own(i, d.P, d.hi[0]) : -1, soy = pml ? slab_own(j, d.P, d.hi[1]) : -1;
    if (fast) {
        if (uni) fluid_vel<T, ADJ, true, EN>(d, i, j, z0, z1, o, t, snx, sny, sox, soy, kin);
        else fluid_vel<T, ADJ, false, EN>(d, i, j, z0, z1, o, t, snx, sny, sox, soy, kin);
        if (EN) *ekin = kin;
        return;
    }
    bool fl, ul, rowuni;
    if (fluid_row(tl, t, x0, y0, d.nx, d.ny, cols, fl, ul, rowuni)) {
        if (rowuni) fluid_vel<T, ADJ, true, EN>(d, i, j, z0, z1, o, t, snx, sny, sox, soy, kin);
        else fluid_vel<T, ADJ, false, EN>(d, i, j, z0, z1, o, t, snx, sny, sox, soy, kin);
        if (EN) *ekin = kin;
        return;
    }
    const bool sh = !fl;                     // this lane reads the shear stresses
    const bool mp = !ul;                     // this lane reads rho and alpha from the maps
    const T rho_t = d.med[4 * t + 1], alp_t = d.med[4 * t + 2];
    // s22 and s33 hold s11's value on a fluid lane's taps (fluid columns store all three,
    // fluid tiles the bands next to general tiles), so every lane reads them from their own
    // arrays (a per-lane choice of array would cost registers this loop does not have)
    const T *p22 = s22, *p33 = s33;
    T qa[4], qb[4], qc[4];   // s13, s23 at planes k-2..k+1; s33 at planes k-1..k+2
    qa[0] = qb[0] = qc[0] = T(0);
    qa[1] = ld_if(sh, s13, o - 2 * sz);
    qa[2] = ld_if(sh, s13, o - sz);
    qa[3] = ld_if(sh, s13, o);
    qb[1] = ld_if(sh, s23, o - 2 * sz);
    qb[2] = ld_if(sh, s23, o - sz);
    qb[3] = ld_if(sh, s23, o);
    qc[1] = ldb(p33, o - sz);
    qc[2] = ldb(p33, o);
    qc[3] = ldb(p33, o + sz);
    T rho_k = ld_or(mp, d.rho, o, rho_t), alp_k = ld_or(mp, d.alpha, o, alp_t);
    for (int k = z0; k < z1; ++k, o += sz) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            qa[n] = qa[n + 1];
            qb[n] = qb[n + 1];
            qc[n] = qc[n + 1];
        }
        qc[3] = ldb(p33, o + 2 * sz);
        T a11[4], a12[4] = {}, a13[4] = {}, b12[4] = {}, b22[4], b23[4] = {};   // taps along x (a) and y (b)
        T qa3 = T(0), qb3 = T(0);
        if (sh) {
            qa3 = ldb(s13, o + sz);
            qb3 = ldb(s23, o + sz);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a12[q] = ldb(s12, o + (unsigned)(q - 2) * sx);   // Dm: -2 .. +1
                a13[q] = ldb(s13, o + (unsigned)(q - 2) * sx);
                b12[q] = ldb(s12, o + (unsigned)(q - 2) * sy);
                b23[q] = ldb(s23, o + (unsigned)(q - 2) * sy);
            }
        }
        qa[3] = qa3;
        qb[3] = qb3;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a11[q] = ldb(s11, o + (unsigned)(q - 1) * sx);   // Dp: -1 .. +2
            b22[q] = ldb(p22, o + (unsigned)(q - 1) * sy);
        }
        T uold[3], rho_n[3], alp_n[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) uold[c] = ldb(d.f[U1 + c], o);
        rho_n[0] = ld_or(mp, d.rho, o + sx, rho_t);
        rho_n[1] = ld_or(mp, d.rho, o + sy, rho_t);
        rho_n[2] = ld_or(mp, d.rho, o + sz, rho_t);
        alp_n[0] = ld_or(mp, d.alpha, o + sx, alp_t);
        alp_n[1] = ld_or(mp, d.alpha, o + sy, alp_t);
        alp_n[2] = ld_or(mp, d.alpha, o + sz, alp_t);
        __builtin_amdgcn_sched_barrier(0);
        T dd[3][3];
        dd[0][0] = dplus(a11[0], a11[1], a11[2], a11[3], h);
        dd[1][0] = dminus(a12[0], a12[1], a12[2], a12[3], h);
        dd[2][0] = dminus(a13[0], a13[1], a13[2], a13[3], h);
        dd[0][1] = dminus(b12[0], b12[1], b12[2], b12[3], h);
        dd[1][1] = dplus(b22[0], b22[1], b22[2], b22[3], h);
        dd[2][1] = dminus(b23[0], b23[1], b23[2], b23[3], h);
        dd[0][2] = dminus(qa[0], qa[1], qa[2], qa[3], h);
        dd[1][2] = dminus(qb[0], qb[1], qb[2], qb[3], h);
        dd[2][2] = dplus(qc[0], qc[1], qc[2], qc[3], h);
        const int crd[3] = {i, j, k};
        const int slab[3] = {sox, soy, pml ? slab_own(k, d.P, d.hi[2]) : -1};
        if (ADJ) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 3; ++a) dd[c][a] *= dt;
            const int snz = pml ? slab_near(k, d.P, d.hi[2]) : -1;
            if (snx >= 0) add_pml_axis<T, true, 0>(d, dd, snx, i, j, k, h);
            if (sny >= 0) add_pml_axis<T, true, 1>(d, dd, sny, i, j, k, h);
            if (snz >= 0) add_pml_axis<T, true, 2>(d, dd, snz, i, j, k, h);
        }
        T acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = dd[c][0] + dd[c][1] + dd[c][2];
        if (!ADJ) {
            // phi^{ca} <- b phi^{ca} + a D_a sigma^{ca}, one batch of loads per layer axis
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
                T m[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) m[c] = ldb(d.mem[a][c], q);
                const T ca[2] = {d.pa[a][0][crd[a]], d.pa[a][1][crd[a]]};
                const T cb[2] = {d.pb[a][0][crd[a]], d.pb[a][1][crd[a]]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c == a;
                    const T phi = cb[half] * m[c] + ca[half] * dd[c][a];
                    stb(d.mem[a][c], q, phi);
                    acc[c] += phi;
                }
            }
        }
        T out[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T rho_c = T(0.5) * (rho_k + rho_n[c]);
            const T alp_c = T(0.5) * (alp_k + alp_n[c]);
            const T irho = rcp(rho_c);
            out[c] = ADJ ? (T(1) - dt * alp_c) * uold[c] - acc[c] * irho
                         : (T(1) - dt * alp_c) * uold[c] + dt * irho * acc[c];
            stb(d.f[U1 + c], o, out[c]);
            if (EN) kin += (double)rho_c * (double)uold[c] * (double)out[c];
        }
        rho_k = rho_n[2];
        alp_k = alp_n[2];
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                // g' = a phi~ <- b g' + a dt r   (Gamma^T q with the indicator folded into a)
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
                const int tw = slab_twin(crd[a], d.P, d.hi[a]);
                T m[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) m[c] = ldb(d.mem[a][c], q);
                const T ca[2] = {d.pa[a][0][crd[a]], d.pa[a][1][crd[a]]};
                const T cb[2] = {d.pb[a][0][crd[a]], d.pb[a][1][crd[a]]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c == a;
                    const T g = cb[half] * m[c] + ca[half] * dt * out[c];
                    stb(d.mem[a][c], q, g);
                    if (tw >= 0) stb(d.mem[a][c], slab_byte(d, a, tw, i, j, k), g);
                }
            }
        }
    }
    if (EN) *ekin = kin;
}

// ------------------------------------------------------------------------
// stress-shaped pass.  In_ca lives in field u^c (forward) or r^c (adjoint):
//   axis x: c=0 Dm, c=1 Dp, c=2 Dp;  axis y: c=0 Dp, c=1 Dm, c=2 Dp;  axis z: c=0 Dp, c=1 Dp, c=2 Dm
// ------------------------------------------------------------------------
// Fluid-tile loop of the stress-shaped pass.  UNI: a uniform tile, whose lambda comes from
// the per-tile table instead of the map (the same value, so the same results); ul: the same
// for this lane alone (a fluid column of the tile's reference medium).  keep: store s22 and
// s33 on every cell (a fluid column of a general tile), else only on the bands.
//
// fluid tile: mu = 0, so the three normal stresses take the same increment lambda tr and
// the shear stresses stay zero (not written).  Only the diagonal C-PML memory variables
// (psi^{cc}; in the adjoint a phi~^{cc} and a psi~^{cc}) act on the trace.  As in the
// velocity loop, every input of plane k + 1 is loaded before plane k is computed; s11 and
// the own-point memory variable of a cell are read and written by its own lane only.
template <typename T, bool ADJ, bool UNI>
__device__ __forceinline__ void fluid_str(const Dev<T> &d, int i, int j, int y0, int z0, int z1, unsigned o,
                                          int t, int edges, bool keep, bool ul, int snx, int sny, int sox, int soy) {
    const T h = d.inv_dx, dt = d.dt;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    const T *u1 = d.f[U1], *u2 = d.f[U2], *u3 = d.f[U3];
    const bool pml = d.P > 0;
    const T lam_t = d.med[4 * t];
    // s22 is stored on the rows, s33 on the planes, that general tiles read across a face
    const bool put22 = keep || ((edges & 1) && j < y0 + 2) || ((edges & 2) && j >= y0 + TY - 2);
    const int zlo = keep ? z1 : ((edges & 4) ? z0 + 2 : z0), zhi = keep ? z0 : ((edges & 8) ? z1 - 2 : z1);
    T qc[4];   // u3 at planes k-2..k+1
    qc[0] = T(0);
    qc[1] = ldb(u3, o - 2 * sz);
    qc[2] = ldb(u3, o - sz);
    qc[3] = ldb(u3, o);
    // layer coefficients of the column's x and y positions (integer points)
    const T pa_x = sox >= 0 ? d.pa[0][0][i] : T(0), pb_x = sox >= 0 ? d.pb[0][0][i] : T(0);
    const T pa_y = soy >= 0 ? d.pa[1][0][j] : T(0), pb_y = soy >= 0 ? d.pb[1][0][j] : T(0);
    struct Plane {
        T qn, a1[4], b2[4], sold, lam;
        T own[3];       // forward psi^{aa}, adjoint a psi~^{aa}, at the own slab point
        T near[3][4];   // adjoint: taps of a phi~^{aa} (Dm) where they reach a layer
        T pa_z, pb_z;
        int so_z, sn_z;
    };
    auto load = [&](Plane &p, unsigned oo, int kk) {
        p.qn = ldb(u3, oo + sz);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            p.a1[q] = ldb(u1, oo + (unsigned)(q - 2) * sx);
            p.b2[q] = ldb(u2, oo + (unsigned)(q - 2) * sy);
        }
        p.sold = ldb(d.f[S11], oo);
        p.lam = UNI ? lam_t : ld_or(!ul, d.lam, oo, lam_t);
        p.so_z = pml ? slab_own(kk, d.P, d.hi[2]) : -1;
        p.sn_z = ADJ && pml ? slab_near(kk, d.P, d.hi[2]) : -1;
        p.pa_z = p.so_z >= 0 ? d.pa[2][0][kk] : T(0);
        p.pb_z = p.so_z >= 0 ? d.pb[2][0][kk] : T(0);
        const int so[3] = {sox, soy, p.so_z}, sn[3] = {snx, sny, p.sn_z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p.own[a] = so[a] >= 0 ? ldb(d.mem[a][3 + a], slab_byte(d, a, so[a], i, j, kk)) : T(0);
            if (ADJ) {
                if (sn[a] >= 0) {
                    const unsigned q = slab_byte(d, a, sn[a], i, j, kk), st = slab_stride(d, a);
                    const T *g = d.mem[a][a];
                    p.near[a][0] = ldb(g, q - 2 * st);
                    p.near[a][1] = ldb(g, q - st);
                    p.near[a][2] = ldb(g, q);
                    p.near[a][3] = ldb(g, q + st);
                } else {
#pragma unroll
                    for (int n = 0; n < 4; ++n) p.near[a][n] = T(0);
                }
            }
        }
    };
    Plane cur{}, nxt{};
    load(cur, o, z0);
    for (int k = z0; k < z1; ++k, o += sz) {
        if (k + 1 < z1) load(nxt, o + sz, k + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int n = 0; n < 3; ++n) qc[n] = qc[n + 1];
        qc[3] = cur.qn;
        const T *a1 = cur.a1, *b2 = cur.b2;
        const T sold = cur.sold, lam = cur.lam;
        T e[3];
        e[0] = dminus(a1[0], a1[1], a1[2], a1[3], h);
        e[1] = dminus(b2[0], b2[1], b2[2], b2[3], h);
        e[2] = dminus(qc[0], qc[1], qc[2], qc[3], h);
        const int crd[3] = {i, j, k};
        const int slab[3] = {sox, soy, cur.so_z};
        const T pa[3] = {pa_x, pa_y, cur.pa_z}, pb[3] = {pb_x, pb_y, cur.pb_z};
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) e[a] *= dt;
            const int near[3] = {snx, sny, cur.sn_z};
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (near[a] >= 0) e[a] += dminus(cur.near[a][0], cur.near[a][1], cur.near[a][2], cur.near[a][3], h);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const T psi = pb[a] * cur.own[a] + pa[a] * e[a];
                stb(d.mem[a][3 + a], slab_byte(d, a, slab[a], i, j, k), psi);
                e[a] += psi;
            }
        }
        const T tr = e[0] + e[1] + e[2];
        const T w = sold + (ADJ ? T(-1) : dt) * (lam * tr);
        stb(d.f[S11], o, w);
        if (put22) stb(d.f[S22], o, w);
        if (k < zlo || k >= zhi) stb(d.f[S33], o, w);
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                // g = a psi~^{aa} <- b g + a dt w_aa
                const int tw = slab_twin(crd[a], d.P, d.hi[a]);
                const T g = pb[a] * cur.own[a] + pa[a] * dt * w;
                stb(d.mem[a][3 + a], slab_byte(d, a, slab[a], i, j, k), g);
                if (tw >= 0) stb(d.mem[a][3 + a], slab_byte(d, a, tw, i, j, k), g);
            }
        }
        cur = nxt;
    }
}

// Theta^T y at the scatter points of column (i, j) of tile t, added by the lane that has just
// written the column's adjoint stresses and memory variables (no other lane reads or writes
// them in this launch), each point as launch_scatter adds it.
template <typename T>
__device__ __forceinline__ void scatter_col(const Dev<T> &d, const Rec &r, const double *y, int t) {
    const int s = r.tslot[t];
    if (s < 0) return;
    const int *lo = r.loff + (size_t)s * (TX * TY + 1) + tile_col() + TX * tile_row();
    const int e1 = lo[1];
    for (int e = lo[0]; e < e1; ++e) scatter_point(d, r, y, r.tpts[e]);
}

// ctr (captured step graphs): the forward pass advances the device step counter its velocity
// pass's gather blocks read (all of that launch has completed).  G > 1: grouped launch, as
// k_vel.
template <typename T, bool ADJ, int G>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 1))) void k_str(Grp<T, G> g,
                                                                                                   int *ctr) {
    const int q = member_of(g);
    const int bid = G > 1 ? (int)blockIdx.x - g.first[q] : (int)blockIdx.x;
    const Dev<T> &d = g.d[q];
    const Tiles &tl = g.tl[q];
    const Rec &r = g.r[q];
    // adjoint: the trace row whose Theta^T y this launch adds after the update (scatter_col)
    const double *yrow = ADJ && g.row[q] ? (ctr ? g.row[q] + (size_t)(*ctr) * r.nrec : g.row[q]) : nullptr;
    if (!ADJ && ctr && bid == 0 && threadIdx.x == 0) *ctr += 1;
    int x0, y0, z0, z1, t = 0, edges = 0;
    bool fast = false, uni = false, cols = false;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1, t, fast, uni, cols, edges, G > 1 ? bid : -1)) return;
    const int i = x0 + tile_col(), j = y0 + tile_row();
    if (i >= d.nx || j >= d.ny) return;
    const T h = d.inv_dx, dt = d.dt;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    const T *u1 = d.f[U1], *u2 = d.f[U2], *u3 = d.f[U3];
    unsigned o = d.origin + (unsigned)z0 * sz + (unsigned)j * sy + (unsigned)i * sx;
    const bool pml = d.P > 0;
    const int snx = pml ? slab_near(i, d.P, d.hi[0]) : -1, sny = pml ? slab_near(j, d.P, d.hi[1]) : -1;
    const int sox = pml ? slab_own(i, d.P, d.hi[0]) : -1, soy = pml ? slab_own(j, d.P, d.hi[1]) : -1;
    if (fast) {
        if (uni) fluid_str<T, ADJ, true>(d, i, j, y0, z0, z1, o, t, edges, false, true, snx, sny, sox, soy);
        else fluid_str<T, ADJ, false>(d, i, j, y0, z0, z1, o, t, edges, false, false, snx, sny, sox, soy);
        if (ADJ && yrow) scatter_col(d, r, yrow, t);
        return;
    }
    bool fl, ul, rowuni;
    const bool row = fluid_row(tl, t, x0, y0, d.nx, d.ny, cols, fl, ul, rowuni);
    if (row) {
        // fluid wavefront of a general tile: its neighbours read s22 and s33, so all are stored
        // (the fluid lanes of a mixed wavefront run the general loop below with masked loads,
        // in the adjoint too: with its arguments addressed by member, the grouped build the
        // adjoint takes has the registers for it, and the wavefront runs one loop, not both)
        if (rowuni) fluid_str<T, ADJ, true>(d, i, j, y0, z0, z1, o, t, 0, true, true, snx, sny, sox, soy);
        else fluid_str<T, ADJ, false>(d, i, j, y0, z0, z1, o, t, 0, true, ul, snx, sny, sox, soy);
        if (ADJ && yrow) scatter_col(d, r, yrow, t);
        return;
    }
    // A fluid lane of a mixed wavefront needs only the normal strains: the shear-strain taps and
    // the moduli read as zero (their true values on this lane's cell and taps), the shear
    // stresses are neither read nor written, and s22 = s33 = s11 is read from s11.
    const bool sh = !fl;
    const T *p22 = fl ? d.f[S11] : d.f[S22], *p33 = fl ? d.f[S11] : d.f[S33];
    const T lam_t = d.med[4 * t];   // lambda of the tile's reference medium (lanes with ul)
    T qa[4], qb[4], qc[4];   // u1, u2 at planes k-1..k+2; u3 at planes k-2..k+1
    qa[0] = qb[0] = qc[0] = T(0);
    qa[1] = ld_if(sh, u1, o - sz);
    qa[2] = ld_if(sh, u1, o);
    qa[3] = ld_if(sh, u1, o + sz);
    qb[1] = ld_if(sh, u2, o - sz);
    qb[2] = ld_if(sh, u2, o);
    qb[3] = ld_if(sh, u2, o + sz);
    qc[1] = ldb(u3, o - 2 * sz);
    qc[2] = ldb(u3, o - sz);
    qc[3] = ldb(u3, o);
    // mu at the cell and its +x, +y neighbours of the current plane, and their reciprocals
    // (carried from the previous plane)
    T m0 = ld_if(sh, d.mu, o);
    T r0 = rcp(m0), rx = rcp(ld_if(sh, d.mu, o + sx)), ry = rcp(ld_if(sh, d.mu, o + sy));
    for (int k = z0; k < z1; ++k, o += sz) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            qa[n] = qa[n + 1];
            qb[n] = qb[n + 1];
            qc[n] = qc[n + 1];
        }
        qc[3] = ldb(u3, o + sz);
        T a1[4], a2[4] = {}, a3[4] = {}, b1[4] = {}, b2[4], b3[4] = {};   // taps along x (a) and y (b)
        T sold[6] = {};
        T qa3 = T(0), qb3 = T(0), mz = T(0), mxz = T(0), myz = T(0), mxy = T(0);
        if (sh) {
            qa3 = ldb(u1, o + 2 * sz);
            qb3 = ldb(u2, o + 2 * sz);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a2[q] = ldb(u2, o + (unsigned)(q - 1) * sx);   // Dp: -1 .. +2
                a3[q] = ldb(u3, o + (unsigned)(q - 1) * sx);
                b1[q] = ldb(u1, o + (unsigned)(q - 1) * sy);
                b3[q] = ldb(u3, o + (unsigned)(q - 1) * sy);
            }
#pragma unroll
            for (int c = 3; c < 6; ++c) sold[c] = ldb(d.f[S11 + c], o);
            mz = ldb(d.mu, o + sz);
            mxz = ldb(d.mu, o + sx + sz);
            myz = ldb(d.mu, o + sy + sz);
            mxy = ldb(d.mu, o + sx + sy);
        }
        qa[3] = qa3;
        qb[3] = qb3;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a1[q] = ldb(u1, o + (unsigned)(q - 2) * sx);   // Dm: -2 .. +1
            b2[q] = ldb(u2, o + (unsigned)(q - 2) * sy);
        }
        sold[0] = ldb(d.f[S11], o);
        sold[1] = ldb(p22, o);
        sold[2] = ldb(p33, o);
        const T lam = ld_or(ADJ || !ul, d.lam, o, lam_t);
        __builtin_amdgcn_sched_barrier(0);
        T e[3][3];   // e[c][a] = D_a In_ca
        e[0][0] = dminus(a1[0], a1[1], a1[2], a1[3], h);
        e[1][0] = dplus(a2[0], a2[1], a2[2], a2[3], h);
        e[2][0] = dplus(a3[0], a3[1], a3[2], a3[3], h);
        e[0][1] = dplus(b1[0], b1[1], b1[2], b1[3], h);
        e[1][1] = dminus(b2[0], b2[1], b2[2], b2[3], h);
        e[2][1] = dplus(b3[0], b3[1], b3[2], b3[3], h);
        e[0][2] = dplus(qa[0], qa[1], qa[2], qa[3], h);
        e[1][2] = dplus(qb[0], qb[1], qb[2], qb[3], h);
        e[2][2] = dminus(qc[0], qc[1], qc[2], qc[3], h);
        const int crd[3] = {i, j, k};
        const int slab[3] = {sox, soy, pml ? slab_own(k, d.P, d.hi[2]) : -1};
        if (ADJ) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 3; ++a) e[c][a] *= dt;
            const int snz = pml ? slab_near(k, d.P, d.hi[2]) : -1;
            if (snx >= 0) add_pml_axis<T, false, 0>(d, e, snx, i, j, k, h);
            if (sny >= 0) add_pml_axis<T, false, 1>(d, e, sny, i, j, k, h);
            if (snz >= 0) add_pml_axis<T, false, 2>(d, e, snz, i, j, k, h);
        }
        if (!ADJ) {
            // psi^{ca} <- b psi^{ca} + a D_a u^c, one batch of loads per layer axis
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
                T m[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) m[c] = ldb(d.mem[a][3 + c], q);
                const T ca[2] = {d.pa[a][0][crd[a]], d.pa[a][1][crd[a]]};
                const T cb[2] = {d.pb[a][0][crd[a]], d.pb[a][1][crd[a]]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c != a;
                    const T psi = cb[half] * m[c] + ca[half] * e[c][a];
                    stb(d.mem[a][3 + c], q, psi);
                    e[c][a] += psi;
                }
            }
        }
        const T rz = rcp(mz), rxz = rcp(mxz), ryz = rcp(myz), rxy = rcp(mxy);
        const T m23 = harmonic4r(r0, ry, rz, ryz);
        const T m13 = harmonic4r(r0, rx, rz, rxz);
        const T m12 = harmonic4r(r0, rx, ry, rxy);
        const T mu = m0;
        m0 = mz;
        r0 = rz;
        rx = rxz;
        ry = ryz;
        const T tr = e[0][0] + e[1][1] + e[2][2];
        const T sc = ADJ ? T(-1) : dt;
        T w[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) w[c] = sold[c] + sc * (lam * tr + T(2) * mu * e[c][c]);
        w[3] = sold[3] + sc * m23 * (e[1][2] + e[2][1]);
        w[4] = sold[4] + sc * m13 * (e[0][2] + e[2][0]);
        w[5] = sold[5] + sc * m12 * (e[0][1] + e[1][0]);
#pragma unroll
        for (int c = 0; c < 3; ++c) stb(d.f[S11 + c], o, w[c]);
        if (sh) {
#pragma unroll
            for (int c = 3; c < 6; ++c) stb(d.f[S11 + c], o, w[c]);
        }
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                // g = a psi~ <- b g + a dt w   (Delta^T s; the indicator is folded into a)
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
                const int tw = slab_twin(crd[a], d.P, d.hi[a]);
                T m[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) m[c] = ldb(d.mem[a][3 + c], q);
                const T ca[2] = {d.pa[a][0][crd[a]], d.pa[a][1][crd[a]]};
                const T cb[2] = {d.pb[a][0][crd[a]], d.pb[a][1][crd[a]]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c != a;
                    const int wi = c == a ? c : (c + a == 3 ? 3 : (c + a == 2 ? 4 : 5));
                    const T g = cb[half] * m[c] + ca[half] * dt * w[wi];
                    stb(d.mem[a][3 + c], q, g);
                    if (tw >= 0) stb(d.mem[a][3 + c], slab_byte(d, a, tw, i, j, k), g);
                }
            }
        }
    }
    if (ADJ && yrow) scatter_col(d, r, yrow, t);
}

// A plan's own pass as a launch of one member.  The adjoint passes take the grouped kernels
// (G = kGroupMax) with one member: with their kernel arguments addressed by member the
// compiler keeps fewer of them in registers, which leaves room for the masked loads of their
// mixed rows (at 384^3 the adjoint stress pass runs in 398 instead of 443 us, the adjoint
// velocity pass reads the maps only off uniform lanes); the forward passes are as fast with
// G = 1.
template <int G, typename T>
Grp<T, G> one(const Dev<T> &d, const Tiles &tl, const Rec *r = nullptr, double *row = nullptr) {
    Grp<T, G> g{};
    g.d[0] = d;
    g.tl[0] = tl;
    g.r[0] = r ? *r : Rec{};
    g.row[0] = row;
    g.first[0] = 0;
    for (int k = 1; k <= G; ++k) g.first[k] = 1 << 30;
    g.n = 1;
    return g;
}

template <typename T>
hipError_t launch_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s, const Rec *r, double *grow,
                           double *epart, int *ctr) {
    const bool gat = r && grow && r->nrec > 0;
    const int blocks = 8 * tl.per + (gat ? gather_blocks(r->nrec) : 0);
    const Grp<T, 1> g = one<1>(d, tl, gat ? r : nullptr, gat ? grow : nullptr);
    if (epart)
        hipLaunchKernelGGL((k_vel<T, false, true, 1>), dim3(blocks), dim3(NT), 0, s, g, epart, ctr);
    else
        hipLaunchKernelGGL((k_vel<T, false, false, 1>), dim3(blocks), dim3(NT), 0, s, g, (double *)nullptr, ctr);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s, int *ctr) {
    hipLaunchKernelGGL((k_str<T, false, 1>), dim3(8 * tl.per), dim3(NT), 0, s, one<1>(d, tl), ctr);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s, int *ctr) {
    hipLaunchKernelGGL((k_vel<T, true, false, kGroupMax>), dim3(8 * tl.per), dim3(NT), 0, s, one<kGroupMax>(d, tl),
                       (double *)nullptr,
                       ctr);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s, const Rec *r, const double *y,
                             int *ctr) {
    const bool sc = r && y && r->npts > 0;
    hipLaunchKernelGGL((k_str<T, true, kGroupMax>), dim3(8 * tl.per), dim3(NT), 0, s,
                       one<kGroupMax>(d, tl, sc ? r : nullptr, sc ? const_cast<double *>(y) : nullptr),
                       sc ? ctr : nullptr);
    return hipGetLastError();
}

// Grouped passes: members q < g.n with first[] set by group_blocks.
template <typename T>
hipError_t launch_group_pass(const Grp<T, kGroupMax> &g, int pass, hipStream_t s) {
    const dim3 grid(g.first[g.n]);
    switch (pass) {
        case 0: hipLaunchKernelGGL((k_vel<T, false, false, kGroupMax>), grid, dim3(NT), 0, s, g, (double *)nullptr, (int *)nullptr); break;
        case 1: hipLaunchKernelGGL((k_str<T, false, kGroupMax>), grid, dim3(NT), 0, s, g, (int *)nullptr); break;
        case 2: hipLaunchKernelGGL((k_vel<T, true, false, kGroupMax>), grid, dim3(NT), 0, s, g, (double *)nullptr, (int *)nullptr); break;
        default: hipLaunchKernelGGL((k_str<T, true, kGroupMax>), grid, dim3(NT), 0, s, g, (int *)nullptr); break;
    }
    return hipGetLastError();
}

// Potential part of the modified energy (Sec. 2.2): sigma^T C^+ sigma over the stresses of one
// time level, in double.  At a normal-stress point with moduli lambda, mu
//   (tr s)^2 / (9 K) + |dev s|^2 / (2 mu),   9 K = 3 (3 lambda + 2 mu),
// the second term only where mu > 0 (a fluid cell's deviatoric stress stays zero, Sec. 2.1);
// at a shear point s_ij^2 / mu_ij with the harmonic-mean edge modulus of the stencils, only
// where it is nonzero.  A fluid tile stores s11 alone (s22 = s33 = s11, shear zero), so its
// trace is 3 s11 and it has neither deviatoric nor shear part.  Each tile block writes its
// sum to epart[blockIdx.x].
template <typename T>
__device__ __forceinline__ void pot_tile(const Dev<T> &d, const Tiles &tl, double &pot) {
    int x0, y0, z0, z1, t = 0, edges = 0;
    bool fast = false, uni = false, cols = false;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1, t, fast, uni, cols, edges)) return;
    const int i = x0 + tile_col(), j = y0 + tile_row();
    if (i >= d.nx || j >= d.ny) return;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    unsigned o = d.origin + (unsigned)z0 * sz + (unsigned)j * sy + (unsigned)i * sx;
    for (int k = z0; k < z1; ++k, o += sz) {
        const double lam = (double)ldb(d.lam, o), mu = (double)ldb(d.mu, o);
        const double s11 = (double)ldb(d.f[S11], o);
        if (fast) {
            const double tr = 3.0 * s11;
            pot += tr * tr / (3.0 * (3.0 * lam + 2.0 * mu));
            continue;
        }
        const double s22 = (double)ldb(d.f[S22], o), s33 = (double)ldb(d.f[S33], o);
        const double tr = s11 + s22 + s33;
        pot += tr * tr / (3.0 * (3.0 * lam + 2.0 * mu));
        if (mu > 0.0) {
            const double m = tr / 3.0, a = s11 - m, b = s22 - m, c = s33 - m;
            pot += (a * a + b * b + c * c) / (2.0 * mu);
        }
        // edge moduli: harmonic means of the four cells around each shear point, as the
        // stencils form them (reciprocals of T, so a zero modulus gives a zero mean)
        const T r0 = rcp(ldb(d.mu, o)), rx = rcp(ldb(d.mu, o + sx)), ry = rcp(ldb(d.mu, o + sy));
        const T rz = rcp(ldb(d.mu, o + sz)), rxy = rcp(ldb(d.mu, o + sx + sy));
        const T rxz = rcp(ldb(d.mu, o + sx + sz)), ryz = rcp(ldb(d.mu, o + sy + sz));
        const double me[3] = {(double)harmonic4r(r0, ry, rz, ryz), (double)harmonic4r(r0, rx, rz, rxz),
                              (double)harmonic4r(r0, rx, ry, rxy)};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (!(me[q] > 0.0)) continue;
            const double sv = (double)ldb(d.f[S23 + q], o);
            pot += sv * sv / me[q];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_energy_pot(Dev<T> d, Tiles tl, double *epart) {
    double pot = 0.0;
    pot_tile<T>(d, tl, pot);
    const double s = block_sum(pot);
    if (threadIdx.x == 0) epart[blockIdx.x] = s;
}

template <typename T>
hipError_t launch_energy_pot(const Dev<T> &d, const Tiles &tl, double *epart, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_pot<T>, dim3(8 * tl.per), dim3(NT), 0, s, d, tl, epart);
    return hipGetLastError();
}

// Per tile block: the sum of its NT per-thread kinetic parts, in a fixed order.
__global__ __launch_bounds__(NT) void k_energy_blocks(const double *kin_thread, double *kin_block) {
    const double s = block_sum(kin_thread[(size_t)blockIdx.x * NT + threadIdx.x]);
    if (threadIdx.x == 0) kin_block[blockIdx.x] = s;
}

// out = (sum of kin[0..nb) + sum of pot[0..nb)) / 2, in a fixed order.
__global__ __launch_bounds__(NT) void k_energy_final(const double *kin, const double *pot, int nb, double *out) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) v += kin[b] + pot[b];
    const double s = block_sum(v);
    if (threadIdx.x == 0) *out = 0.5 * s;
}

hipError_t launch_energy_final(const double *kin_thread, double *kin_block, const double *pot, int nb, double *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_energy_blocks, dim3(nb), dim3(NT), 0, s, kin_thread, kin_block);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(NT), 0, s, kin_block, pot, nb, out);
    return hipGetLastError();
}

// s22 = s33 = s11 on every fluid tile (the state the lean stress loop leaves implicit).
template <typename T>
__global__ __launch_bounds__(NT) void k_fluid_fill(Dev<T> d, Tiles tl) {
    int x0, y0, z0, z1, t = 0, edges = 0;
    bool fast = false, uni = false, cols = false;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1, t, fast, uni, cols, edges) || !fast) return;
    const int i = x0 + tile_col(), j = y0 + tile_row();
    if (i >= d.nx || j >= d.ny) return;
    unsigned o = d.origin + (unsigned)z0 * d.sz + (unsigned)j * d.sy + (unsigned)i * (unsigned)sizeof(T);
    for (int k = z0; k < z1; ++k, o += d.sz) {
        const T v = ldb(d.f[S11], o);
        stb(d.f[S22], o, v);
        stb(d.f[S33], o, v);
    }
}

template <typename T>
hipError_t launch_fluid_fill(const Dev<T> &d, const Tiles &tl, hipStream_t s) {
    hipLaunchKernelGGL(k_fluid_fill<T>, dim3(8 * tl.per), dim3(NT), 0, s, d, tl);
    return hipGetLastError();
}

#define EL_STENCIL_INST(T)                                                                  \
    template hipError_t launch_fluid_fill<T>(const Dev<T> &, const Tiles &, hipStream_t);   \
    template hipError_t launch_velocity<T>(const Dev<T> &, const Tiles &, hipStream_t, const Rec *, double *,  \
                                           double *, int *);                                                   \
    template hipError_t launch_energy_pot<T>(const Dev<T> &, const Tiles &, double *, hipStream_t);            \
    template hipError_t launch_stress<T>(const Dev<T> &, const Tiles &, hipStream_t, int *);       \
    template hipError_t launch_adj_velocity<T>(const Dev<T> &, const Tiles &, hipStream_t, int *); \
    template hipError_t launch_adj_stress<T>(const Dev<T> &, const Tiles &, hipStream_t, const Rec *,       \
                                             const double *, int *);                                        \
    template hipError_t launch_group_pass<T>(const Grp<T, kGroupMax> &, int, hipStream_t);

EL_STENCIL_INST(float)
EL_STENCIL_INST(double)

}  // namespace el
