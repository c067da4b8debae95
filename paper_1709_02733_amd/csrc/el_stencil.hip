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
// Tiling: a block owns a 64 x 4 column tile (one wavefront per row) and each
// thread marches along z through a chunk of planes of its own column.
// Inputs differentiated along z sit in four-deep register queues; taps along
// x and y are read from memory, where the neighbouring rows of the tile and
// the tiles processed next to it keep them in L1/L2.  There is no LDS and no
// barrier.  The padded volume layout (see el_impl.h) makes every tap a plain
// load: addresses are a 32-bit byte offset, shared by all fields, from the
// field's base pointer.  Blocks are numbered so that each XCD (block id mod
// 8) receives a contiguous range of tiles.
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

template <typename T>
__device__ __forceinline__ T harmonic4(T m0, T m1, T m2, T m3) {
    if (m0 == T(0) || m1 == T(0) || m2 == T(0) || m3 == T(0)) return T(0);
    return T(4) / (T(1) / m0 + T(1) / m1 + T(1) / m2 + T(1) / m3);
}

// Logical tile of this block (XCD-aware numbering); false for padding blocks.
__device__ __forceinline__ bool tile_of(const Tiles &tl, int nz, int &x0, int &y0, int &z0, int &z1) {
    const int b = blockIdx.x;
    const int t = (b & 7) * tl.per + (b >> 3);
    if (t >= tl.ntiles) return false;
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

// ------------------------------------------------------------------------
// velocity-shaped pass.  In_ca lives in field sigma^{ca} (forward) or w_(ca) (adjoint):
//   axis x: c=0 s11 (Dp), c=1 s12 (Dm), c=2 s13 (Dm)
//   axis y: c=0 s12 (Dm), c=1 s22 (Dp), c=2 s23 (Dm)
//   axis z: c=0 s13 (Dm), c=1 s23 (Dm), c=2 s33 (Dp)
// ------------------------------------------------------------------------
template <typename T, bool ADJ>
__global__ __launch_bounds__(NT) void k_vel(Dev<T> d, Tiles tl) {
    int x0, y0, z0, z1;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1)) return;
    const int i = x0 + (int)threadIdx.x % TX, j = y0 + (int)threadIdx.x / TX;
    if (i >= d.nx || j >= d.ny) return;
    const T h = d.inv_dx;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    const T *s11 = d.f[S11], *s22 = d.f[S22], *s33 = d.f[S33], *s23 = d.f[S23], *s13 = d.f[S13], *s12 = d.f[S12];
    unsigned o = d.origin + (unsigned)z0 * sz + (unsigned)j * sy + (unsigned)i * sx;
    T qa[4], qb[4], qc[4];   // s13, s23 at planes k-2..k+1; s33 at planes k-1..k+2
    qa[0] = qb[0] = qc[0] = T(0);
    qa[1] = ldb(s13, o - 2 * sz);
    qa[2] = ldb(s13, o - sz);
    qa[3] = ldb(s13, o);
    qb[1] = ldb(s23, o - 2 * sz);
    qb[2] = ldb(s23, o - sz);
    qb[3] = ldb(s23, o);
    qc[1] = ldb(s33, o - sz);
    qc[2] = ldb(s33, o);
    qc[3] = ldb(s33, o + sz);
    T rho_k = ldb(d.rho, o), alp_k = ldb(d.alpha, o);
    const bool pml = d.P > 0;
    const int snx = pml ? slab_near(i, d.P, d.hi[0]) : -1, sny = pml ? slab_near(j, d.P, d.hi[1]) : -1;
    for (int k = z0; k < z1; ++k, o += sz) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            qa[n] = qa[n + 1];
            qb[n] = qb[n + 1];
            qc[n] = qc[n + 1];
        }
        qa[3] = ldb(s13, o + sz);
        qb[3] = ldb(s23, o + sz);
        qc[3] = ldb(s33, o + 2 * sz);
        T dd[3][3];
        dd[0][0] = dp_at(s11, o, sx, h);
        dd[1][0] = dm_at(s12, o, sx, h);
        dd[2][0] = dm_at(s13, o, sx, h);
        dd[0][1] = dm_at(s12, o, sy, h);
        dd[1][1] = dp_at(s22, o, sy, h);
        dd[2][1] = dm_at(s23, o, sy, h);
        dd[0][2] = dminus(qa[0], qa[1], qa[2], qa[3], h);
        dd[1][2] = dminus(qb[0], qb[1], qb[2], qb[3], h);
        dd[2][2] = dplus(qc[0], qc[1], qc[2], qc[3], h);
        if (ADJ) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 3; ++a) dd[c][a] *= d.dt;
            const int snz = pml ? slab_near(k, d.P, d.hi[2]) : -1;
            if (snx >= 0) add_pml_axis<T, true, 0>(d, dd, snx, i, j, k, h);
            if (sny >= 0) add_pml_axis<T, true, 1>(d, dd, sny, i, j, k, h);
            if (snz >= 0) add_pml_axis<T, true, 2>(d, dd, snz, i, j, k, h);
        }
        T acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = dd[c][0] + dd[c][1] + dd[c][2];
        const int crd[3] = {i, j, k};
        int slab[3] = {-1, -1, -1};
        if (pml) {
#pragma unroll
            for (int a = 0; a < 3; ++a) slab[a] = slab_own(crd[a], d.P, d.hi[a]);
        }
        if (!ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c == a;
                    const T phi = d.pb[a][half][crd[a]] * ldb(d.mem[a][c], q) + d.pa[a][half][crd[a]] * dd[c][a];
                    stb(d.mem[a][c], q, phi);
                    acc[c] += phi;
                }
            }
        }
        const T rho_z = ldb(d.rho, o + sz), alp_z = ldb(d.alpha, o + sz);
        const T rho_n[3] = {ldb(d.rho, o + sx), ldb(d.rho, o + sy), rho_z};
        const T alp_n[3] = {ldb(d.alpha, o + sx), ldb(d.alpha, o + sy), alp_z};
        T out[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T rho_c = T(0.5) * (rho_k + rho_n[c]);
            const T alp_c = T(0.5) * (alp_k + alp_n[c]);
            const T old = ldb(d.f[U1 + c], o);
            out[c] = ADJ ? (T(1) - d.dt * alp_c) * old - acc[c] / rho_c
                         : (T(1) - d.dt * alp_c) * old + d.dt / rho_c * acc[c];
            stb(d.f[U1 + c], o, out[c]);
        }
        rho_k = rho_z;
        alp_k = alp_z;
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                // g = a phi~ <- b g + a dt r   (Gamma^T q with the indicator folded into a)
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
                const int tw = slab_twin(crd[a], d.P, d.hi[a]);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c == a;
                    const T g = d.pb[a][half][crd[a]] * ldb(d.mem[a][c], q) + d.pa[a][half][crd[a]] * d.dt * out[c];
                    stb(d.mem[a][c], q, g);
                    if (tw >= 0) stb(d.mem[a][c], slab_byte(d, a, tw, i, j, k), g);
                }
            }
        }
    }
}

// ------------------------------------------------------------------------
// stress-shaped pass.  In_ca lives in field u^c (forward) or r^c (adjoint):
//   axis x: c=0 Dm, c=1 Dp, c=2 Dp;  axis y: c=0 Dp, c=1 Dm, c=2 Dp;  axis z: c=0 Dp, c=1 Dp, c=2 Dm
// ------------------------------------------------------------------------
template <typename T, bool ADJ>
__global__ __launch_bounds__(NT) void k_str(Dev<T> d, Tiles tl) {
    int x0, y0, z0, z1;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1)) return;
    const int i = x0 + (int)threadIdx.x % TX, j = y0 + (int)threadIdx.x / TX;
    if (i >= d.nx || j >= d.ny) return;
    const T h = d.inv_dx;
    const unsigned sx = sizeof(T), sy = d.sy, sz = d.sz;
    const T *u1 = d.f[U1], *u2 = d.f[U2], *u3 = d.f[U3];
    unsigned o = d.origin + (unsigned)z0 * sz + (unsigned)j * sy + (unsigned)i * sx;
    T qa[4], qb[4], qc[4];   // u1, u2 at planes k-1..k+2; u3 at planes k-2..k+1
    qa[0] = qb[0] = qc[0] = T(0);
    qa[1] = ldb(u1, o - sz);
    qa[2] = ldb(u1, o);
    qa[3] = ldb(u1, o + sz);
    qb[1] = ldb(u2, o - sz);
    qb[2] = ldb(u2, o);
    qb[3] = ldb(u2, o + sz);
    qc[1] = ldb(u3, o - 2 * sz);
    qc[2] = ldb(u3, o - sz);
    qc[3] = ldb(u3, o);
    // mu at the cell and its +x, +y neighbours of the current plane (carried from the previous plane)
    T m0 = ldb(d.mu, o), mx = ldb(d.mu, o + sx), my = ldb(d.mu, o + sy);
    const bool pml = d.P > 0;
    const int snx = pml ? slab_near(i, d.P, d.hi[0]) : -1, sny = pml ? slab_near(j, d.P, d.hi[1]) : -1;
    for (int k = z0; k < z1; ++k, o += sz) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            qa[n] = qa[n + 1];
            qb[n] = qb[n + 1];
            qc[n] = qc[n + 1];
        }
        qa[3] = ldb(u1, o + 2 * sz);
        qb[3] = ldb(u2, o + 2 * sz);
        qc[3] = ldb(u3, o + sz);
        T e[3][3];   // e[c][a] = D_a In_ca
        e[0][0] = dm_at(u1, o, sx, h);
        e[1][0] = dp_at(u2, o, sx, h);
        e[2][0] = dp_at(u3, o, sx, h);
        e[0][1] = dp_at(u1, o, sy, h);
        e[1][1] = dm_at(u2, o, sy, h);
        e[2][1] = dp_at(u3, o, sy, h);
        e[0][2] = dplus(qa[0], qa[1], qa[2], qa[3], h);
        e[1][2] = dplus(qb[0], qb[1], qb[2], qb[3], h);
        e[2][2] = dminus(qc[0], qc[1], qc[2], qc[3], h);
        if (ADJ) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 3; ++a) e[c][a] *= d.dt;
            const int snz = pml ? slab_near(k, d.P, d.hi[2]) : -1;
            if (snx >= 0) add_pml_axis<T, false, 0>(d, e, snx, i, j, k, h);
            if (sny >= 0) add_pml_axis<T, false, 1>(d, e, sny, i, j, k, h);
            if (snz >= 0) add_pml_axis<T, false, 2>(d, e, snz, i, j, k, h);
        }
        const int crd[3] = {i, j, k};
        int slab[3] = {-1, -1, -1};
        if (pml) {
#pragma unroll
            for (int a = 0; a < 3; ++a) slab[a] = slab_own(crd[a], d.P, d.hi[a]);
        }
        if (!ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c != a;
                    const T psi = d.pb[a][half][crd[a]] * ldb(d.mem[a][3 + c], q) + d.pa[a][half][crd[a]] * e[c][a];
                    stb(d.mem[a][3 + c], q, psi);
                    e[c][a] += psi;
                }
            }
        }
        const T lam = ldb(d.lam, o);
        const T mz = ldb(d.mu, o + sz), mxz = ldb(d.mu, o + sx + sz), myz = ldb(d.mu, o + sy + sz);
        const T mxy = ldb(d.mu, o + sx + sy);
        const T m23 = harmonic4(m0, my, mz, myz);
        const T m13 = harmonic4(m0, mx, mz, mxz);
        const T m12 = harmonic4(m0, mx, my, mxy);
        const T mu = m0;
        m0 = mz;
        mx = mxz;
        my = myz;
        const T tr = e[0][0] + e[1][1] + e[2][2];
        const T sc = ADJ ? T(-1) : d.dt;
        T w[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w[c] = ldb(d.f[S11 + c], o) + sc * (lam * tr + T(2) * mu * e[c][c]);
            stb(d.f[S11 + c], o, w[c]);
        }
        w[3] = ldb(d.f[S23], o) + sc * m23 * (e[1][2] + e[2][1]);
        w[4] = ldb(d.f[S13], o) + sc * m13 * (e[0][2] + e[2][0]);
        w[5] = ldb(d.f[S12], o) + sc * m12 * (e[0][1] + e[1][0]);
        stb(d.f[S23], o, w[3]);
        stb(d.f[S13], o, w[4]);
        stb(d.f[S12], o, w[5]);
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                // g = a psi~ <- b g + a dt w   (Delta^T s; the indicator is folded into a)
                const unsigned q = slab_byte(d, a, slab[a], i, j, k);
                const int tw = slab_twin(crd[a], d.P, d.hi[a]);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c != a;
                    const int wi = c == a ? c : (c + a == 3 ? 3 : (c + a == 2 ? 4 : 5));
                    const T g = d.pb[a][half][crd[a]] * ldb(d.mem[a][3 + c], q) + d.pa[a][half][crd[a]] * d.dt * w[wi];
                    stb(d.mem[a][3 + c], q, g);
                    if (tw >= 0) stb(d.mem[a][3 + c], slab_byte(d, a, tw, i, j, k), g);
                }
            }
        }
    }
}

template <typename T>
hipError_t launch_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s) {
    hipLaunchKernelGGL((k_vel<T, false>), dim3(8 * tl.per), dim3(NT), 0, s, d, tl);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s) {
    hipLaunchKernelGGL((k_str<T, false>), dim3(8 * tl.per), dim3(NT), 0, s, d, tl);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_velocity(const Dev<T> &d, const Tiles &tl, hipStream_t s) {
    hipLaunchKernelGGL((k_vel<T, true>), dim3(8 * tl.per), dim3(NT), 0, s, d, tl);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_stress(const Dev<T> &d, const Tiles &tl, hipStream_t s) {
    hipLaunchKernelGGL((k_str<T, true>), dim3(8 * tl.per), dim3(NT), 0, s, d, tl);
    return hipGetLastError();
}

#define EL_STENCIL_INST(T)                                                                  \
    template hipError_t launch_velocity<T>(const Dev<T> &, const Tiles &, hipStream_t);     \
    template hipError_t launch_stress<T>(const Dev<T> &, const Tiles &, hipStream_t);       \
    template hipError_t launch_adj_velocity<T>(const Dev<T> &, const Tiles &, hipStream_t); \
    template hipError_t launch_adj_stress<T>(const Dev<T> &, const Tiles &, hipStream_t);

EL_STENCIL_INST(float)
EL_STENCIL_INST(double)

}  // namespace el
