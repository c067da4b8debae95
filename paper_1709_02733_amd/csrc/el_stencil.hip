// Tiled stencil passes of the forward operator H and of its adjoint H^T (gfx950).
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
// These follow from Psi^T = -dt Div C, Phi^T = -dt Eps Q^{-1} and the
// zero-extended identity Dp^T = -Dm between the two difference types.
//
// Tiling: a block owns a 64 x 8 column tile (one wavefront per row) and
// marches along z over a chunk of planes.  Inputs differentiated along x or
// y are staged per plane in LDS with a two-cell halo; inputs differentiated
// along z sit in four-deep register queues of the thread's own column.
// Blocks are numbered so that each XCD (block id mod 8) receives a
// contiguous range of tiles, keeping neighbouring tiles in one L2.
#include "el_impl.h"

namespace el {

constexpr int TX = kTileX;
constexpr int TY = kTileY;
constexpr int NT = TX * TY;
constexpr int HX = 2, HY = 2;
constexpr int XW = TX + 2 * HX;
constexpr int YH = TY + 2 * HY;

template <typename T>
__device__ __forceinline__ T dplus(T fm1, T f0, T f1, T f2, T h) {
    return (T(9) / T(8) * (f1 - f0) + T(-1) / T(24) * (f2 - fm1)) * h;
}
template <typename T>
__device__ __forceinline__ T dminus(T fm2, T fm1, T f0, T f1, T h) {
    return (T(9) / T(8) * (f0 - fm1) + T(-1) / T(24) * (f1 - fm2)) * h;
}

__host__ __device__ constexpr int sig_of(int c, int a) {
    return c == a ? S11 + c : (c + a == 3 ? S23 : (c + a == 2 ? S13 : S12));
}

__device__ __forceinline__ int slab_of(int c, int P, int hi) {
    if (c <= P) return c;
    if (c >= hi) return c - hi + P + 1;
    return -1;
}

template <typename T>
__device__ __forceinline__ long long slab_at(const Dev<T> &d, int axis, int s, int i, int j, int k) {
    if (axis == 0) return ((long long)k * d.ny + j) * d.W + s;
    if (axis == 1) return ((long long)k * d.W + s) * d.nx + i;
    return ((long long)s * d.ny + j) * d.nx + i;
}

template <typename T>
__device__ __forceinline__ T at_clamped(const T *f, const Dev<T> &d, int i, int j, int k) {
    i = min(i, d.nx - 1);
    j = min(j, d.ny - 1);
    k = min(k, d.nz - 1);
    return f[i + (long long)d.nx * j + d.nxy * k];
}

template <typename T>
__device__ __forceinline__ T mu_harmonic(const Dev<T> &d, int a, int b, int i, int j, int k) {
    const int ai = a == 0, aj = a == 1, ak = a == 2, bi = b == 0, bj = b == 1, bk = b == 2;
    const T m0 = at_clamped(d.mu, d, i, j, k);
    const T m1 = at_clamped(d.mu, d, i + ai, j + aj, k + ak);
    const T m2 = at_clamped(d.mu, d, i + bi, j + bj, k + bk);
    const T m3 = at_clamped(d.mu, d, i + ai + bi, j + aj + bj, k + ak + bk);
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

// Stencil input of the velocity-shaped pass at a grid point (zero outside the grid).
template <typename T, bool ADJ>
__device__ __forceinline__ T vel_in(const Dev<T> &d, int c, int a, int i, int j, int k) {
    if (i < 0 || i >= d.nx || j < 0 || j >= d.ny || k < 0 || k >= d.nz) return T(0);
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    T v = d.f[sig_of(c, a)][p];
    if (!ADJ) return v;
    v *= d.dt;
    if (d.P > 0) {
        const int crd = a == 0 ? i : (a == 1 ? j : k);
        const int s = slab_of(crd, d.P, d.hi[a]);
        if (s >= 0) v += d.pa[a][c != a][crd] * d.mem[a][3 + c][slab_at(d, a, s, i, j, k)];
    }
    return v;
}

// Stencil input of the stress-shaped pass at a grid point (zero outside the grid).
template <typename T, bool ADJ>
__device__ __forceinline__ T str_in(const Dev<T> &d, int c, int a, int i, int j, int k) {
    if (i < 0 || i >= d.nx || j < 0 || j >= d.ny || k < 0 || k >= d.nz) return T(0);
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    T v = d.f[U1 + c][p];
    if (!ADJ) return v;
    v *= d.dt;
    if (d.P > 0) {
        const int crd = a == 0 ? i : (a == 1 ? j : k);
        const int s = slab_of(crd, d.P, d.hi[a]);
        if (s >= 0) v += d.pa[a][c == a][crd] * d.mem[a][c][slab_at(d, a, s, i, j, k)];
    }
    return v;
}

// ------------------------------------------------------------------------
// velocity-shaped pass
// ------------------------------------------------------------------------
template <typename T, bool ADJ>
__global__ __launch_bounds__(NT) void k_vel(Dev<T> d, Tiles tl) {
    __shared__ T lx[3][TY][XW];   // In_c,x with x halo
    __shared__ T ly[3][YH][TX];   // In_c,y with y halo
    int x0, y0, z0, z1;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1)) return;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = x0 + tx, j = y0 + ty;
    const bool own = i < d.nx && j < d.ny;
    const T h = d.inv_dx;
    // z queues: In_0z, In_1z use Dm (planes k-2..k+1), In_2z uses Dp (planes k-1..k+2)
    T qa[4], qb[4], qc[4];
    qa[0] = qb[0] = qc[0] = T(0);
    for (int n = 1; n < 4; ++n) {
        qa[n] = own ? vel_in<T, ADJ>(d, 0, 2, i, j, z0 - 3 + n) : T(0);
        qb[n] = own ? vel_in<T, ADJ>(d, 1, 2, i, j, z0 - 3 + n) : T(0);
        qc[n] = own ? vel_in<T, ADJ>(d, 2, 2, i, j, z0 - 2 + n) : T(0);
    }
    for (int k = z0; k < z1; ++k) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            qa[n] = qa[n + 1];
            qb[n] = qb[n + 1];
            qc[n] = qc[n + 1];
        }
        qa[3] = own ? vel_in<T, ADJ>(d, 0, 2, i, j, k + 1) : T(0);
        qb[3] = own ? vel_in<T, ADJ>(d, 1, 2, i, j, k + 1) : T(0);
        qc[3] = own ? vel_in<T, ADJ>(d, 2, 2, i, j, k + 2) : T(0);
        __syncthreads();
        for (int e = tid; e < 3 * TY * XW; e += NT) {
            const int c = e / (TY * XW);
            const int r = e - c * (TY * XW);
            const int yy = r / XW;
            const int xx = r - yy * XW;
            lx[c][yy][xx] = vel_in<T, ADJ>(d, c, 0, x0 - HX + xx, y0 + yy, k);
        }
        for (int e = tid; e < 3 * YH * TX; e += NT) {
            const int c = e / (YH * TX);
            const int r = e - c * (YH * TX);
            const int yy = r / TX;
            const int xx = r - yy * TX;
            ly[c][yy][xx] = vel_in<T, ADJ>(d, c, 1, x0 + xx, y0 - HY + yy, k);
        }
        __syncthreads();
        if (!own) continue;
        const int X = tx + HX, Y = ty + HY;
        T dd[3][3];
        dd[0][0] = dplus(lx[0][ty][X - 1], lx[0][ty][X], lx[0][ty][X + 1], lx[0][ty][X + 2], h);
        dd[1][0] = dminus(lx[1][ty][X - 2], lx[1][ty][X - 1], lx[1][ty][X], lx[1][ty][X + 1], h);
        dd[2][0] = dminus(lx[2][ty][X - 2], lx[2][ty][X - 1], lx[2][ty][X], lx[2][ty][X + 1], h);
        dd[0][1] = dminus(ly[0][Y - 2][tx], ly[0][Y - 1][tx], ly[0][Y][tx], ly[0][Y + 1][tx], h);
        dd[1][1] = dplus(ly[1][Y - 1][tx], ly[1][Y][tx], ly[1][Y + 1][tx], ly[1][Y + 2][tx], h);
        dd[2][1] = dminus(ly[2][Y - 2][tx], ly[2][Y - 1][tx], ly[2][Y][tx], ly[2][Y + 1][tx], h);
        dd[0][2] = dminus(qa[0], qa[1], qa[2], qa[3], h);
        dd[1][2] = dminus(qb[0], qb[1], qb[2], qb[3], h);
        dd[2][2] = dplus(qc[0], qc[1], qc[2], qc[3], h);
        T acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = dd[c][0] + dd[c][1] + dd[c][2];
        const int crd[3] = {i, j, k};
        int slab[3] = {-1, -1, -1};
        if (d.P > 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) slab[a] = slab_of(crd[a], d.P, d.hi[a]);
        }
        if (!ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const long long q = slab_at(d, a, slab[a], i, j, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c == a;
                    const T phi = d.pb[a][half][crd[a]] * d.mem[a][c][q] + d.pa[a][half][crd[a]] * dd[c][a];
                    d.mem[a][c][q] = phi;
                    acc[c] += phi;
                }
            }
        }
        const long long p = i + (long long)d.nx * j + d.nxy * k;
        const T r0 = d.rho[p], a0 = d.alpha[p];
        T out[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T rho_c = T(0.5) * (r0 + at_clamped(d.rho, d, i + (c == 0), j + (c == 1), k + (c == 2)));
            const T alp_c = T(0.5) * (a0 + at_clamped(d.alpha, d, i + (c == 0), j + (c == 1), k + (c == 2)));
            const T old = d.f[U1 + c][p];
            out[c] = ADJ ? (T(1) - d.dt * alp_c) * old - acc[c] / rho_c
                         : (T(1) - d.dt * alp_c) * old + d.dt / rho_c * acc[c];
            d.f[U1 + c][p] = out[c];
        }
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const long long q = slab_at(d, a, slab[a], i, j, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c == a;
                    const T chi = d.pa[a][half][crd[a]] != T(0) ? T(1) : T(0);
                    d.mem[a][c][q] = d.pb[a][half][crd[a]] * d.mem[a][c][q] + chi * d.dt * out[c];
                }
            }
        }
    }
}

// ------------------------------------------------------------------------
// stress-shaped pass
// ------------------------------------------------------------------------
template <typename T, bool ADJ>
__global__ __launch_bounds__(NT) void k_str(Dev<T> d, Tiles tl) {
    __shared__ T lx[3][TY][XW];
    __shared__ T ly[3][YH][TX];
    int x0, y0, z0, z1;
    if (!tile_of(tl, d.nz, x0, y0, z0, z1)) return;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = x0 + tx, j = y0 + ty;
    const bool own = i < d.nx && j < d.ny;
    const T h = d.inv_dx;
    // z queues: In_0z, In_1z use Dp (planes k-1..k+2), In_2z uses Dm (planes k-2..k+1)
    T qa[4], qb[4], qc[4];
    qa[0] = qb[0] = qc[0] = T(0);
    for (int n = 1; n < 4; ++n) {
        qa[n] = own ? str_in<T, ADJ>(d, 0, 2, i, j, z0 - 2 + n) : T(0);
        qb[n] = own ? str_in<T, ADJ>(d, 1, 2, i, j, z0 - 2 + n) : T(0);
        qc[n] = own ? str_in<T, ADJ>(d, 2, 2, i, j, z0 - 3 + n) : T(0);
    }
    for (int k = z0; k < z1; ++k) {
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            qa[n] = qa[n + 1];
            qb[n] = qb[n + 1];
            qc[n] = qc[n + 1];
        }
        qa[3] = own ? str_in<T, ADJ>(d, 0, 2, i, j, k + 2) : T(0);
        qb[3] = own ? str_in<T, ADJ>(d, 1, 2, i, j, k + 2) : T(0);
        qc[3] = own ? str_in<T, ADJ>(d, 2, 2, i, j, k + 1) : T(0);
        __syncthreads();
        for (int e = tid; e < 3 * TY * XW; e += NT) {
            const int c = e / (TY * XW);
            const int r = e - c * (TY * XW);
            const int yy = r / XW;
            const int xx = r - yy * XW;
            lx[c][yy][xx] = str_in<T, ADJ>(d, c, 0, x0 - HX + xx, y0 + yy, k);
        }
        for (int e = tid; e < 3 * YH * TX; e += NT) {
            const int c = e / (YH * TX);
            const int r = e - c * (YH * TX);
            const int yy = r / TX;
            const int xx = r - yy * TX;
            ly[c][yy][xx] = str_in<T, ADJ>(d, c, 1, x0 + xx, y0 - HY + yy, k);
        }
        __syncthreads();
        if (!own) continue;
        const int X = tx + HX, Y = ty + HY;
        T e[3][3];   // e[c][a] = D_a In_ca
        e[0][0] = dminus(lx[0][ty][X - 2], lx[0][ty][X - 1], lx[0][ty][X], lx[0][ty][X + 1], h);
        e[1][0] = dplus(lx[1][ty][X - 1], lx[1][ty][X], lx[1][ty][X + 1], lx[1][ty][X + 2], h);
        e[2][0] = dplus(lx[2][ty][X - 1], lx[2][ty][X], lx[2][ty][X + 1], lx[2][ty][X + 2], h);
        e[0][1] = dplus(ly[0][Y - 1][tx], ly[0][Y][tx], ly[0][Y + 1][tx], ly[0][Y + 2][tx], h);
        e[1][1] = dminus(ly[1][Y - 2][tx], ly[1][Y - 1][tx], ly[1][Y][tx], ly[1][Y + 1][tx], h);
        e[2][1] = dplus(ly[2][Y - 1][tx], ly[2][Y][tx], ly[2][Y + 1][tx], ly[2][Y + 2][tx], h);
        e[0][2] = dplus(qa[0], qa[1], qa[2], qa[3], h);
        e[1][2] = dplus(qb[0], qb[1], qb[2], qb[3], h);
        e[2][2] = dminus(qc[0], qc[1], qc[2], qc[3], h);
        const int crd[3] = {i, j, k};
        int slab[3] = {-1, -1, -1};
        if (d.P > 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) slab[a] = slab_of(crd[a], d.P, d.hi[a]);
        }
        if (!ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const long long q = slab_at(d, a, slab[a], i, j, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c != a;
                    const T psi = d.pb[a][half][crd[a]] * d.mem[a][3 + c][q] + d.pa[a][half][crd[a]] * e[c][a];
                    d.mem[a][3 + c][q] = psi;
                    e[c][a] += psi;
                }
            }
        }
        const long long p = i + (long long)d.nx * j + d.nxy * k;
        const T lam = d.lam[p], mu = d.mu[p];
        const T m23 = mu_harmonic(d, 1, 2, i, j, k);
        const T m13 = mu_harmonic(d, 0, 2, i, j, k);
        const T m12 = mu_harmonic(d, 0, 1, i, j, k);
        const T tr = e[0][0] + e[1][1] + e[2][2];
        const T sc = ADJ ? T(-1) : d.dt;
        T w[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w[c] = d.f[S11 + c][p] + sc * (lam * tr + T(2) * mu * e[c][c]);
            d.f[S11 + c][p] = w[c];
        }
        w[3] = d.f[S23][p] + sc * m23 * (e[1][2] + e[2][1]);
        w[4] = d.f[S13][p] + sc * m13 * (e[0][2] + e[2][0]);
        w[5] = d.f[S12][p] + sc * m12 * (e[0][1] + e[1][0]);
        d.f[S23][p] = w[3];
        d.f[S13][p] = w[4];
        d.f[S12][p] = w[5];
        if (ADJ) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (slab[a] < 0) continue;
                const long long q = slab_at(d, a, slab[a], i, j, k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int half = c != a;
                    const T wc = w[sig_of(c, a) - S11];
                    d.mem[a][3 + c][q] = d.pb[a][half][crd[a]] * d.mem[a][3 + c][q] + d.dt * wc;
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
