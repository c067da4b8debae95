// HIP kernels of the elastic operator pair for gfx950.
//
// Forward step (Appendix, Discrete formulation): a velocity pass that also
// advances the C-PML memory variables phi^{ij} on the boundary slabs, then a
// stress pass that advances psi^{ij}; the pressure is sampled after every
// step.  Adjoint step: the transposes of the four sub-updates, regrouped into
// two stencil passes of the same shapes (see the comments of adj_velocity and
// adj_stress).
//
// Staggering: normal stresses, lambda, mu on cells (i,j,k); u1/u2/u3 at
// +1/2 along x/y/z; s12, s13, s23 at +1/2 along both of their axes.  The 4th
// order difference (Sec. 2.2, eq. derivative) comes in two types:
//   Dp f[i] = (c1 (f[i+1] - f[i]) + c2 (f[i+2] - f[i-1])) / dx   (value at i + 1/2)
//   Dm f[i] = (c1 (f[i] - f[i-1]) + c2 (f[i+1] - f[i-2])) / dx   (value at i)
// with c1 = 9/8, c2 = -1/24 and fields extended by zero outside the grid.
#include "el_impl.h"

namespace el {

#define C1 (T(9) / T(8))
#define C2 (T(-1) / T(24))

// ------------------------------------------------------------------ helpers

template <typename T>
__device__ __forceinline__ T ld(const T *f, const Dev<T> &d, int i, int j, int k) {
    if (i < 0 || i >= d.nx || j < 0 || j >= d.ny || k < 0 || k >= d.nz) return T(0);
    return f[i + (long long)d.nx * j + d.nxy * k];
}

// Position of coordinate c in the boundary slab of an axis, -1 outside it.
__device__ __forceinline__ int slab_pos(int c, int P, int hi) {
    if (c <= P) return c;
    if (c >= hi) return c - hi + P + 1;
    return -1;
}

template <typename T>
__device__ __forceinline__ long long slab_idx(const Dev<T> &d, int axis, int s, int i, int j, int k) {
    if (axis == 0) return ((long long)k * d.ny + j) * d.W + s;
    if (axis == 1) return ((long long)k * d.W + s) * d.nx + i;
    return ((long long)s * d.ny + j) * d.nx + i;
}

// Difference along `axis` at (i,j,k) of a function given pointwise by `g(i,j,k)`.
template <typename T, typename G>
__device__ __forceinline__ T dp(G g, int axis, int i, int j, int k, T inv_dx) {
    const int a = axis == 0, b = axis == 1, c = axis == 2;
    return (C1 * (g(i + a, j + b, k + c) - g(i, j, k)) + C2 * (g(i + 2 * a, j + 2 * b, k + 2 * c) - g(i - a, j - b, k - c))) *
           inv_dx;
}
template <typename T, typename G>
__device__ __forceinline__ T dm(G g, int axis, int i, int j, int k, T inv_dx) {
    const int a = axis == 0, b = axis == 1, c = axis == 2;
    return (C1 * (g(i, j, k) - g(i - a, j - b, k - c)) + C2 * (g(i + a, j + b, k + c) - g(i - 2 * a, j - 2 * b, k - 2 * c))) *
           inv_dx;
}

// Voigt field id of sigma^{ij}.
__host__ __device__ constexpr int sig_id(int i, int j) {
    return i == j ? S11 + i : (i + j == 3 ? S23 : (i + j == 2 ? S13 : S12));
}

template <typename T>
__device__ __forceinline__ T clampld(const T *f, const Dev<T> &d, int i, int j, int k) {
    i = min(i, d.nx - 1);
    j = min(j, d.ny - 1);
    k = min(k, d.nz - 1);
    return f[i + (long long)d.nx * j + d.nxy * k];
}

// rho or alpha at the u^a point of cell (i,j,k): mean of the cell and its +a neighbour (replicated at the end).
template <typename T>
__device__ __forceinline__ T avg2(const T *m, const Dev<T> &d, int a, int i, int j, int k) {
    return T(0.5) * (clampld(m, d, i, j, k) + clampld(m, d, i + (a == 0), j + (a == 1), k + (a == 2)));
}

// mu at the shear point of axes (a, b) of cell (i,j,k): harmonic mean of four cells, 0 if any is 0.
template <typename T>
__device__ __forceinline__ T mu_shear(const Dev<T> &d, int a, int b, int i, int j, int k) {
    const int ai = a == 0, aj = a == 1, ak = a == 2, bi = b == 0, bj = b == 1, bk = b == 2;
    const T m0 = clampld(d.mu, d, i, j, k);
    const T m1 = clampld(d.mu, d, i + ai, j + aj, k + ak);
    const T m2 = clampld(d.mu, d, i + bi, j + bj, k + bk);
    const T m3 = clampld(d.mu, d, i + ai + bi, j + aj + bj, k + ak + bk);
    if (m0 == T(0) || m1 == T(0) || m2 == T(0) || m3 == T(0)) return T(0);
    return T(4) / (T(1) / m0 + T(1) / m1 + T(1) / m2 + T(1) / m3);
}

template <typename T>
__device__ __forceinline__ bool inside(const Dev<T> &d, int i, int j, int k) {
    return i >= 0 && i < d.nx && j >= 0 && j < d.ny && k >= 0 && k < d.nz;
}

// ---------------------------------------------------------------- set-up

template <typename T>
__global__ void k_convert_maps(Dev<T> d, const float *lam, const float *mu, const float *rho, const float *alpha,
                               long long n) {
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const_cast<T *>(d.lam)[p] = T(lam[p]);
        const_cast<T *>(d.mu)[p] = T(mu[p]);
        const_cast<T *>(d.rho)[p] = T(rho[p]);
        const_cast<T *>(d.alpha)[p] = T(alpha[p]);
    }
}

template <typename T>
hipError_t launch_convert_maps(const Dev<T> &d, const float *lam, const float *mu, const float *rho,
                               const float *alpha, hipStream_t s) {
    const long long n = d.nxy * d.nz;
    hipLaunchKernelGGL(k_convert_maps<T>, dim3(2048), dim3(256), 0, s, d, lam, mu, rho, alpha, n);
    return hipGetLastError();
}

// Media statistics in double: [0] max (lambda+2mu)/rho, [1] min rho, [2] min mu, [3] min lambda+2mu,
// [4] max dt*alpha, [5] min dt*alpha, [6] count of non-finite values.
__global__ void k_media_stats_partial(const float *lam, const float *mu, const float *rho, const float *alpha,
                                      long long n, double dt, double *partial) {
    double v[7] = {0.0, INFINITY, INFINITY, INFINITY, -INFINITY, INFINITY, 0.0};
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const double l = lam[p], m = mu[p], r = rho[p], a = alpha[p];
        if (!isfinite(l) || !isfinite(m) || !isfinite(r) || !isfinite(a)) v[6] += 1.0;
        const double lm = l + 2.0 * m;
        if (r > 0.0) v[0] = fmax(v[0], lm / r);
        v[1] = fmin(v[1], r);
        v[2] = fmin(v[2], m);
        v[3] = fmin(v[3], lm);
        v[4] = fmax(v[4], dt * a);
        v[5] = fmin(v[5], dt * a);
    }
    __shared__ double sh[7][256];
    for (int q = 0; q < 7; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const int t = threadIdx.x;
            sh[0][t] = fmax(sh[0][t], sh[0][t + st]);
            sh[1][t] = fmin(sh[1][t], sh[1][t + st]);
            sh[2][t] = fmin(sh[2][t], sh[2][t + st]);
            sh[3][t] = fmin(sh[3][t], sh[3][t + st]);
            sh[4][t] = fmax(sh[4][t], sh[4][t + st]);
            sh[5][t] = fmin(sh[5][t], sh[5][t + st]);
            sh[6][t] = sh[6][t] + sh[6][t + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 7; ++q) partial[q * kDotBlocks + blockIdx.x] = sh[q][0];
}

__global__ void k_media_stats_final(const double *partial, int nb, double *stats) {
    if (threadIdx.x != 0) return;
    double v[7] = {0.0, INFINITY, INFINITY, INFINITY, -INFINITY, INFINITY, 0.0};
    for (int b = 0; b < nb; ++b) {
        v[0] = fmax(v[0], partial[0 * kDotBlocks + b]);
        v[1] = fmin(v[1], partial[1 * kDotBlocks + b]);
        v[2] = fmin(v[2], partial[2 * kDotBlocks + b]);
        v[3] = fmin(v[3], partial[3 * kDotBlocks + b]);
        v[4] = fmax(v[4], partial[4 * kDotBlocks + b]);
        v[5] = fmin(v[5], partial[5 * kDotBlocks + b]);
        v[6] += partial[6 * kDotBlocks + b];
    }
    for (int q = 0; q < 7; ++q) stats[q] = v[q];
}

hipError_t launch_media_stats(const float *lam, const float *mu, const float *rho, const float *alpha, long long n,
                              double dt, double *stats, double *partial, hipStream_t s) {
    const int nb = 128;   // partial holds 7 * kDotBlocks doubles
    hipLaunchKernelGGL(k_media_stats_partial, dim3(nb), dim3(256), 0, s, lam, mu, rho, alpha, n, dt, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_media_stats_final, dim3(1), dim3(64), 0, s, partial, nb, stats);
    return hipGetLastError();
}

// --------------------------------------------------------- state set-up

template <typename T>
__global__ void k_fill(T *p, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] = T(0);
}

template <typename T>
hipError_t launch_zero_state(const Dev<T> &d, hipStream_t s) {
    const long long n = d.nxy * d.nz;
    for (int f = 0; f < NFIELD; ++f) {
        hipLaunchKernelGGL(k_fill<T>, dim3(2048), dim3(256), 0, s, d.f[f], n);
    }
    if (d.P > 0) {
        const long long ns[3] = {(long long)d.W * d.ny * d.nz, (long long)d.nx * d.W * d.nz, d.nxy * d.W};
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < 6; ++q) hipLaunchKernelGGL(k_fill<T>, dim3(512), dim3(256), 0, s, d.mem[a][q], ns[a]);
    }
    return hipGetLastError();
}

// tau': s11 = s22 = s33 = -p0/3 (Sec. 3, eq. initialp0); other fields were zeroed.
template <typename T>
__global__ void k_inject(Dev<T> d, const T *p0, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const T v = -p0[q] / T(3);
        d.f[S11][q] = v;
        d.f[S22][q] = v;
        d.f[S33][q] = v;
    }
}

template <typename T>
hipError_t launch_inject(const Dev<T> &d, const T *p0, hipStream_t s) {
    hipLaunchKernelGGL(k_inject<T>, dim3(2048), dim3(256), 0, s, d, p0, d.nxy * d.nz);
    return hipGetLastError();
}

// -------------------------------------------------------- forward passes

// Velocity pass: phi^{ij} <- b_j phi^{ij} + a_j D_j sigma^{ij} on the slabs, then
// u^i <- (1 - dt alpha_i) u^i + dt / rho_i sum_j (D_j sigma^{ij} + phi^{ij})
// (Appendix, Discrete formulation, first two lines; Sec. 2.2 eq. it without PML).
template <typename T>
__global__ void k_velocity(Dev<T> d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    const T h = d.inv_dx;
    T dd[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T *f = d.f[sig_id(c, a)];
            auto g = [&](int x, int y, int z) { return ld(f, d, x, y, z); };
            dd[c][a] = (c == a) ? dp<T>(g, a, i, j, k, h) : dm<T>(g, a, i, j, k, h);
        }
    T acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = dd[c][0] + dd[c][1] + dd[c][2];
    if (d.P > 0) {
        const int crd[3] = {i, j, k};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int s = slab_pos(crd[a], d.P, d.hi[a]);
            if (s < 0) continue;
            const long long q = slab_idx(d, a, s, i, j, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int half = (c == a);
                const T phi = d.pb[a][half][crd[a]] * d.mem[a][c][q] + d.pa[a][half][crd[a]] * dd[c][a];
                d.mem[a][c][q] = phi;
                acc[c] += phi;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T r = avg2(d.rho, d, c, i, j, k);
        const T al = avg2(d.alpha, d, c, i, j, k);
        d.f[U1 + c][p] = (T(1) - d.dt * al) * d.f[U1 + c][p] + d.dt / r * acc[c];
    }
}

// Stress pass: psi^{ij} <- b_j psi^{ij} + a_j D_j u^i on the slabs, then
// s_ii += dt [lambda sum_k (D_k u^k + psi^{kk}) + 2 mu (D_i u^i + psi^{ii})],
// s_ij += dt mu_ij (D_j u^i + psi^{ij} + D_i u^j + psi^{ji})
// (Appendix, Discrete formulation, last two lines; Sec. 2.2 operator Psi).
template <typename T>
__global__ void k_stress(Dev<T> d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    const T h = d.inv_dx;
    T e[3][3];   // e[c][a] = D_a u^c
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T *f = d.f[U1 + c];
            auto g = [&](int x, int y, int z) { return ld(f, d, x, y, z); };
            e[c][a] = (c == a) ? dm<T>(g, a, i, j, k, h) : dp<T>(g, a, i, j, k, h);
        }
    if (d.P > 0) {
        const int crd[3] = {i, j, k};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int s = slab_pos(crd[a], d.P, d.hi[a]);
            if (s < 0) continue;
            const long long q = slab_idx(d, a, s, i, j, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int half = (c != a);
                const T psi = d.pb[a][half][crd[a]] * d.mem[a][3 + c][q] + d.pa[a][half][crd[a]] * e[c][a];
                d.mem[a][3 + c][q] = psi;
                e[c][a] += psi;
            }
        }
    }
    const T lam = d.lam[p], mu = d.mu[p];
    const T tr = e[0][0] + e[1][1] + e[2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) d.f[S11 + c][p] += d.dt * (lam * tr + T(2) * mu * e[c][c]);
    d.f[S23][p] += d.dt * mu_shear(d, 1, 2, i, j, k) * (e[1][2] + e[2][1]);
    d.f[S13][p] += d.dt * mu_shear(d, 0, 2, i, j, k) * (e[0][2] + e[2][0]);
    d.f[S12][p] += d.dt * mu_shear(d, 0, 1, i, j, k) * (e[0][1] + e[1][0]);
}

template <typename T>
hipError_t launch_velocity(const Dev<T> &d, hipStream_t s) {
    dim3 b(64, 4), g((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
    hipLaunchKernelGGL(k_velocity<T>, g, b, 0, s, d);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_stress(const Dev<T> &d, hipStream_t s) {
    dim3 b(64, 4), g((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
    hipLaunchKernelGGL(k_stress<T>, g, b, 0, s, d);
    return hipGetLastError();
}

// ------------------------------------------------------- receivers

// p_hat_m[l] = -sum_c w_lc (s11 + s22 + s33)[c]  (Sec. 3, eq. interpgrid), in double.
// One wavefront serves 8 receivers; lane = 8 * receiver + corner, reduced over 8 lanes.
template <typename T>
__global__ void k_gather(Dev<T> d, Rec r, double *out) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int l = wave * 8 + (lane >> 3);
    const int c = lane & 7;
    double v = 0.0;
    if (l < r.nrec) {
        const long long q = r.idx[8 * l + c];
        v = r.w[8 * l + c] * ((double)d.f[S11][q] + (double)d.f[S22][q] + (double)d.f[S33][q]);
    }
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (l < r.nrec && c == 0) out[l] = -v;
}

template <typename T>
hipError_t launch_gather(const Dev<T> &d, const Rec &r, double *row, hipStream_t s) {
    if (r.nrec == 0) return hipSuccess;
    const int waves = (r.nrec + 7) / 8;
    const int blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_gather<T>, dim3(blocks), dim3(256), 0, s, d, r, row);
    return hipGetLastError();
}

// s_kk += Theta^T y_m at the touched cells (entries summed in a fixed order), and the
// matching correction of the adjoint normal memory variables (see adj_stress).
template <typename T>
__global__ void k_scatter(Dev<T> d, Rec r, const double *y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r.npts) return;
    double acc = 0.0;
    for (int e = r.row[t]; e < r.row[t + 1]; ++e) acc += r.ent_w[e] * y[r.ent_rec[e]];
    const T v = T(-acc);
    const long long q = r.pt[t];
    d.f[S11][q] += v;
    d.f[S22][q] += v;
    d.f[S33][q] += v;
    if (d.P > 0) {
        const int i = (int)(q % d.nx), j = (int)((q / d.nx) % d.ny), k = (int)(q / d.nxy);
        const int crd[3] = {i, j, k};
        const T wkk = d.dt * (T(3) * d.lam[q] + T(2) * d.mu[q]) * v;
        for (int a = 0; a < 3; ++a) {
            const int s = slab_pos(crd[a], d.P, d.hi[a]);
            if (s < 0) continue;
            d.mem[a][3 + a][slab_idx(d, a, s, i, j, k)] += wkk;
        }
    }
}

template <typename T>
hipError_t launch_scatter(const Dev<T> &d, const Rec &r, const double *y, hipStream_t s) {
    if (r.npts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter<T>, dim3((r.npts + 255) / 256), dim3(256), 0, s, d, r, y);
    return hipGetLastError();
}

// -------------------------------------------------------- adjoint passes
//
// One adjoint step applies W'^T = S1^T S2^T S3^T S4^T to the state
// (phi~, q, psi~, s), with the diagonal factors B, J, B~ of each step
// deferred into the next one.  In that form a step is
//   psi~ <- b psi~ + Delta^T s                   (done at the end of the previous adj_stress)
//   q    <- (1 - dt alpha) q + Psi^T s + E~^T psi~       = adj_velocity, stencil part
//   phi~ <- b phi~ + Gamma^T q                          = adj_velocity, own point
//   s    <- s + Phi^T q + E^T phi~                      = adj_stress, stencil part
// Psi^T s = -dt Div(C s) and E~^T psi~ = -sum_j D_j (a_j psi~^{ij}) use the
// forward velocity stencil; Phi^T q = -dt Eps(q / rho) and E^T phi~ use the
// forward stress stencil (zero-extended Dp^T = -Dm).

// w = C s at a cell: w_ii = lambda tr s + 2 mu s_ii, w_ij = mu_ij s_ij.
template <typename T>
__device__ __forceinline__ T w_at(const Dev<T> &d, int c, int a, int i, int j, int k) {
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    if (c == a) {
        const T tr = d.f[S11][p] + d.f[S22][p] + d.f[S33][p];
        return d.lam[p] * tr + T(2) * d.mu[p] * d.f[S11 + c][p];
    }
    const int lo = min(c, a), hi = max(c, a);
    return mu_shear(d, lo, hi, i, j, k) * d.f[sig_id(c, a)][p];
}

template <typename T>
__global__ void k_adj_velocity(Dev<T> d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    const T h = d.inv_dx;
    T acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // G(pt) = dt w_(ca)(pt) + a_a(pt) psi~^{ca}(pt), zero outside the grid
            auto g = [&](int x, int y, int z) -> T {
                if (!inside(d, x, y, z)) return T(0);
                T v = d.dt * w_at(d, c, a, x, y, z);
                if (d.P > 0) {
                    const int crd[3] = {x, y, z};
                    const int s = slab_pos(crd[a], d.P, d.hi[a]);
                    if (s >= 0) v += d.pa[a][c != a][crd[a]] * d.mem[a][3 + c][slab_idx(d, a, s, x, y, z)];
                }
                return v;
            };
            acc[c] += (c == a) ? dp<T>(g, a, i, j, k, h) : dm<T>(g, a, i, j, k, h);
        }
    }
    T q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T al = avg2(d.alpha, d, c, i, j, k);
        q[c] = (T(1) - d.dt * al) * d.f[U1 + c][p] - acc[c];
        d.f[U1 + c][p] = q[c];
    }
    if (d.P > 0) {
        const int crd[3] = {i, j, k};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int s = slab_pos(crd[a], d.P, d.hi[a]);
            if (s < 0) continue;
            const long long sq = slab_idx(d, a, s, i, j, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int half = (c == a);
                const T chi = d.pa[a][half][crd[a]] != T(0) ? T(1) : T(0);
                d.mem[a][c][sq] = d.pb[a][half][crd[a]] * d.mem[a][c][sq] + chi * d.dt * q[c] / avg2(d.rho, d, c, i, j, k);
            }
        }
    }
}

template <typename T>
__global__ void k_adj_stress(Dev<T> d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= d.nx || j >= d.ny) return;
    const long long p = i + (long long)d.nx * j + d.nxy * k;
    const T h = d.inv_dx;
    // H_ca(pt) = dt q^c(pt) / rho_c(pt) + a_a(pt) phi~^{ca}(pt)
    T e[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            auto g = [&](int x, int y, int z) -> T {
                if (!inside(d, x, y, z)) return T(0);
                const long long pp = x + (long long)d.nx * y + d.nxy * z;
                T v = d.dt * d.f[U1 + c][pp] / avg2(d.rho, d, c, x, y, z);
                if (d.P > 0) {
                    const int crd[3] = {x, y, z};
                    const int s = slab_pos(crd[a], d.P, d.hi[a]);
                    if (s >= 0) v += d.pa[a][c == a][crd[a]] * d.mem[a][c][slab_idx(d, a, s, x, y, z)];
                }
                return v;
            };
            e[c][a] = (c == a) ? dm<T>(g, a, i, j, k, h) : dp<T>(g, a, i, j, k, h);
        }
    T s[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] = d.f[S11 + c][p] - e[c][c];
    s[3] = d.f[S23][p] - (e[1][2] + e[2][1]);
    s[4] = d.f[S13][p] - (e[0][2] + e[2][0]);
    s[5] = d.f[S12][p] - (e[0][1] + e[1][0]);
#pragma unroll
    for (int q = 0; q < 6; ++q) d.f[S11 + q][p] = s[q];
    // next step's psi~ <- b psi~ + Delta^T s at the own point (slabs only)
    if (d.P > 0) {
        const int crd[3] = {i, j, k};
        const T tr = s[0] + s[1] + s[2];
        const T lam = d.lam[p], mu = d.mu[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int sp = slab_pos(crd[a], d.P, d.hi[a]);
            if (sp < 0) continue;
            const long long sq = slab_idx(d, a, sp, i, j, k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int half = (c != a);
                T w;
                if (c == a) {
                    w = lam * tr + T(2) * mu * s[c];
                } else {
                    const int lo = min(c, a), hi = max(c, a);
                    w = mu_shear(d, lo, hi, i, j, k) * s[sig_id(c, a) - S11];
                }
                d.mem[a][3 + c][sq] = d.pb[a][half][crd[a]] * d.mem[a][3 + c][sq] + d.dt * w;
            }
        }
    }
}

template <typename T>
hipError_t launch_adj_velocity(const Dev<T> &d, hipStream_t s) {
    dim3 b(64, 4), g((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
    hipLaunchKernelGGL(k_adj_velocity<T>, g, b, 0, s, d);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_stress(const Dev<T> &d, hipStream_t s) {
    dim3 b(64, 4), g((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
    hipLaunchKernelGGL(k_adj_stress<T>, g, b, 0, s, d);
    return hipGetLastError();
}

// p_adj = tau'^T v_0 = -(s11 + s22 + s33) / 3
template <typename T>
__global__ void k_extract(Dev<T> d, T *out, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        out[q] = -(d.f[S11][q] + d.f[S22][q] + d.f[S33][q]) / T(3);
}
template <typename T>
hipError_t launch_extract(const Dev<T> &d, T *p, hipStream_t s) {
    hipLaunchKernelGGL(k_extract<T>, dim3(2048), dim3(256), 0, s, d, p, d.nxy * d.nz);
    return hipGetLastError();
}

// ------------------------------------------------------ inner products

template <typename T>
__global__ void k_dot_partial(const T *a, const T *b, long long n, double *partial) {
    double v = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        v += (double)a[q] * (double)b[q];
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_dot_final(const double *partial, double *out) {
    __shared__ double sh[256];
    double v = 0.0;
    for (int b = threadIdx.x; b < kDotBlocks; b += 256) v += partial[b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

template <typename T>
hipError_t launch_dot(const T *a, const T *b, long long n, double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kDotBlocks), dim3(256), 0, s, a, b, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, partial, out);
    return hipGetLastError();
}

// ------------------------------------------------------- instantiation

#define EL_INST(T)                                                                                                   \
    template hipError_t launch_convert_maps<T>(const Dev<T> &, const float *, const float *, const float *,          \
                                               const float *, hipStream_t);                                          \
    template hipError_t launch_zero_state<T>(const Dev<T> &, hipStream_t);                                           \
    template hipError_t launch_inject<T>(const Dev<T> &, const T *, hipStream_t);                                    \
    template hipError_t launch_velocity<T>(const Dev<T> &, hipStream_t);                                             \
    template hipError_t launch_stress<T>(const Dev<T> &, hipStream_t);                                               \
    template hipError_t launch_gather<T>(const Dev<T> &, const Rec &, double *, hipStream_t);                        \
    template hipError_t launch_adj_velocity<T>(const Dev<T> &, hipStream_t);                                         \
    template hipError_t launch_adj_stress<T>(const Dev<T> &, hipStream_t);                                           \
    template hipError_t launch_scatter<T>(const Dev<T> &, const Rec &, const double *, hipStream_t);                 \
    template hipError_t launch_extract<T>(const Dev<T> &, T *, hipStream_t);                                         \
    template hipError_t launch_dot<T>(const T *, const T *, long long, double *, double *, hipStream_t);

EL_INST(float)
EL_INST(double)

}  // namespace el
