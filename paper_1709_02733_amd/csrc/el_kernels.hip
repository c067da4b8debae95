// Set-up, injection, receiver and reduction kernels of the elastic operator
// pair (gfx950).  The stencil passes live in el_stencil.hip.
//
// The adjoint state is kept as r = Q^{-1} q (velocity adjoint over the
// staggered density) and w = C s (Voigt stiffness times the stress adjoint),
// so the scatter of Theta^T y adds C applied to an isotropic increment and
// the extraction tau'^T v_0 = -(s11+s22+s33)/3 recovers tr s from w.
#include "el_impl.h"

namespace el {

// ------------------------------------------------------------------ helpers

// ---------------------------------------------------------------- set-up

// Copy the cell maps into the padded layout; the +x, +y, +z padding receives the value of the
// nearest cell (coordinates clamped independently), the rest of the padding zero.
template <typename T>
__global__ void k_convert_maps(Dev<T> d, const float *lam, const float *mu, const float *rho, const float *alpha,
                               long long total) {
    const long long plane = d.plane;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long zp = e / plane;
        const long long rem = e - zp * plane;
        const int y = (int)(rem / d.px), x = (int)(rem - (long long)y * d.px);
        const int z = (int)zp - 2;
        T vl = T(0), vm = T(0), vr = T(0), va = T(0);
        if (z >= 0 && z <= d.nz && y <= d.ny && x <= d.nx) {
            const long long src = min(x, d.nx - 1) + (long long)d.nx * (min(y, d.ny - 1) + (long long)d.ny * min(z, d.nz - 1));
            vl = T(lam[src]);
            vm = T(mu[src]);
            if (vm == T(0)) vm = T(0);   // -0 -> +0: the stencils take 1/mu, which must be +inf
            vr = T(rho[src]);
            va = T(alpha[src]);
        }
        const_cast<T *>(d.lam)[e] = vl;
        const_cast<T *>(d.mu)[e] = vm;
        const_cast<T *>(d.rho)[e] = vr;
        const_cast<T *>(d.alpha)[e] = va;
    }
}

template <typename T>
hipError_t launch_convert_maps(const Dev<T> &d, const float *lam, const float *mu, const float *rho,
                               const float *alpha, hipStream_t s) {
    const long long total = d.plane * (d.nz + 4);
    hipLaunchKernelGGL(k_convert_maps<T>, dim3(4096), dim3(256), 0, s, d, lam, mu, rho, alpha, total);
    return hipGetLastError();
}

// Media statistics in double: [0] max (lambda+2mu)/rho, [1] min rho, [2] min mu, [3] min lambda+2mu,
// [4] max dt*alpha, [5] min dt*alpha, [6] count of non-finite values, [7] min 3 lambda + 2 mu (three
// times the bulk modulus).
__global__ void k_media_stats_partial(const float *lam, const float *mu, const float *rho, const float *alpha,
                                      long long n, double dt, double *partial) {
    double v[kStats] = {0.0, INFINITY, INFINITY, INFINITY, -INFINITY, INFINITY, 0.0, INFINITY};
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
        v[7] = fmin(v[7], 3.0 * l + 2.0 * m);
    }
    __shared__ double sh[kStats][256];
    for (int q = 0; q < kStats; ++q) sh[q][threadIdx.x] = v[q];
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
            sh[7][t] = fmin(sh[7][t], sh[7][t + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < kStats; ++q) partial[q * kDotBlocks + blockIdx.x] = sh[q][0];
}

__global__ void k_media_stats_final(const double *partial, int nb, double *stats) {
    if (threadIdx.x != 0) return;
    double v[kStats] = {0.0, INFINITY, INFINITY, INFINITY, -INFINITY, INFINITY, 0.0, INFINITY};
    for (int b = 0; b < nb; ++b) {
        v[0] = fmax(v[0], partial[0 * kDotBlocks + b]);
        v[1] = fmin(v[1], partial[1 * kDotBlocks + b]);
        v[2] = fmin(v[2], partial[2 * kDotBlocks + b]);
        v[3] = fmin(v[3], partial[3 * kDotBlocks + b]);
        v[4] = fmax(v[4], partial[4 * kDotBlocks + b]);
        v[5] = fmin(v[5], partial[5 * kDotBlocks + b]);
        v[6] += partial[6 * kDotBlocks + b];
        v[7] = fmin(v[7], partial[7 * kDotBlocks + b]);
    }
    for (int q = 0; q < kStats; ++q) stats[q] = v[q];
}

hipError_t launch_media_stats(const float *lam, const float *mu, const float *rho, const float *alpha, long long n,
                              double dt, double *stats, double *partial, hipStream_t s) {
    const int nb = 128;   // partial holds kStats * kDotBlocks doubles
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
    const long long n = d.plane * (d.nz + 4);
    for (int f = 0; f < NFIELD; ++f) {
        hipLaunchKernelGGL(k_fill<T>, dim3(2048), dim3(256), 0, s, d.f[f], n);
    }
    if (d.P > 0) {
        const long long ns[3] = {(long long)d.W * d.ny * d.nz, (long long)d.nx * d.W * d.nz,
                                 (long long)d.nx * d.ny * d.W};
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < 6; ++q) hipLaunchKernelGGL(k_fill<T>, dim3(512), dim3(256), 0, s, d.mem[a][q], ns[a]);
    }
    return hipGetLastError();
}

// Fluid tiles.  Where mu = 0 the stress update keeps s11 = s22 = s33 and leaves the shear
// stresses at zero (their edge moduli are harmonic means that vanish next to a fluid cell),
// in both operators (forward: sigma; adjoint: w = C s).  A tile whose cells and the cells
// within two of them are all fluid can therefore be updated from the normal stress s11
// alone, with only the diagonal C-PML memory variables (a solid cell is at least three
// cells from the tile, out of reach of its taps).  One block per tile checks mu over that
// box; cells outside the grid count as fluid (zero extension).
//
// Inside a tile that is not fluid, column (i, j) of its chunk is fluid when mu = 0 on the
// cells within two of it (x, y in [i-2, i+2] x [j-2, j+2], z from z0-2 to z1+1, clipped to
// the grid): bit i-x0 of lanes[kTileY q + j-y0], set for such columns, lets the lanes of those
// columns run the fluid update inside the general tile.  The tile's first fluid column (in
// row-major lane order) gives a reference medium, written to med[4 q + 0..2]; bit i-x0 of
// lanes[kTileY (ntiles + q) + j-y0] marks the fluid columns whose lambda, rho and alpha equal the
// reference bit for bit on that same box, which then take them from the table.
//
// A fluid tile whose lambda, rho and alpha are each one value (bit for bit) over the same
// box is also marked uniform, and its three values are written to med[4 q + 0..2]: the
// stencil passes then take them from there instead of reading the maps (the box holds every
// map cell the fluid loops read, the edge-replicated padding included), with the same
// arithmetic and so the same results.
template <typename T>
__device__ __forceinline__ bool same_bits(T a, T b);
template <>
__device__ __forceinline__ bool same_bits<float>(float a, float b) {
    return __float_as_uint(a) == __float_as_uint(b);
}
template <>
__device__ __forceinline__ bool same_bits<double>(double a, double b) {
    return __double_as_longlong(a) == __double_as_longlong(b);
}

template <typename T>
__global__ __launch_bounds__(kTileX * kTileY) void k_classify(Dev<T> d, Tiles tl, unsigned char *fast,
                                                             unsigned char *uni, T *med, unsigned long long *lanes) {
    const int q = blockIdx.x;
    if (q >= tl.ntiles) return;
    const int bx = q % tl.ntx, r = q / tl.ntx, by = r % tl.nty, bz = r / tl.nty;
    const int x0 = bx * kTileX, y0 = by * kTileY, z0 = bz * tl.zc;
    const int x1 = min(x0 + kTileX, d.nx), y1 = min(y0 + kTileY, d.ny), z1 = min(z0 + tl.zc, d.nz);
    int solid = 0, vary = 0;
    const int ax = max(x0 - 2, 0), ay = max(y0 - 2, 0), az = max(z0 - 2, 0);
    const long long e0 = (long long)(az + 2) * d.plane + (long long)ay * d.px + ax;
    const T l0 = d.lam[e0], r0 = d.rho[e0], a0 = d.alpha[e0];
    {
        const int w = min(x1 + 2, d.nx) - ax, hgt = min(y1 + 2, d.ny) - ay, dep = min(z1 + 2, d.nz) - az;
        const long long n = (long long)w * hgt * dep;
        for (long long e = threadIdx.x; e < n; e += blockDim.x) {
            const int xx = ax + (int)(e % w);
            const long long rr = e / w;
            const int yy = ay + (int)(rr % hgt), zz = az + (int)(rr / hgt);
            const long long c = (long long)(zz + 2) * d.plane + (long long)yy * d.px + xx;
            if (d.mu[c] != T(0)) solid = 1;
            if (!same_bits(d.lam[c], l0) || !same_bits(d.rho[c], r0) || !same_bits(d.alpha[c], a0)) vary = 1;
        }
    }
    solid = __syncthreads_or(solid);
    vary = __syncthreads_or(vary);
    // columns of the tile and two around it: does mu vanish from z0-2 to z1+1?
    constexpr int HX = kTileX + 4, HY = kTileY + 4;
    __shared__ unsigned char col_solid[HX * HY];
    for (int e = threadIdx.x; e < HX * HY; e += blockDim.x) {
        const int xx = x0 - 2 + e % HX, yy = y0 - 2 + e / HX;
        int sol = 0;
        if (xx >= 0 && xx < d.nx && yy >= 0 && yy < d.ny)
            for (int zz = az; zz < min(z1 + 2, d.nz); ++zz)
                if (d.mu[(long long)(zz + 2) * d.plane + (long long)yy * d.px + xx] != T(0)) sol = 1;
        col_solid[e] = (unsigned char)sol;
    }
    __syncthreads();
    const int lx = (int)threadIdx.x % kTileX, ly = (int)threadIdx.x / kTileX;
    int colfluid = 0;
    if (x0 + lx < d.nx && y0 + ly < d.ny) {
        colfluid = 1;
        for (int dy = 0; dy < 5; ++dy)
            for (int dx = 0; dx < 5; ++dx)
                if (col_solid[(ly + dy) * HX + lx + dx]) colfluid = 0;
    }
    const unsigned long long m = __ballot(colfluid);
    __shared__ unsigned long long rowm[kTileY];
    __shared__ T ref[3];
    if ((threadIdx.x & 63) == 0) {
        lanes[kTileY * (size_t)q + threadIdx.x / 64] = m;
        rowm[threadIdx.x / 64] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // reference medium: the first fluid column's cell of plane z0, else the box corner's
        T rl = l0, rr = r0, ra = a0;
        for (int row = 0; row < kTileY; ++row)
            if (rowm[row]) {
                const int lane = __ffsll((long long)rowm[row]) - 1;
                const long long c = (long long)(z0 + 2) * d.plane + (long long)(y0 + row) * d.px + x0 + lane;
                rl = d.lam[c];
                rr = d.rho[c];
                ra = d.alpha[c];
                break;
            }
        ref[0] = rl;
        ref[1] = rr;
        ref[2] = ra;
    }
    __syncthreads();
    // columns of the tile and two around it: are lambda, rho, alpha the reference's from z0-2
    // to z1+1?  (Columns outside the grid hold nothing the loops read.)
    __shared__ unsigned char col_vary[HX * HY];
    for (int e = threadIdx.x; e < HX * HY; e += blockDim.x) {
        const int xx = x0 - 2 + e % HX, yy = y0 - 2 + e / HX;
        int v = 0;
        if (xx >= 0 && xx < d.nx && yy >= 0 && yy < d.ny)
            for (int zz = az; zz < min(z1 + 2, d.nz); ++zz) {
                const long long c = (long long)(zz + 2) * d.plane + (long long)yy * d.px + xx;
                if (!same_bits(d.lam[c], ref[0]) || !same_bits(d.rho[c], ref[1]) || !same_bits(d.alpha[c], ref[2])) v = 1;
            }
        col_vary[e] = (unsigned char)v;
    }
    __syncthreads();
    int colunif = colfluid;
    for (int dy = 0; dy < 5 && colunif; ++dy)
        for (int dx = 0; dx < 5; ++dx)
            if (col_vary[(ly + dy) * HX + lx + dx]) colunif = 0;
    const unsigned long long um = __ballot(colunif);
    if ((threadIdx.x & 63) == 0) lanes[kTileY * ((size_t)tl.ntiles + q) + threadIdx.x / 64] = um;
    if (threadIdx.x == 0) {
        fast[q] = solid ? 0 : 1;
        uni[q] = solid || vary ? 0 : 1;
        // a fluid tile keeps its box corner's values (every cell's, when it is uniform)
        med[4 * (size_t)q + 0] = solid ? ref[0] : l0;
        med[4 * (size_t)q + 1] = solid ? ref[1] : r0;
        med[4 * (size_t)q + 2] = solid ? ref[2] : a0;
        med[4 * (size_t)q + 3] = T(0);
    }
}

template <typename T>
hipError_t launch_classify(const Dev<T> &d, const Tiles &tl, unsigned char *fast, unsigned char *uni, T *med,
                           unsigned long long *lanes, hipStream_t s) {
    static_assert(kTileX == 64 && kTileY == 4, "one wavefront per tile row");
    if (tl.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify<T>, dim3(tl.ntiles), dim3(kTileX * kTileY), 0, s, d, tl, fast, uni, med, lanes);
    return hipGetLastError();
}

// Padded element of cell number q (x fastest).
template <typename T>
__device__ __forceinline__ long long padded(const Dev<T> &d, long long q) {
    const long long nxy = (long long)d.nx * d.ny;
    const long long k = q / nxy;
    const long long r = q - k * nxy;
    const long long j = r / d.nx;
    const long long i = r - j * d.nx;
    return (k + 2) * d.plane + j * d.px + i;
}

// tau': s11 = s22 = s33 = -p0/3 (Sec. 3, eq. initialp0); other fields were zeroed.
template <typename T>
__global__ void k_inject(Dev<T> d, const T *p0, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const T v = -p0[q] / T(3);
        const long long e = padded(d, q);
        d.f[S11][e] = v;
        d.f[S22][e] = v;
        d.f[S33][e] = v;
    }
}

template <typename T>
hipError_t launch_inject(const Dev<T> &d, const T *p0, hipStream_t s) {
    hipLaunchKernelGGL(k_inject<T>, dim3(4096), dim3(256), 0, s, d, p0, (long long)d.nx * d.ny * d.nz);
    return hipGetLastError();
}

// ------------------------------------------------------- receivers

// Receiver gather (gather_block in el_impl.h), standalone.
template <typename T>
__global__ __launch_bounds__(256) void k_gather(Dev<T> d, Rec r, double *out) {
    gather_block(d, r, out, (int)blockIdx.x);
}

template <typename T>
hipError_t launch_gather(const Dev<T> &d, const Rec &r, double *row, hipStream_t s) {
    if (r.nrec == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<T>, dim3(gather_blocks(r.nrec)), dim3(256), 0, s, d, r, row);
    return hipGetLastError();
}

// ctr != null (captured step graphs): y is the whole trace array and the row is *ctr (the
// adjoint velocity launch before it has stepped the counter back), so one graph of K steps
// serves every chunk of the time loop.
template <typename T>
__global__ void k_scatter(Dev<T> d, Rec r, const double *y, const int *ctr) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r.npts) return;
    scatter_point(d, r, ctr ? y + (size_t)(*ctr) * r.nrec : y, t);
}

template <typename T>
hipError_t launch_scatter(const Dev<T> &d, const Rec &r, const double *y, hipStream_t s, const int *ctr) {
    if (r.npts == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter<T>, dim3((r.npts + 255) / 256), dim3(256), 0, s, d, r, y, ctr);
    return hipGetLastError();
}

__global__ void k_set_counter(int *ctr, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = v;
}

hipError_t launch_set_counter(int *ctr, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, s, ctr, v);
    return hipGetLastError();
}

// p_adj = tau'^T v_0 = -(s11 + s22 + s33) / 3, with tr s = (w11 + w22 + w33) / (3 lambda + 2 mu).
template <typename T>
__global__ void k_extract(Dev<T> d, T *out, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long e = padded(d, q);
        out[q] = -(d.f[S11][e] + d.f[S22][e] + d.f[S33][e]) / (T(3) * (T(3) * d.lam[e] + T(2) * d.mu[e]));
    }
}
template <typename T>
hipError_t launch_extract(const Dev<T> &d, T *p, hipStream_t s) {
    hipLaunchKernelGGL(k_extract<T>, dim3(4096), dim3(256), 0, s, d, p, (long long)d.nx * d.ny * d.nz);
    return hipGetLastError();
}

// ---------------------------------------------------- transducer response
//
// Every trace (time-major [M][L] doubles) convolved in time with one causal kernel
// h[0..nh-1], or correlated with it (the adjoint).  One thread per output sample; the
// lanes of a wavefront cover consecutive receivers, so every load is coalesced, and a
// block's 64 consecutive time samples share the inputs of their window in L1.
__global__ void k_eir(const double *h, int nh, const double *in, double *out, int M, int L, int transpose) {
    const int nlb = (L + 63) / 64;
    const int l = (int)(blockIdx.x % nlb) * 64 + (int)(threadIdx.x & 63);
    const int m = (int)(blockIdx.x / nlb) * 4 + (int)(threadIdx.x >> 6);
    if (l >= L || m >= M) return;
    double acc = 0.0;
    if (!transpose) {
        const int kmax = min(m, nh - 1);
        for (int k = 0; k <= kmax; ++k) acc += h[k] * in[(size_t)(m - k) * L + l];
    } else {
        const int kmax = min(M - 1 - m, nh - 1);
        for (int k = 0; k <= kmax; ++k) acc += h[k] * in[(size_t)(m + k) * L + l];
    }
    out[(size_t)m * L + l] = acc;
}

hipError_t launch_eir(const double *h, int nh, const double *in, double *out, int M, int L, int transpose,
                      hipStream_t s) {
    if (M == 0 || L == 0) return hipSuccess;
    const long long blocks = (long long)((L + 63) / 64) * ((M + 3) / 4);   // < 2^31 (checked by the caller)
    hipLaunchKernelGGL(k_eir, dim3((unsigned)blocks), dim3(256), 0, s, h, nh, in, out, M, L, transpose);
    return hipGetLastError();
}

// ------------------------------------------------- frequency-dependent absorption
//
// Relaxation mechanisms l (include/el.h, el_relaxation): after each velocity pass,
//   u' = (u + dt sum_l beta_l zeta_l) / (1 + dt B),  zeta_l' = c_l zeta_l + (1 - c_l) u'
// with beta_l = w_l beta, B = sum_l beta_l, beta the mean of alpha_r over the two cells
// adjacent to the velocity point; the adjoint applies the transposed matrix,
//   s = r + sum_l (1 - c_l) z_l,  r' = s / (1 + dt B),  z_l' = dt beta_l s / (1 + dt B) + c_l z_l.
// Both are pointwise, so the adjoint's scaled variable r = q / rho takes the transpose as is.
// Where beta = 0 the forward leaves u alone and the adjoint's z stays zero, so only tiles
// holding a velocity point with beta > 0 are visited (flag).

// [0] min alpha_r, [1] non-finite count, [2] max alpha_r over the cells within `margin` of a face.
__global__ void k_relax_stats_partial(const float *ar, int nx, int ny, int nz, int margin, double *partial) {
    double v[3] = {INFINITY, 0.0, 0.0};
    const long long n = (long long)nx * ny * nz;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const double a = ar[p];
        if (!isfinite(a)) v[1] += 1.0;
        v[0] = fmin(v[0], a);
        const long long nxy = (long long)nx * ny;
        const int k = (int)(p / nxy), j = (int)((p - (long long)k * nxy) / nx), i = (int)(p % nx);
        if (i < margin || j < margin || k < margin || i >= nx - margin || j >= ny - margin || k >= nz - margin)
            v[2] = fmax(v[2], fabs(a));
    }
    __shared__ double sh[3][256];
    for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const int t = threadIdx.x;
            sh[0][t] = fmin(sh[0][t], sh[0][t + st]);
            sh[1][t] = sh[1][t] + sh[1][t + st];
            sh[2][t] = fmax(sh[2][t], sh[2][t + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) partial[q * kDotBlocks + blockIdx.x] = sh[q][0];
}

__global__ void k_relax_stats_final(const double *partial, int nb, double *stats) {
    if (threadIdx.x != 0) return;
    double v[3] = {INFINITY, 0.0, 0.0};
    for (int b = 0; b < nb; ++b) {
        v[0] = fmin(v[0], partial[b]);
        v[1] += partial[kDotBlocks + b];
        v[2] = fmax(v[2], partial[2 * kDotBlocks + b]);
    }
    for (int q = 0; q < 3; ++q) stats[q] = v[q];
}

hipError_t launch_relax_stats(const float *ar, int nx, int ny, int nz, int margin, double *stats, double *partial,
                              hipStream_t s) {
    const int nb = 128;
    hipLaunchKernelGGL(k_relax_stats_partial, dim3(nb), dim3(256), 0, s, ar, nx, ny, nz, margin, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_relax_stats_final, dim3(1), dim3(64), 0, s, partial, nb, stats);
    return hipGetLastError();
}

// Padded copy of alpha_r (as k_convert_maps: the +x, +y, +z padding holds the nearest cell).
template <typename T>
__global__ void k_relax_map(Dev<T> d, const float *ar, T *dst, long long total) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long zp = e / d.plane;
        const long long rem = e - zp * d.plane;
        const int y = (int)(rem / d.px), x = (int)(rem - (long long)y * d.px);
        const int z = (int)zp - 2;
        T v = T(0);
        if (z >= 0 && z <= d.nz && y <= d.ny && x <= d.nx)
            v = T(ar[min(x, d.nx - 1) + (long long)d.nx * (min(y, d.ny - 1) + (long long)d.ny * min(z, d.nz - 1))]);
        dst[e] = v;
    }
}

// Tile q is flagged when some velocity point of it has beta > 0 (the mean of alpha_r over the
// point's two cells, the upper one edge-replicated); count[q] receives the number of such
// (cell, component) points.
template <typename T>
__global__ __launch_bounds__(256) void k_relax_flags(Dev<T> d, Tiles tl, const T *ar, unsigned char *flag,
                                                     int *count) {
    const int q = blockIdx.x;
    if (q >= tl.ntiles) return;
    const int bx = q % tl.ntx, r = q / tl.ntx, by = r % tl.nty, bz = r / tl.nty;
    const int x0 = bx * kTileX, y0 = by * kTileY, z0 = bz * tl.zc;
    const int w = min(kTileX, d.nx - x0), hgt = min(kTileY, d.ny - y0), dep = min(tl.zc, d.nz - z0);
    const long long stride[3] = {1, d.px, d.plane};
    int n = 0;
    for (long long e = threadIdx.x; e < (long long)w * hgt * dep; e += blockDim.x) {
        const int xx = x0 + (int)(e % w);
        const long long rr = e / w;
        const int yy = y0 + (int)(rr % hgt), zz = z0 + (int)(rr / hgt);
        const long long c = (long long)(zz + 2) * d.plane + (long long)yy * d.px + xx;
        for (int a = 0; a < 3; ++a)
            if (T(0.5) * (ar[c] + ar[c + stride[a]]) > T(0)) ++n;
    }
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    if (n) atomicAdd(&total, n);
    __syncthreads();
    if (threadIdx.x == 0) {
        flag[q] = total > 0 ? 1 : 0;
        count[q] = total;
    }
}

template <typename T>
hipError_t launch_relax_setup(const Dev<T> &d, const Tiles &tl, const float *ar_cells, const Relax<T> &r,
                              hipStream_t s) {
    const long long total = d.plane * (d.nz + 4);
    hipLaunchKernelGGL(k_relax_map<T>, dim3(4096), dim3(256), 0, s, d, ar_cells, const_cast<T *>(r.ar), total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || tl.ntiles == 0) return e;
    hipLaunchKernelGGL(k_relax_flags<T>, dim3(tl.ntiles), dim3(256), 0, s, d, tl, r.ar,
                       const_cast<unsigned char *>(r.flag), r.count);
    return hipGetLastError();
}

// The point list (Relax::pts): block q writes the points of tile q from off[q] on, in the order
// component, plane, row, column, each with its beta, by the same test as k_relax_flags; a
// prefix sum over the block places each lane's point.  Exactly count[q] points are written.
template <typename T>
__global__ __launch_bounds__(256) void k_relax_compact(Dev<T> d, Tiles tl, Relax<T> r) {
    const int q = blockIdx.x;
    if (q >= tl.ntiles || !r.flag[q]) return;
    const int bx = q % tl.ntx, rr = q / tl.ntx, by = rr % tl.nty, bz = rr / tl.nty;
    const int x0 = bx * kTileX, y0 = by * kTileY, z0 = bz * tl.zc;
    const int w = min(kTileX, d.nx - x0), hgt = min(kTileY, d.ny - y0), dep = min(tl.zc, d.nz - z0);
    const int ncell = w * hgt * dep;
    const long long base = r.off[q];
    const int limit = r.count[q];
    const long long stride[3] = {1, d.px, d.plane};
    __shared__ int wave_n[4];
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    int done = 0;
    for (int c = 0; c < 3; ++c) {
        for (int e0 = 0; e0 < ncell; e0 += 256) {
            const int e = e0 + (int)threadIdx.x;
            bool on = false;
            long long el = 0;
            T beta = T(0);
            if (e < ncell) {
                const int xx = x0 + e % w, rem = e / w;
                const int yy = y0 + rem % hgt, zz = z0 + rem / hgt;
                el = (long long)(zz + 2) * d.plane + (long long)yy * d.px + xx;
                beta = T(0.5) * (r.ar[el] + r.ar[el + stride[c]]);
                on = beta > T(0);
            }
            const unsigned long long m = __ballot(on);
            const int before = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wave_n[wave] = __popcll(m);
            __syncthreads();
            int pos = done + before;
            int total = 0;
            for (int v = 0; v < 4; ++v) {
                if (v < wave) pos += wave_n[v];
                total += wave_n[v];
            }
            if (on && pos < limit) {
                r.pts[base + pos] = (unsigned)el | ((unsigned)c << 30);
                r.beta[base + pos] = beta;
            }
            done += total;
            __syncthreads();
        }
    }
    // the flags kernel counted these points with the same test, so nothing is left; were any
    // left, they become points with beta = 0 (R the identity) on the tile's first cell
    for (int pos = done + (int)threadIdx.x; pos < limit; pos += 256) {
        r.pts[base + pos] = (unsigned)((long long)(z0 + 2) * d.plane + (long long)y0 * d.px + x0);
        r.beta[base + pos] = T(0);
    }
}

template <typename T>
hipError_t launch_relax_compact(const Dev<T> &d, const Tiles &tl, const Relax<T> &r, hipStream_t s) {
    if (r.L == 0 || tl.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_relax_compact<T>, dim3(tl.ntiles), dim3(256), 0, s, d, tl, r);
    return hipGetLastError();
}

// Memory variables set to zero (initial state of an operation).
template <typename T>
__global__ __launch_bounds__(256) void k_relax_zero(Relax<T> r) {
    const long long n = r.npts * r.L;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) r.zeta[e] = T(0);
}

template <typename T>
hipError_t launch_relax_zero(const Tiles &, const Relax<T> &r, hipStream_t s) {
    if (r.L == 0 || r.npts == 0) return hipSuccess;
    const long long n = r.npts * r.L;
    const long long blocks = std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_relax_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, r);
    return hipGetLastError();
}

// The sub-update R (ADJ: R^T) at one velocity point with beta > 0 per lane (elsewhere R is the
// identity), the points and their memory variables read in list order.
template <typename T, bool ADJ, int L>
__global__ __launch_bounds__(256) void k_relax(Dev<T> d, Relax<T> r) {
    const long long p = blockIdx.x * 256LL + threadIdx.x;
    if (p >= r.npts) return;
    const unsigned pk = r.pts[p];
    const int c = (int)(pk >> 30);
    const long long e = pk & kRelaxElemMask;
    const T beta = r.beta[p];
    T z[L];
#pragma unroll
    for (int l = 0; l < L; ++l) z[l] = r.zeta[l * r.npts + p];
    T *u = c == 0 ? d.f[U1] : (c == 1 ? d.f[U2] : d.f[U3]);
    const T uo = u[e];
    const T dt = d.dt;
    T bl[L];
    T B = T(0);
#pragma unroll
    for (int l = 0; l < L; ++l) {
        bl[l] = r.w[l] * beta;
        B += bl[l];
    }
    const T a = T(1) / (T(1) + dt * B);
    if (!ADJ) {
        T acc = uo;
#pragma unroll
        for (int l = 0; l < L; ++l) acc += dt * bl[l] * z[l];
        const T un = acc * a;
        u[e] = un;
#pragma unroll
        for (int l = 0; l < L; ++l) r.zeta[l * r.npts + p] = r.c[l] * z[l] + (T(1) - r.c[l]) * un;
    } else {
        T sum = uo;
#pragma unroll
        for (int l = 0; l < L; ++l) sum += (T(1) - r.c[l]) * z[l];
        u[e] = a * sum;
#pragma unroll
        for (int l = 0; l < L; ++l) r.zeta[l * r.npts + p] = dt * bl[l] * a * sum + r.c[l] * z[l];
    }
}

template <typename T, bool ADJ>
hipError_t launch_relax_l(const Dev<T> &d, const Relax<T> &r, hipStream_t s) {
    const dim3 g((unsigned)((r.npts + 255) / 256)), b(256);
    switch (r.L) {
        case 1: hipLaunchKernelGGL((k_relax<T, ADJ, 1>), g, b, 0, s, d, r); break;
        case 2: hipLaunchKernelGGL((k_relax<T, ADJ, 2>), g, b, 0, s, d, r); break;
        case 3: hipLaunchKernelGGL((k_relax<T, ADJ, 3>), g, b, 0, s, d, r); break;
        default: hipLaunchKernelGGL((k_relax<T, ADJ, 4>), g, b, 0, s, d, r); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_relax(const Dev<T> &d, const Tiles &, const Relax<T> &r, bool adjoint, hipStream_t s) {
    if (r.L == 0 || r.npts == 0) return hipSuccess;
    return adjoint ? launch_relax_l<T, true>(d, r, s) : launch_relax_l<T, false>(d, r, s);
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
    template hipError_t launch_classify<T>(const Dev<T> &, const Tiles &, unsigned char *, unsigned char *, T *,     \
                                           unsigned long long *, hipStream_t);                                       \
    template hipError_t launch_inject<T>(const Dev<T> &, const T *, hipStream_t);                                    \
    template hipError_t launch_gather<T>(const Dev<T> &, const Rec &, double *, hipStream_t);                        \
    template hipError_t launch_scatter<T>(const Dev<T> &, const Rec &, const double *, hipStream_t, const int *);    \
    template hipError_t launch_extract<T>(const Dev<T> &, T *, hipStream_t);                                         \
    template hipError_t launch_dot<T>(const T *, const T *, long long, double *, double *, hipStream_t);           \
    template hipError_t launch_relax_setup<T>(const Dev<T> &, const Tiles &, const float *, const Relax<T> &,      \
                                              hipStream_t);                                                        \
    template hipError_t launch_relax_zero<T>(const Tiles &, const Relax<T> &, hipStream_t);                         \
    template hipError_t launch_relax_compact<T>(const Dev<T> &, const Tiles &, const Relax<T> &, hipStream_t);      \
    template hipError_t launch_relax<T>(const Dev<T> &, const Tiles &, const Relax<T> &, bool, hipStream_t);

EL_INST(float)
EL_INST(double)

}  // namespace el
