// geometry.hip -- per-plan geometry kernels for gfx950 (Algorithm A2 kernels 1-4):
//   smooth_xy / smooth_z_factors       smoothed density and per-voxel correction
//                                      factors (Section 2.1, A1 step 1), with
//                                      smooth_pass / smooth_last_factors for
//                                      radii beyond the LDS tiles
//   beamlet_setup                      beamlet frames and angles (A1 step 3)
//   ray_trace                          entrance point and uniform-sampled
//                                      radiological-depth / weight-drift tables
//                                      (A1 steps 4-6, Section 2.2)
#include "fspb_internal.h"
#include "kernels.h"

#include <math.h>

namespace fspb {

// ---------------------------------------------------------------------------
// Kernel 1: separable Gaussian smoothing with clamp-to-edge borders.  The
// normalised 3D cube-truncated Gaussian is the product of three normalised
// 1D kernels, so three 1D passes give the same sums.  The single-axis passes
// below (one thread per voxel; the 64 lanes of a wave read consecutive x, so
// every tap load is coalesced whatever the pass axis; taps taken eight at a
// time so that their loads are in flight together; 32-bit indices, grids
// hold fewer than 2^31 voxels) serve radii beyond the LDS-staged kernels
// further down, which sum the same taps in the same order.
__device__ __forceinline__ float smooth_taps(const float* __restrict__ base, int c, int n, int stride,
                                            const float* __restrict__ w, int r) {
    float acc = 0.0f;
    for (int d0 = -r; d0 <= r; d0 += 8) {
        float x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int d = min(d0 + q, r);   // past the last tap: a repeat with weight 0
            x[q] = base[min(max(c + d, 0), n - 1) * stride];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (d0 + q <= r) acc = fmaf(w[d0 + q + r], x[q], acc);
    }
    return acc;
}

__global__ __launch_bounds__(256) void smooth_pass(const float* __restrict__ in,
                                                   float* __restrict__ out, int nx, int ny,
                                                   int nz, int axis,
                                                   const float* __restrict__ w, int r,
                                                   float* __restrict__ copy) {
    const int n = nx * ny * nz;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (copy) copy[v] = in[v];   // the input grid, copied on the way
    const int i = v % nx;
    const int j = (v / nx) % ny;
    const int k = v / (nx * ny);
    float acc;
    if (axis == 0)
        acc = smooth_taps(in + (v - i), i, nx, 1, w, r);
    else if (axis == 1)
        acc = smooth_taps(in + (k * ny * nx + i), j, ny, nx, w, r);
    else
        acc = smooth_taps(in + (j * nx + i), k, nz, nx * ny, w, r);
    out[v] = acc;
}

// Last (z) pass fused with the per-voxel factors of Section 2.1:
//   fac = (f_u1(rho), f_u2(rho_hat), f_w1(rho_hat), f_w2(rho_hat)),
// densities clamped to the commissioned range.
__global__ __launch_bounds__(256) void smooth_last_factors(
    const float* __restrict__ in, const float* __restrict__ rho, float* __restrict__ rhohat,
    float4* __restrict__ fac, int nx, int ny, int nz, const float* __restrict__ w, int r,
    const float* __restrict__ tabs, DensTabs dt) {
    const int n = nx * ny * nz;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int i = v % nx;
    const int j = (v / nx) % ny;
    const int k = v / (nx * ny);
    const float acc = smooth_taps(in + (j * nx + i), k, nz, nx * ny, w, r);
    rhohat[v] = acc;
    float rc = fminf(fmaxf(rho[v], dt.rho_min), dt.rho_max);
    float hc = fminf(fmaxf(acc, dt.rho_min), dt.rho_max);
    fac[v] = make_float4(dens_lookup(tabs, dt.fu1, rc), dens_lookup(tabs, dt.fu2, hc),
                         dens_lookup(tabs, dt.fw1, hc), dens_lookup(tabs, dt.fw2, hc));
}

// LDS-staged form of the three passes, for radii up to kSmMaxR voxels: a
// workgroup stages a clamped (clamp-to-edge) neighbourhood of its tile in LDS
// and sums the taps there, in the order smooth_taps uses, so the results are
// bitwise those of the single-axis passes.
constexpr int kSmTX = 64, kSmTY = 16, kSmTZ = 16, kSmMaxR = 24;

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  The
// tiles of these kernels share their halos with their neighbours, so each
// XCD takes a contiguous run of tiles (x fastest): workgroup q works on tile
// (q mod 8) per + q / 8 of a grid of 8 per workgroups; tiles past n_tiles
// return at once.
__device__ __forceinline__ int xcd_tile(int per) {
    return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// x and y passes of one 64 x 16 tile of a z-plane: the (64 + 2 rx) x
// (16 + 2 ry) neighbourhood is staged, the x-pass runs on every staged row,
// the y-pass on its results.  A wave takes whole rows, lane = x offset.  The
// staged interior is the handle's copy of the input when `copy` is set.
__global__ __launch_bounds__(256) void smooth_xy(const float* __restrict__ in,
                                                 float* __restrict__ out, int nx, int ny, int nz,
                                                 const float* __restrict__ wx, int rx,
                                                 const float* __restrict__ wy, int ry,
                                                 float* __restrict__ copy, int per) {
    extern __shared__ float sm[];
    constexpr int kWaves = 256 / kWave;
    const int nbx = (nx + kSmTX - 1) / kSmTX, nby = (ny + kSmTY - 1) / kSmTY;
    const int tile = xcd_tile(per);
    if (tile >= nbx * nby * nz) return;   // the whole workgroup
    const int W = kSmTX + 2 * rx, H = kSmTY + 2 * ry;
    float* s_in = sm;           // [H][W]
    float* s_x = sm + W * H;    // [H][kSmTX]
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int i0 = (tile % nbx) * kSmTX, j0 = ((tile / nbx) % nby) * kSmTY;
    const long plane = (long)(tile / (nbx * nby)) * nx * ny;
    for (int jj = wid; jj < H; jj += kWaves) {
        const float* src = in + plane + (long)min(max(j0 - ry + jj, 0), ny - 1) * nx;
        for (int ii = lane; ii < W; ii += kWave) s_in[jj * W + ii] = src[min(max(i0 - rx + ii, 0), nx - 1)];
    }
    __syncthreads();
    for (int jj = wid; jj < H; jj += kWaves) {
        const float* row = s_in + jj * W + lane;   // tap d (-rx..rx) at row[d + rx]
        float acc = 0.0f;
        for (int d = 0; d <= 2 * rx; ++d) acc = fmaf(wx[d], row[d], acc);
        s_x[jj * kSmTX + lane] = acc;
    }
    __syncthreads();
    const int i = i0 + lane;
    if (i >= nx) return;
    for (int jj = wid; jj < kSmTY; jj += kWaves) {
        const int j = j0 + jj;
        if (j >= ny) break;
        const float* col = s_x + jj * kSmTX + lane;   // tap d at col[(d + ry) kSmTX]
        float acc = 0.0f;
        for (int d = 0; d <= 2 * ry; ++d) acc = fmaf(wy[d], col[d * kSmTX], acc);
        const long v = plane + (long)j * nx + i;
        out[v] = acc;
        if (copy) copy[v] = s_in[(jj + ry) * W + lane + rx];
    }
}

// z pass of one 64 x 16 tile of an x-z plane (fixed j), fused with the
// per-voxel factors as smooth_last_factors computes them.
__global__ __launch_bounds__(256) void smooth_z_factors(
    const float* __restrict__ in, const float* __restrict__ rho, float* __restrict__ rhohat,
    float4* __restrict__ fac, int nx, int ny, int nz, const float* __restrict__ wz, int rz,
    const float* __restrict__ tabs, DensTabs dt, int per) {
    extern __shared__ float sm[];   // [16 + 2 rz][kSmTX]
    constexpr int kWaves = 256 / kWave;
    const int nbx = (nx + kSmTX - 1) / kSmTX, nbk = (nz + kSmTZ - 1) / kSmTZ;
    const int tile = xcd_tile(per);
    if (tile >= nbx * nbk * ny) return;   // the whole workgroup
    const int H = kSmTZ + 2 * rz;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int i0 = (tile % nbx) * kSmTX, k0 = ((tile / nbx) % nbk) * kSmTZ, j = tile / (nbx * nbk);
    const int gi = min(i0 + lane, nx - 1);
    for (int kk = wid; kk < H; kk += kWaves) {
        const int gk = min(max(k0 - rz + kk, 0), nz - 1);
        sm[kk * kSmTX + lane] = in[((long)gk * ny + j) * nx + gi];
    }
    __syncthreads();
    const int i = i0 + lane;
    if (i >= nx) return;
    for (int kk = wid; kk < kSmTZ; kk += kWaves) {
        const int k = k0 + kk;
        if (k >= nz) break;
        const float* col = sm + kk * kSmTX + lane;   // tap d at col[(d + rz) kSmTX]
        float acc = 0.0f;
        for (int d = 0; d <= 2 * rz; ++d) acc = fmaf(wz[d], col[d * kSmTX], acc);
        const long v = ((long)k * ny + j) * nx + i;
        rhohat[v] = acc;
        const float rc = fminf(fmaxf(rho[v], dt.rho_min), dt.rho_max);
        const float hc = fminf(fmaxf(acc, dt.rho_min), dt.rho_max);
        fac[v] = make_float4(dens_lookup(tabs, dt.fu1, rc), dens_lookup(tabs, dt.fu2, hc),
                             dens_lookup(tabs, dt.fw1, hc), dens_lookup(tabs, dt.fw2, hc));
    }
}

// ---------------------------------------------------------------------------
// Kernel 2: beamlet frames in FP64, one thread per beamlet.
// Beam (gantry phi, couch psi): central axis cax = Rc (-sin phi, cos phi, 0),
// lateral axes ex = Rc (cos phi, sin phi, 0), ey = Rc (0, 0, 1), with Rc the
// couch rotation about y; source = iso - SAD cax.  Beamlet (n, m) aims at the
// isocentre-plane point iso + a ex + b ey; its own lateral axes are ex made
// orthogonal to the beamlet direction and ey_i = ex_i x d_i; theta is the
// angle to the central axis (Eq. 2 definitions).
struct GridBox {
    double lo[3], hi[3];
    double step;  // ray sample step
};

__device__ inline double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ inline void rot_couch(double psi, const double* a, double* b) {
    double c = cos(psi), s = sin(psi);
    b[0] = c * a[0] + s * a[2];
    b[1] = a[1];
    b[2] = -s * a[0] + c * a[2];
}

__global__ __launch_bounds__(256) void beamlet_setup(const BeamIn* __restrict__ beams,
                                                     int n_beams, int n_beamlets, GridBox box,
                                                     Frame64* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_beamlets) return;
    int b = 0;
    while (b + 1 < n_beams && beams[b + 1].first <= i) ++b;
    const BeamIn bm = beams[b];
    int loc = i - bm.first;
    int n = loc / bm.nbx, m = loc % bm.nbx;
    double phi = bm.gantry;
    double c0[3] = {-sin(phi), cos(phi), 0.0}, ex0[3] = {cos(phi), sin(phi), 0.0},
           ey0[3] = {0.0, 0.0, 1.0};
    double cax[3], ex[3], ey[3];
    rot_couch(bm.couch, c0, cax);
    rot_couch(bm.couch, ex0, ex);
    rot_couch(bm.couch, ey0, ey);
    Frame64 f;
    for (int q = 0; q < 3; ++q) f.src[q] = bm.iso[q] - bm.sad * cax[q];
    double a = (m - 0.5 * (bm.nbx - 1)) * bm.wx + bm.cx;
    double bb = (n - 0.5 * (bm.nby - 1)) * bm.wy + bm.cy;
    double d[3];
    for (int q = 0; q < 3; ++q) d[q] = bm.sad * cax[q] + a * ex[q] + bb * ey[q];
    double nd = sqrt(dot3(d, d));
    for (int q = 0; q < 3; ++q) f.d[q] = d[q] / nd;
    double pr = dot3(ex, f.d);
    double e[3];
    for (int q = 0; q < 3; ++q) e[q] = ex[q] - pr * f.d[q];
    double ne = sqrt(dot3(e, e));
    for (int q = 0; q < 3; ++q) f.ex[q] = e[q] / ne;
    f.ey[0] = f.ex[1] * f.d[2] - f.ex[2] * f.d[1];
    f.ey[1] = f.ex[2] * f.d[0] - f.ex[0] * f.d[2];
    f.ey[2] = f.ex[0] * f.d[1] - f.ex[1] * f.d[0];
    f.theta = atan(sqrt(a * a + bb * bb) / bm.sad);
    f.beam = b;
    f.sad = bm.sad;
    f.x0 = 0.5 * bm.wx;
    f.y0 = 0.5 * bm.wy;
    // slab clip of the axis against the grid box
    double s_in = -1e300, s_out = 1e300;
    bool miss = false;
    for (int q = 0; q < 3; ++q) {
        if (f.d[q] == 0.0) {
            if (f.src[q] < box.lo[q] || f.src[q] > box.hi[q]) miss = true;
            continue;
        }
        double t1 = (box.lo[q] - f.src[q]) / f.d[q], t2 = (box.hi[q] - f.src[q]) / f.d[q];
        s_in = fmax(s_in, fmin(t1, t2));
        s_out = fmin(s_out, fmax(t1, t2));
    }
    s_in = fmax(s_in, 0.0);
    f.s_in = s_in;
    f.s_cover = 0.0;
    f.n_samples = 0;
    if (!miss && s_in < s_out) {
        double cover = -1e300;
        for (int c = 0; c < 8; ++c) {
            double p[3] = {(c & 1) ? box.hi[0] : box.lo[0], (c & 2) ? box.hi[1] : box.lo[1],
                           (c & 4) ? box.hi[2] : box.lo[2]};
            double v[3] = {p[0] - f.src[0], p[1] - f.src[1], p[2] - f.src[2]};
            cover = fmax(cover, dot3(v, f.d));
        }
        f.s_cover = cover;
        // table runs past the deepest box point by one sample
        f.n_samples = (int)floor((cover - s_in) / box.step) + 2;
    }
    out[i] = f;
}

// ---------------------------------------------------------------------------
// Kernels 3-4: one wavefront per beamlet, FP64.
__device__ inline double trilinear64(const float* __restrict__ rho, const TraceGrid& g,
                                     const double* p) {
    double gx = (p[0] - g.o[0]) * g.inv[0], gy = (p[1] - g.o[1]) * g.inv[1],
           gz = (p[2] - g.o[2]) * g.inv[2];
    double fx0 = floor(gx), fy0 = floor(gy), fz0 = floor(gz);
    int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
    double fx = gx - fx0, fy = gy - fy0, fz = gz - fz0;
    int x0 = min(max(ix, 0), g.n[0] - 1), x1 = min(max(ix + 1, 0), g.n[0] - 1);
    int y0 = min(max(iy, 0), g.n[1] - 1), y1 = min(max(iy + 1, 0), g.n[1] - 1);
    int z0 = min(max(iz, 0), g.n[2] - 1), z1 = min(max(iz + 1, 0), g.n[2] - 1);
    long sx = 1, sy = g.n[0], sz = (long)g.n[0] * g.n[1];
    auto at = [&](int x, int y, int z) { return (double)rho[z * sz + y * sy + x * sx]; };
    double c00 = at(x0, y0, z0) * (1 - fx) + at(x1, y0, z0) * fx;
    double c10 = at(x0, y1, z0) * (1 - fx) + at(x1, y1, z0) * fx;
    double c01 = at(x0, y0, z1) * (1 - fx) + at(x1, y0, z1) * fx;
    double c11 = at(x0, y1, z1) * (1 - fx) + at(x1, y1, z1) * fx;
    double c0 = c00 * (1 - fy) + c10 * fy;
    double c1 = c01 * (1 - fy) + c11 * fy;
    return c0 * (1 - fz) + c1 * fz;
}

__device__ inline double b_lookup64(const float* __restrict__ v, DTab t, double rho_c) {
    double c = (rho_c - (double)t.start) / (double)t.step;
    c = fmin(fmax(c, 0.0), (double)(t.n - 1));
    int i = (int)floor(c);
    i = max(min(i, t.n - 2), 0);
    double f = (t.n > 1) ? c - i : 0.0;
    double a = v[t.off + i], b = v[t.off + min(i + 1, t.n - 1)];
    return (1.0 - f) * a + f * b;
}

__device__ inline double wave_incl_scan(double x, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        double y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ inline double wave_min64(double x) {
    for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, kWave));
    return x;
}

__global__ __launch_bounds__(256) void ray_trace(const Frame64* __restrict__ frames,
                                                 int n_beamlets, const float* __restrict__ rho,
                                                 TraceGrid g, TraceParams tp,
                                                 const float* __restrict__ dtabs, DensTabs dt,
                                                 float2* __restrict__ tT, float4* __restrict__ tTW,
                                                 float2* __restrict__ tW2,
                                                 BeamletDesc* __restrict__ desc,
                                                 TraceInfo* __restrict__ info) {
    int lane = threadIdx.x & (kWave - 1);
    int ib = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (ib >= n_beamlets) return;  // wave-uniform exit
    const Frame64 f = frames[ib];
    const double d = tp.step;
    auto sample = [&](int k) {
        double s = f.s_in + k * d;
        double p[3] = {f.src[0] + s * f.d[0], f.src[1] + s * f.d[1], f.src[2] + s * f.d[2]};
        return trilinear64(rho, g, p);
    };
    const int N = min(f.n_samples, tp.k_stride);  // the host reserves k_stride >= n_samples
    // entrance: first sample at or above the surface threshold (ballot)
    int ke = -1;
    double margin = 1e300;
    for (int base = 0; base < N; base += kWave) {
        int k = base + lane;
        double r = (k < N) ? sample(k) : -1.0;
        bool at_body = (k < N) && (r >= tp.rho_surface);
        unsigned long long ball = __ballot(at_body);
        double m = (k < N) ? fabs(r - tp.rho_surface) : 1e300;
        if (ball) {
            ke = base + __ffsll((long long)ball) - 1;
            margin = fmin(margin, wave_min64(k <= ke ? m : 1e300));
            break;
        }
        margin = fmin(margin, wave_min64(m));
    }
    BeamletDesc o = {};
    TraceInfo ti = {};
    ti.n_samples = N;
    ti.k_entry = ke;
    ti.margin = margin;
    const double* P0 = tp.p0;
    double v0[3] = {P0[0] - f.src[0], P0[1] - f.src[1], P0[2] - f.src[2]};
    for (int q = 0; q < 3; ++q) {
        o.d[q] = (float)f.d[q];
        o.ex[q] = (float)f.ex[q];
        o.ey[q] = (float)f.ey[q];
    }
    o.c_x = (float)(v0[0] * f.ex[0] + v0[1] * f.ex[1] + v0[2] * f.ex[2]);
    o.c_y = (float)(v0[0] * f.ey[0] + v0[1] * f.ey[1] + v0[2] * f.ey[2]);
    o.sad = (float)f.sad;
    o.theta = (float)f.theta;
    o.beam = f.beam;
    o.j_last = 0;
    o.nx2 = (float)(-2.0 * f.x0);   // exactly -2 (float)x0
    o.ny2 = (float)(-2.0 * f.y0);
    {
        double c = f.theta / tp.theta_step;
        c = fmin(fmax(c, 0.0), (double)(tp.n_theta - 1));
        int r = (tp.n_theta > 1) ? min((int)floor(c), tp.n_theta - 2) : 0;
        o.a_off = r * tp.n_A;
        o.th_frac = (tp.n_theta > 1) ? (float)(c - r) : 0.0f;
    }
    o.tab_off = ib * tp.k_stride;
    if (ke < 0) {
        o.hit = 0;
        o.K = 0;
        o.c_t = -1e30f;
        if (lane == 0) {
            desc[ib] = o;
            info[ib] = ti;
        }
        return;
    }
    const int K = N - ke;
    const double s_entry = f.s_in + ke * d;
    o.hit = 1;
    o.K = K;
    o.j_last = max(K - 2, 0);
    o.s_entry = (float)s_entry;
    o.c_t = (float)(v0[0] * f.d[0] + v0[1] * f.d[1] + v0[2] * f.d[2] - s_entry);
    ti.s_entry = s_entry;

    // tables: T_j = sum_{l<j} d (rho_l + rho_{l+1}) / 2 from the entrance,
    // W_c likewise with b_c(clamped rho); exclusive wave scans in FP64.
    // The samples of the next 64 are gathered while the current ones are
    // scanned; the first of them is the last lane's right neighbour.
    double cT = 0.0, c1 = 0.0, c2 = 0.0;
    double r_next = (lane < K) ? sample(ke + lane) : 0.0;
    for (int base = 0; base < K; base += kWave) {
        const int j = base + lane;
        const double r = r_next;
        r_next = (j + kWave < K) ? sample(ke + j + kWave) : 0.0;
        double rn = __shfl_down(r, 1, kWave);
        const double first_next = __shfl(r_next, 0, kWave);
        if (lane == kWave - 1) rn = first_next;
        double rc = fmin(fmax(r, (double)dt.rho_min), (double)dt.rho_max);
        double rcn = fmin(fmax(rn, (double)dt.rho_min), (double)dt.rho_max);
        bool has_next = j + 1 < K;
        double iT = has_next ? d * 0.5 * (r + rn) : 0.0;
        double i1 = has_next ? d * 0.5 * (b_lookup64(dtabs, dt.b1, rc) + b_lookup64(dtabs, dt.b1, rcn)) : 0.0;
        double i2 = has_next ? d * 0.5 * (b_lookup64(dtabs, dt.b2, rc) + b_lookup64(dtabs, dt.b2, rcn)) : 0.0;
        double sT = wave_incl_scan(iT, lane), s1 = wave_incl_scan(i1, lane),
               s2 = wave_incl_scan(i2, lane);
        double T = cT + sT - iT, W1 = c1 + s1 - i1, W2 = c2 + s2 - i2;
        if (j < K) {
            tT[o.tab_off + j] = make_float2((float)T, (float)iT);
            if (tTW) {
                tTW[o.tab_off + j] = make_float4((float)T, (float)iT, (float)W1, (float)i1);
                tW2[o.tab_off + j] = make_float2((float)W2, (float)i2);
            }
        }
        cT += __shfl(sT, kWave - 1, kWave);
        c1 += __shfl(s1, kWave - 1, kWave);
        c2 += __shfl(s2, kWave - 1, kWave);
    }
    if (lane == 0) {
        desc[ib] = o;
        info[ib] = ti;
    }
}

// ---------------------------------------------------------------------------
void launch_smooth(const float* rho, float* copy, hipEvent_t after_copy, float* tmp0, float* tmp1,
                   float* rhohat, float4* fac, int nx, int ny, int nz, const float* w3,
                   const int r[3], const float* dtabs, const DensTabs& dt, hipStream_t s) {
    long n = (long)nx * ny * nz;
    int blocks = (int)((n + 255) / 256);
    const float* wx = w3;
    const float* wy = w3 + (2 * r[0] + 1);
    const float* wz = wy + (2 * r[1] + 1);
    if (r[0] <= kSmMaxR && r[1] <= kSmMaxR && r[2] <= kSmMaxR) {
        const long bx = (nx + kSmTX - 1) / kSmTX;
        const long t_xy = bx * ((ny + kSmTY - 1) / kSmTY) * nz;   // tiles of each kernel
        const long t_z = bx * ((nz + kSmTZ - 1) / kSmTZ) * ny;
        const int per_xy = (int)((t_xy + 7) / 8), per_z = (int)((t_z + 7) / 8);
        const size_t sh_xy =
            sizeof(float) * (size_t)(kSmTY + 2 * r[1]) * (kSmTX + 2 * r[0] + kSmTX);
        hipLaunchKernelGGL(smooth_xy, dim3(8 * per_xy), dim3(256), sh_xy, s, rho, tmp0, nx, ny,
                           nz, wx, r[0], wy, r[1], copy, per_xy);
        if (after_copy) (void)hipEventRecord(after_copy, s);
        const size_t sh_z = sizeof(float) * (size_t)(kSmTZ + 2 * r[2]) * kSmTX;
        hipLaunchKernelGGL(smooth_z_factors, dim3(8 * per_z), dim3(256), sh_z, s,
                           (const float*)tmp0, copy ? (const float*)copy : rho, rhohat, fac, nx,
                           ny, nz, wz, r[2], dtabs, dt, per_z);
        return;
    }
    hipLaunchKernelGGL(smooth_pass, dim3(blocks), dim3(256), 0, s, rho, tmp0, nx, ny, nz, 0, wx, r[0],
                       copy);
    if (after_copy) (void)hipEventRecord(after_copy, s);
    hipLaunchKernelGGL(smooth_pass, dim3(blocks), dim3(256), 0, s, (const float*)tmp0, tmp1, nx, ny,
                       nz, 1, wy, r[1], (float*)nullptr);
    hipLaunchKernelGGL(smooth_last_factors, dim3(blocks), dim3(256), 0, s, (const float*)tmp1,
                       copy ? (const float*)copy : rho, rhohat, fac, nx, ny, nz, wz, r[2], dtabs, dt);
}

void launch_setup(const BeamIn* beams, int n_beams, int n_beamlets, const double lo[3],
                  const double hi[3], double step, Frame64* out, hipStream_t s) {
    GridBox box;
    for (int q = 0; q < 3; ++q) {
        box.lo[q] = lo[q];
        box.hi[q] = hi[q];
    }
    box.step = step;
    hipLaunchKernelGGL(beamlet_setup, dim3((n_beamlets + 255) / 256), dim3(256), 0, s, beams,
                       n_beams, n_beamlets, box, out);
}

// ---------------------------------------------------------------------------
// Exact radiological path (Siddon): one thread per beamlet, FP64.  The axis
// is cut at every voxel-boundary plane between the grid-box entry and exit;
// the three axes' crossings are merged in order (each computed directly from
// its plane, not accumulated), zero-length pieces (edges, corners) are
// dropped, and each segment takes the density of the voxel holding its
// midpoint.  The entrance is the start of the first segment whose voxel
// density reaches rho_surface; records start there.  The descriptor's
// entrance, depth offset and record count are rewritten.
__global__ __launch_bounds__(256) void siddon_trace(const Frame64* __restrict__ frames,
                                                    int n_beamlets, const float* __restrict__ rho,
                                                    TraceGrid g, TraceParams tp, int stride,
                                                    const float* __restrict__ dtabs, DensTabs dt,
                                                    float4* __restrict__ sid,
                                                    BeamletDesc* __restrict__ desc,
                                                    TraceInfo* __restrict__ info) {
    const int ib = blockIdx.x * blockDim.x + threadIdx.x;
    if (ib >= n_beamlets) return;
    const Frame64 f = frames[ib];
    BeamletDesc o = desc[ib];
    TraceInfo ti = info[ib];
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = g.o[a] - 0.5 * g.del[a];
        hi[a] = g.o[a] + (g.n[a] - 0.5) * g.del[a];
    }
    // grid-box clip of the axis (as for the uniform samples)
    double s_in = -1e300, s_out = 1e300;
    bool miss = false;
    for (int a = 0; a < 3; ++a) {
        if (f.d[a] == 0.0) {
            if (f.src[a] < lo[a] || f.src[a] > hi[a]) miss = true;
            continue;
        }
        const double t1 = (lo[a] - f.src[a]) / f.d[a], t2 = (hi[a] - f.src[a]) / f.d[a];
        s_in = fmax(s_in, fmin(t1, t2));
        s_out = fmin(s_out, fmax(t1, t2));
    }
    s_in = fmax(s_in, 0.0);
    o.hit = 0;
    o.K = 0;
    o.j_last = 0;
    o.c_t = -1e30f;
    o.tab_off = ib * stride;
    if (!miss && s_in < s_out) {
        // next plane crossing per axis, in travel order
        int m[3], step[3];
        for (int a = 0; a < 3; ++a) {
            step[a] = f.d[a] > 0.0 ? 1 : -1;
            if (f.d[a] == 0.0) {
                m[a] = -1;
                continue;
            }
            // first plane index whose crossing lies beyond s_in
            const double c = (f.src[a] + s_in * f.d[a] - lo[a]) / g.del[a];
            int k = step[a] > 0 ? (int)floor(c) + 1 : (int)ceil(c) - 1;
            while (k >= 0 && k <= g.n[a] && (lo[a] + k * g.del[a] - f.src[a]) / f.d[a] <= s_in) k += step[a];
            m[a] = k;
        }
        auto crossing = [&](int a) -> double {
            if (m[a] < 0 || m[a] > g.n[a]) return 1e300;
            return (lo[a] + m[a] * g.del[a] - f.src[a]) / f.d[a];
        };
        const long sy = g.n[0], sz = (long)g.n[0] * g.n[1];
        double s = s_in, s_entry = 0.0, T = 0.0, W1 = 0.0, W2 = 0.0;
        int K = 0;
        bool entered = false;
        while (s < s_out && K < stride) {
            const double c0 = crossing(0), c1 = crossing(1), c2 = crossing(2);
            double s_next = fmin(fmin(c0, c1), fmin(c2, s_out));
            for (int a = 0; a < 3; ++a)
                if (crossing(a) == s_next) m[a] += step[a];
            if (!(s_next > s)) continue;          // zero-length piece
            const double mid = 0.5 * (s + s_next);
            int idx[3];
            for (int a = 0; a < 3; ++a)
                idx[a] = min(max((int)floor((f.src[a] + mid * f.d[a] - lo[a]) * g.inv[a]), 0), g.n[a] - 1);
            const double r = rho[idx[2] * sz + idx[1] * sy + idx[0]];
            if (!entered && r >= tp.rho_surface) {
                entered = true;
                s_entry = s;
            }
            if (entered) {
                const double rc = fmin(fmax(r, (double)dt.rho_min), (double)dt.rho_max);
                const double b1 = b_lookup64(dtabs, dt.b1, rc), b2 = b_lookup64(dtabs, dt.b2, rc);
                const long q = 2 * ((long)o.tab_off + K);
                sid[q] = make_float4((float)(s - s_entry), (float)T, (float)r, (float)W1);
                sid[q + 1] = make_float4((float)b1, (float)W2, (float)b2, 0.0f);
                const double len = s_next - s;
                T += r * len;
                W1 += b1 * len;
                W2 += b2 * len;
                ++K;
            }
            s = s_next;
        }
        if (entered) {
            double v0[3];
            for (int a = 0; a < 3; ++a) v0[a] = tp.p0[a] - f.src[a];
            o.hit = 1;
            o.K = K;
            o.j_last = max(K - 2, 0);
            o.s_entry = (float)s_entry;
            o.c_t = (float)(v0[0] * f.d[0] + v0[1] * f.d[1] + v0[2] * f.d[2] - s_entry);
            ti.s_entry = s_entry;
        }
    }
    desc[ib] = o;
    info[ib] = ti;
}

void launch_siddon(const Frame64* frames, int n_beamlets, const float* rho, const TraceGrid& g,
                   const TraceParams& tp, int stride, const float* dtabs, const DensTabs& dt,
                   float4* sid, BeamletDesc* desc, TraceInfo* info, hipStream_t s) {
    hipLaunchKernelGGL(siddon_trace, dim3((n_beamlets + 255) / 256), dim3(256), 0, s, frames,
                       n_beamlets, rho, g, tp, stride, dtabs, dt, sid, desc, info);
}

void launch_trace(const Frame64* frames, int n_beamlets, const float* rho, const TraceGrid& g,
                  const TraceParams& tp, const float* dtabs, const DensTabs& dt, float2* tT,
                  float4* tTW, float2* tW2, BeamletDesc* desc, TraceInfo* info, hipStream_t s) {
    int waves_per_block = 4;
    int blocks = (n_beamlets + waves_per_block - 1) / waves_per_block;
    hipLaunchKernelGGL(ray_trace, dim3(blocks), dim3(waves_per_block * kWave), 0, s, frames,
                       n_beamlets, rho, g, tp, dtabs, dt, tT, tTW, tW2, desc, info);
}

}  // namespace fspb
