// Device kernels of the recycled shifted solver (gfx950, FP64).
//
// The systems are (A + gamma E) x = b with A = K^T K (K: zero-boundary 2-D
// convolution by the PSF) and E = D^T W D (D: forward differences, W diagonal
// weights), Section 2.1 eq. blkeqn.  The unit of cost is one application of
// the shifted operator (Section 6), so the stencil that applies it is the
// centre of this file:
//
//   * k_apply (stencil.hpp): one workgroup computes a TY x TX tile of
//     cA K^T K v + cE E v.  v is staged once into LDS with a 2r halo; K^T K is
//     applied as four 1-D passes (x conv, x corr, y conv, y corr) for a
//     rank-1 PSF, or as a direct 2-D conv + corr otherwise, with the
//     intermediate masked to the image after each forward pass (zero
//     boundary).  Each thread produces RB consecutive outputs per pass from a
//     register window, so an output costs (RB+S-1)/RB LDS reads instead of S.
//   * the persistent CG kernel lives in cg.hip; this file holds the
//     operator-application, weight, tall-skinny and gradient kernels.
#include "internal.hpp"
#include "outer.hpp"
#include "stencil.hpp"

#include <algorithm>

#include <hip/hip_runtime.h>

namespace rsr {

int tile_lds_doubles(int ty, int tx, int sy, int sx, int sep)
{
    const Geo g = make_geo(ty, tx, sy, sx, sep);
    return g.total < 2048 ? 2048 : g.total;   // the persistent kernel reuses it as reduction scratch
}

int taps_lds_doubles(int s, int sep) { return taps_doubles(s, sep); }

// ---------------------------------------------------------- apply kernel --
// y = cA A v + cE E v for one tile per workgroup; blockIdx.y selects the job.
__global__ __launch_bounds__(NT) void k_apply(const InstDev *__restrict__ insts, const Jobs<ApplyJob> jobs)
{
    extern __shared__ double lds[];
    const ApplyJob J = jobs[blockIdx.y];
    const InstDev I = insts[J.inst];
    const int ntile = I.nty * I.ntx;
    if ((int)blockIdx.x >= ntile) return;
    const int y0 = (blockIdx.x / I.ntx) * I.ty, x0 = (blockIdx.x % I.ntx) * I.tx;
    const Geo g = make_geo(I.ty, I.tx, I.sy, I.sx, I.sep);
    constexpr int NBW = 12;   // window rows per thread whose loads are issued together
    const double *__restrict__ vin = J.v;
    const WinMap wm = win_map(g.W0);
    const int lj = threadIdx.x & ((1 << wm.lw_log) - 1);
    const int gx = x0 - g.hx + lj;
    const bool colok = lj < g.W0 && gx >= 0 && gx < I.nx;
    double *taps = lds + g.total;
    EWts ew;
    tile_E_load(I, y0, x0, 0, J.cE, ew);   // in flight with the window loads
    stage_taps(I, taps);
    for (int li0 = threadIdx.x >> wm.lw_log; li0 < g.H0; li0 += wm.rs * NBW) {
        double v[NBW];
#pragma unroll
        for (int u = 0; u < NBW; ++u) {
            const int li = li0 + u * wm.rs;
            const int gy = y0 - g.hy + li;
            const bool ok = colok && li < g.H0 && gy >= 0 && gy < I.ny;
            v[u] = ok ? gp(vin)[(long)gy * I.nx + gx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NBW; ++u) {
            const int li = li0 + u * wm.rs;
            if (lj < g.W0 && li < g.H0) lds[li * g.P0 + lj] = v[u];
        }
    }
    __syncthreads();
    tile_E(I, g, lds, y0, x0, J.cE, ew);
    if (J.cA != 0.0) tile_A(I, g, lds, taps, y0, x0, J.cA);
    const double *ebuf = lds + g.offE;
    for (int k = threadIdx.x; k < I.ty * I.tx; k += NT) {
        const int i = k >> I.ltx, j = k & (I.tx - 1);
        const int gy = y0 + i, gx = x0 + j;
        if (gy < I.ny && gx < I.nx) gp(J.y)[(long)gy * I.nx + gx] = ebuf[i * g.PE + j];
    }
}

// K v (op 3) or K^T v (op 4) straight from global memory (setup work only).
__global__ __launch_bounds__(NT) void k_blur(const InstDev *__restrict__ insts,
                                             const ApplyJob *__restrict__ jobs)
{
    const ApplyJob J = jobs[blockIdx.y];
    const InstDev I = insts[J.inst];
    const long n = (long)I.ny * I.nx;
    const int cy = I.sy / 2, cx = I.sx / 2;
    for (long gi = blockIdx.x * (long)NT + threadIdx.x; gi < n; gi += (long)gridDim.x * NT) {
        const int i = gi / I.nx, j = gi % I.nx;
        double s = 0.0;
        for (int a = 0; a < I.sy; ++a) {
            const int ii = J.op == 3 ? i + cy - a : i - cy + a;
            if (ii < 0 || ii >= I.ny) continue;
            for (int c = 0; c < I.sx; ++c) {
                const int jj = J.op == 3 ? j + cx - c : j - cx + c;
                if (jj < 0 || jj >= I.nx) continue;
                const double h = I.sep == 1 ? I.fy[a] * I.fx[c] : I.psf[a * I.sx + c];
                s = fma(h, J.v[(long)ii * I.nx + jj], s);
            }
        }
        J.y[gi] = s;
    }
}

hipError_t launch_apply(const InstDev *inst_dev, const InstDev &ih, const ApplyJob *jobs_dev,
                        const ApplyJob *jobs_host, int njobs, size_t lds, hipStream_t s)
{
    if (!jobs_dev && njobs > KJ) return hipErrorInvalidValue;
    dim3 grid(ih.nty * ih.ntx, njobs);
    hipLaunchKernelGGL(k_apply, grid, dim3(NT), lds, s, inst_dev, make_jobs(jobs_dev, jobs_host, njobs));
    return hipGetLastError();
}

hipError_t launch_blur(const InstDev *inst_dev, const InstDev &ih, const ApplyJob *jobs_dev, int njobs,
                       hipStream_t s)
{
    long n = (long)ih.ny * ih.nx;
    int gx = (int)((n + NT - 1) / NT);
    if (gx > 4096) gx = 4096;
    hipLaunchKernelGGL(k_blur, dim3(gx, njobs), dim3(NT), 0, s, inst_dev, jobs_dev);
    return hipGetLastError();
}

// -------------------------------------------------------- weight kernels --
__global__ void k_weights(const double *__restrict__ x, double beta, double *__restrict__ wh,
                          double *__restrict__ wv, int ny, int nx)
{
    const long n = (long)ny * nx;
    for (long gi = blockIdx.x * (long)blockDim.x + threadIdx.x; gi < n; gi += (long)gridDim.x * blockDim.x) {
        const int i = gi / nx, j = gi % nx;
        const double xc = x[gi];
        double a = 0.0, b = 0.0;
        if (j < nx - 1) { const double d = x[gi + 1] - xc; a = 1.0 / sqrt(d * d + beta); }
        if (i < ny - 1) { const double d = x[gi + nx] - xc; b = 1.0 / sqrt(d * d + beta); }
        wh[gi] = a;
        wv[gi] = b;
    }
}

__global__ void k_copy_weights(const double *__restrict__ wh_in, const double *__restrict__ wv_in,
                               double *__restrict__ wh, double *__restrict__ wv, int ny, int nx)
{
    const long n = (long)ny * nx;
    for (long gi = blockIdx.x * (long)blockDim.x + threadIdx.x; gi < n; gi += (long)gridDim.x * blockDim.x) {
        const int i = gi / nx, j = gi % nx;
        wh[gi] = (j < nx - 1) ? (wh_in ? wh_in[gi] : 1.0) : 0.0;
        wv[gi] = (i < ny - 1) ? (wv_in ? wv_in[gi] : 1.0) : 0.0;
    }
}

__global__ void k_fill(double *p, double v, long n)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

static int grid_for(long n)
{
    long g = (n + NT - 1) / NT;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_weights(const double *x, double beta, double *wh, double *wv, int ny, int nx, hipStream_t s)
{
    hipLaunchKernelGGL(k_weights, dim3(grid_for((long)ny * nx)), dim3(NT), 0, s, x, beta, wh, wv, ny, nx);
    return hipGetLastError();
}

hipError_t launch_copy_weights(const double *wh_in, const double *wv_in, double *wh, double *wv, int ny,
                               int nx, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_weights, dim3(grid_for((long)ny * nx)), dim3(NT), 0, s, wh_in, wv_in, wh, wv,
                       ny, nx);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, double v, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(NT), 0, s, p, v, n);
    return hipGetLastError();
}

// ------------------------------------------- edge weights of Sec. 2.1 --
// With D_{k-1} = W_{k-1}^{1/2} per difference and q = D_{k-1} L x, the rule is
// w = 1 - (|q| / max|q|)^p and D_k = diag(w) D_{k-1}, so W_k = w^2 W_{k-1}.
// Stage 1 writes one maximum of |q| per workgroup; stage 2 has every
// workgroup fold those maxima itself and then rescales its weights in place.
constexpr int EDGE_BLOCKS = 256;   // stage-1 workgroups (grid-stride)

__device__ inline double block_max(double v, double *sm)
{
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = sm[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(NT) void k_edge_max(const double *__restrict__ x, const double *__restrict__ wh,
                                                 const double *__restrict__ wv, int ny, int nx,
                                                 double *__restrict__ part)
{
    __shared__ double sm[NT];
    const long n = (long)ny * nx;
    double m = 0.0;
    for (long gi = blockIdx.x * (long)NT + threadIdx.x; gi < n; gi += (long)gridDim.x * NT) {
        const int i = gi / nx, j = gi % nx;
        const double xc = x[gi];
        if (j < nx - 1) m = fmax(m, sqrt(wh[gi]) * fabs(x[gi + 1] - xc));
        if (i < ny - 1) m = fmax(m, sqrt(wv[gi]) * fabs(x[gi + nx] - xc));
    }
    m = block_max(m, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__device__ inline double edge_factor(double q, double qmax, double p)
{
    // q = qmax gives 0; a flat image (qmax = 0) leaves the weights unchanged
    if (!(qmax > 0.0)) return 1.0;
    const double w = 1.0 - pow(q / qmax, p);
    return w * w;
}

__global__ __launch_bounds__(NT) void k_edge_rule(const double *__restrict__ x, double *__restrict__ wh,
                                                  double *__restrict__ wv, int ny, int nx,
                                                  const double *__restrict__ part, int npart, double p)
{
    __shared__ double sm[NT];
    double m = 0.0;
    for (int k = threadIdx.x; k < npart; k += NT) m = fmax(m, part[k]);
    const double qmax = block_max(m, sm);
    const long n = (long)ny * nx;
    for (long gi = blockIdx.x * (long)NT + threadIdx.x; gi < n; gi += (long)gridDim.x * NT) {
        const int i = gi / nx, j = gi % nx;
        const double xc = x[gi];
        if (j < nx - 1) {
            const double W = wh[gi];
            wh[gi] = edge_factor(sqrt(W) * fabs(x[gi + 1] - xc), qmax, p) * W;
        } else {
            wh[gi] = 0.0;
        }
        if (i < ny - 1) {
            const double W = wv[gi];
            wv[gi] = edge_factor(sqrt(W) * fabs(x[gi + nx] - xc), qmax, p) * W;
        } else {
            wv[gi] = 0.0;
        }
    }
}

int edge_rule_parts() { return EDGE_BLOCKS; }

hipError_t launch_edge_rule(const double *x, double *wh, double *wv, int ny, int nx, double p, double *part,
                            hipStream_t s)
{
    const long n = (long)ny * nx;
    const int g1 = std::min(EDGE_BLOCKS, grid_for(n));
    hipLaunchKernelGGL(k_edge_max, dim3(g1), dim3(NT), 0, s, x, wh, wv, ny, nx, part);
    hipLaunchKernelGGL(k_edge_rule, dim3(grid_for(n)), dim3(NT), 0, s, x, wh, wv, ny, nx, part, g1, p);
    return hipGetLastError();
}

// ------------------------------------------ correction right-hand side --
// out = gamma (E_k - E_{k-1}) x with E = D^T W D: per pixel, the sum over its
// incident differences of gamma (w_k - w_{k-1}) (x_p - x_other).
__global__ __launch_bounds__(NT) void k_weight_delta(const double *__restrict__ x, const double *__restrict__ wh,
                                                     const double *__restrict__ wv, const double *__restrict__ wh0,
                                                     const double *__restrict__ wv0, double gamma, int ny, int nx,
                                                     double *__restrict__ out)
{
    const long n = (long)ny * nx;
    for (long gi = blockIdx.x * (long)NT + threadIdx.x; gi < n; gi += (long)gridDim.x * NT) {
        const int i = gi / nx, j = gi % nx;
        const double xc = x[gi];
        double acc = 0.0;
        if (j < nx - 1) acc += (wh[gi] - wh0[gi]) * (xc - x[gi + 1]);
        if (j > 0) acc += (wh[gi - 1] - wh0[gi - 1]) * (xc - x[gi - 1]);
        if (i < ny - 1) acc += (wv[gi] - wv0[gi]) * (xc - x[gi + nx]);
        if (i > 0) acc += (wv[gi - nx] - wv0[gi - nx]) * (xc - x[gi - nx]);
        out[gi] = gamma * acc;
    }
}

hipError_t launch_weight_delta(const double *x, const double *wh, const double *wv, const double *wh0,
                               const double *wv0, double gamma, int ny, int nx, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_weight_delta, dim3(grid_for((long)ny * nx)), dim3(NT), 0, s, x, wh, wv, wh0, wv0, gamma, ny,
                       nx, out);
    return hipGetLastError();
}

// ------------------------------------------------ L-curve coordinates --
// For system y (blockIdx.y): per-workgroup partial sums of (K x - d)^2 and of
// the weighted squared differences sum_e W_e (L x)_e^2 = x^T E x.  K x is the
// direct zero-boundary convolution (setup-grade, straight from global memory).
__global__ __launch_bounds__(NT) void k_lcurve(const InstDev *__restrict__ insts, int ii,
                                               const double *__restrict__ X, long ld_x,
                                               const double *__restrict__ d, double *__restrict__ part)
{
    __shared__ double sr[NT], se[NT];
    const InstDev I = insts[ii];
    const double *__restrict__ x = X + blockIdx.y * ld_x;
    const long n = (long)I.ny * I.nx;
    const int cy = I.sy / 2, cx = I.sx / 2;
    double ar = 0.0, ae = 0.0;
    for (long gi = blockIdx.x * (long)NT + threadIdx.x; gi < n; gi += (long)gridDim.x * NT) {
        const int i = gi / I.nx, j = gi % I.nx;
        double kx = 0.0;
        for (int a = 0; a < I.sy; ++a) {
            const int yi = i + cy - a;
            if (yi < 0 || yi >= I.ny) continue;
            for (int c = 0; c < I.sx; ++c) {
                const int xj = j + cx - c;
                if (xj < 0 || xj >= I.nx) continue;
                const double h = I.sep == 1 ? I.fy[a] * I.fx[c] : I.psf[a * I.sx + c];
                kx = fma(h, x[(long)yi * I.nx + xj], kx);
            }
        }
        const double r = kx - d[gi];
        ar = fma(r, r, ar);
        const double xc = x[gi];
        if (j < I.nx - 1) { const double t = x[gi + 1] - xc; ae = fma(I.wh[gi] * t, t, ae); }
        if (i < I.ny - 1) { const double t = x[gi + I.nx] - xc; ae = fma(I.wv[gi] * t, t, ae); }
    }
    sr[threadIdx.x] = ar;
    se[threadIdx.x] = ae;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *o = part + 2 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
        o[0] = sr[0];
        o[1] = se[0];
    }
}

int lcurve_parts(long n) { return std::min(256, grid_for(n)); }

hipError_t launch_lcurve(const InstDev *inst_dev, int ii, long n, int m, const double *X, long ld_x,
                         const double *d, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_lcurve, dim3(lcurve_parts(n), m), dim3(NT), 0, s, inst_dev, ii, X, ld_x, d, part);
    return hipGetLastError();
}

// ------------------------------------------------ tall-skinny products --
// C = X^T Y for n x a and n x c panels.  Grid: (row chunks, 64 x 64 output
// blocks, jobs).  Each workgroup stages 32-row slabs of up to 64 X columns and
// 64 Y columns in LDS and each thread accumulates a 4 x 4 register block of
// the output (rows ti + 16u, columns tj + 16v), so every panel element is read
// once per output block.  The next slab's loads are issued into registers
// before the current slab's FMAs.  Chunk partials go to scratch in 16 x 16
// output tiles and k_gram_reduce sums them in order; every output sums its
// rows in order, so the result does not depend on the launch shape.
constexpr int GT = 16;       // output tile edge of the partial-sum layout
constexpr int GB = 64;       // output block edge per workgroup
constexpr int GR = 32;       // rows per slab
constexpr int GLD = GR * GB / NT;   // slab elements per thread and panel

// rows per chunk, a whole number of slabs: about 256 chunks (256..4096 rows)
// for the blocked products, about 64 (512..4096 rows) for the small ones
// (c <= 8), whose per-workgroup reduction is the larger fixed cost
__host__ __device__ inline long gram_chunk_rows(long n, int c)
{
    const long per = c <= 8 ? 64 : 256, lo = c <= 8 ? 512 : 256;
    const long r = (n / per + 63) / 64 * 64;
    return r < lo ? lo : (r > 4096 ? 4096 : r);
}

__host__ __device__ inline long gram_chunks(long n, int c)
{
    return (n + gram_chunk_rows(n, c) - 1) / gram_chunk_rows(n, c);
}

__global__ __launch_bounds__(NT) void k_gram(const Jobs<GramJob> jobs, double *__restrict__ scratch)
{
    __shared__ double xs[GR][GB + 1];
    __shared__ double ys[GR][GB + 1];
    const GramJob J = jobs[blockIdx.z];
    if (J.c <= 8) return;   // done by k_gram_small
    const int blocks_c = (J.c + GB - 1) / GB;
    const int blocks_a = (J.a + GB - 1) / GB;
    const int ob = blockIdx.y;
    if (ob >= blocks_a * blocks_c) return;
    const long nchunk = gram_chunks(J.n, J.c);
    if ((long)blockIdx.x >= nchunk) return;
    const int ia0 = (ob / blocks_c) * GB, jc0 = (ob % blocks_c) * GB;
    const int na = J.a - ia0 < GB ? J.a - ia0 : GB;
    const int nc = J.c - jc0 < GB ? J.c - jc0 : GB;
    const long gch = gram_chunk_rows(J.n, J.c);
    const long r0 = (long)blockIdx.x * gch;
    const long r1 = r0 + gch < J.n ? r0 + gch : J.n;
    const int ti = threadIdx.x % 16, tj = threadIdx.x / 16;
    double vx[GLD], vy[GLD];
    auto load = [&](long rb) {
#pragma unroll
        for (int u = 0; u < GLD; ++u) {
            const int k = threadIdx.x + u * NT;
            const int rr = k % GR, cc = k / GR;
            const long row = rb + rr;
            vx[u] = (row < r1 && cc < na) ? gp(J.X)[row + (long)(ia0 + cc) * J.ldx] : 0.0;
            vy[u] = (row < r1 && cc < nc) ? gp(J.Y)[row + (long)(jc0 + cc) * J.ldy] : 0.0;
        }
    };
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    load(r0);
    for (long rb = r0; rb < r1; rb += GR) {
#pragma unroll
        for (int u = 0; u < GLD; ++u) {
            const int k = threadIdx.x + u * NT;
            xs[k % GR][k / GR] = vx[u];
            ys[k % GR][k / GR] = vy[u];
        }
        __syncthreads();
        if (rb + GR < r1) load(rb + GR);   // in flight during this slab's FMAs
#pragma unroll 4
        for (int rr = 0; rr < GR; ++rr) {
            double xv[4], yv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = xs[rr][ti + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v) yv[v] = ys[rr][tj + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(xv[u], yv[v], acc[u][v]);
        }
        __syncthreads();
    }
    const int tiles_c = (J.c + GT - 1) / GT;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = ia0 + ti + 16 * u, j = jc0 + tj + 16 * v;
            if (i < J.a && j < J.c) {
                const int ot = (i / GT) * tiles_c + j / GT;
                scratch[J.sc_off + ((long)ot * nchunk + blockIdx.x) * (GT * GT) + (i % GT) * GT + (j % GT)] =
                    acc[u][v];
            }
        }
}

__global__ void k_gram_reduce(const Jobs<GramJob> jobs, const double *__restrict__ scratch)
{
    const GramJob J = jobs[blockIdx.y];
    const int tiles_c = (J.c + GT - 1) / GT;
    const long nchunk = gram_chunks(J.n, J.c);
    const int total = J.a * J.c;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
        const int i = k / J.c, j = k % J.c;
        const int ot = (i / GT) * tiles_c + (j / GT);
        const double *src = scratch + J.sc_off + (long)ot * nchunk * (GT * GT) + (i % GT) * GT + (j % GT);
        double s = 0.0;
#pragma unroll 8
        for (long ch = 0; ch < nchunk; ++ch) s += src[ch * (GT * GT)];
        J.C[k] = s;
    }
}

// Small products (a * c <= GSMALL, e.g. norms, W^T r, W^T Z): every thread runs
// over its rows once with all a*c accumulators in registers, then the
// workgroup reduces them in a fixed order.  Chunk partials use the same
// scratch layout as k_gram (output tile 0), so k_gram_reduce finishes both.
constexpr int GSMALL = 64;
constexpr int GSMALL_A = 8;
__global__ __launch_bounds__(NT) void k_gram_small(const Jobs<GramJob> jobs, double *__restrict__ scratch)
{
    __shared__ double red[NT / 64][GSMALL];
    const GramJob J = jobs[blockIdx.z];
    if (J.c > GSMALL_A) return;
    // rows ia0 .. ia0+7 of the output (a of any size is split over blockIdx.y)
    const int ia0 = blockIdx.y * GSMALL_A;
    if (ia0 >= J.a) return;
    const int na = J.a - ia0 < GSMALL_A ? J.a - ia0 : GSMALL_A;
    const long nchunk = gram_chunks(J.n, J.c);
    if ((long)blockIdx.x >= nchunk) return;
    const long gch = gram_chunk_rows(J.n, J.c);
    const long r0 = (long)blockIdx.x * gch;
    const long r1 = r0 + gch < J.n ? r0 + gch : J.n;
    double acc[GSMALL_A][GSMALL_A];
#pragma unroll
    for (int i = 0; i < GSMALL_A; ++i)
#pragma unroll
        for (int j = 0; j < GSMALL_A; ++j) acc[i][j] = 0.0;
    for (long r = r0 + threadIdx.x; r < r1; r += NT) {
        double xv[GSMALL_A], yv[GSMALL_A];
#pragma unroll
        for (int i = 0; i < GSMALL_A; ++i) xv[i] = i < na ? gp(J.X)[r + (long)(ia0 + i) * J.ldx] : 0.0;
#pragma unroll
        for (int j = 0; j < GSMALL_A; ++j) yv[j] = j < J.c ? gp(J.Y)[r + (long)j * J.ldy] : 0.0;
#pragma unroll
        for (int i = 0; i < GSMALL_A; ++i)
#pragma unroll
            for (int j = 0; j < GSMALL_A; ++j) acc[i][j] = fma(xv[i], yv[j], acc[i][j]);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < GSMALL_A; ++i)
#pragma unroll
        for (int j = 0; j < GSMALL_A; ++j)
            if (i < na && j < J.c) {
                const double v = wave_sum(acc[i][j]);
                if (lane == 0) red[wid][i * GSMALL_A + j] = v;
            }
    __syncthreads();
    if (threadIdx.x < GSMALL_A * GSMALL_A) {
        const int i = threadIdx.x / GSMALL_A, j = threadIdx.x % GSMALL_A;
        if (i < na && j < J.c) {
            double v = 0.0;
            for (int w = 0; w < NT / 64; ++w) v += red[w][i * GSMALL_A + j];
            // k_gram's layout: output tile (gi / GT, 0), entry (gi % GT, j), chunk blockIdx.x
            const int gi = ia0 + i;
            scratch[J.sc_off + ((long)(gi / GT) * nchunk + blockIdx.x) * (GT * GT) + (gi % GT) * GT + j] = v;
        }
    }
}

size_t gram_scratch_doubles(const GramJob *jh, int njobs)
{
    size_t t = 0;
    for (int i = 0; i < njobs; ++i) {
        const long nchunk = gram_chunks(jh[i].n, jh[i].c);
        const long ntiles = (long)((jh[i].a + GT - 1) / GT) * ((jh[i].c + GT - 1) / GT);
        t += (size_t)(nchunk * ntiles * GT * GT);
    }
    return t;
}

hipError_t launch_gram(const GramJob *jobs_dev, const GramJob *jh, int njobs, double *scratch,
                       size_t scratch_doubles, hipStream_t s)
{
    if (!jobs_dev && njobs > KJ) return hipErrorInvalidValue;
    const Jobs<GramJob> ja = make_jobs(jobs_dev, jh, njobs);
    long maxchunk = 1;
    bool any_big = false, any_small = false;
    for (int i = 0; i < njobs; ++i) {
        const long nchunk = gram_chunks(jh[i].n, jh[i].c);
        const long ntiles = (long)((jh[i].a + GT - 1) / GT) * ((jh[i].c + GT - 1) / GT);
        if (nchunk > maxchunk) maxchunk = nchunk;
        if (jh[i].sc_off + (size_t)(nchunk * ntiles * GT * GT) > scratch_doubles) return hipErrorInvalidValue;
        const bool small = jh[i].c <= GSMALL_A;
        any_small |= small;
        any_big |= !small;
    }
    hipError_t e;
    if (any_small) {
        long maxa8 = 1;
        for (int i = 0; i < njobs; ++i) maxa8 = std::max<long>(maxa8, (jh[i].a + GSMALL_A - 1) / GSMALL_A);
        hipLaunchKernelGGL(k_gram_small, dim3(maxchunk, maxa8, njobs), dim3(NT), 0, s, ja, scratch);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (any_big) {
        long maxblocks = 1;
        for (int i = 0; i < njobs; ++i)
            maxblocks = std::max<long>(maxblocks, (long)((jh[i].a + GB - 1) / GB) * ((jh[i].c + GB - 1) / GB));
        hipLaunchKernelGGL(k_gram, dim3(maxchunk, maxblocks, njobs), dim3(NT), 0, s, ja, scratch);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    long outs = 1;
    for (int i = 0; i < njobs; ++i) outs = std::max<long>(outs, (long)jh[i].a * jh[i].c);
    const int gr = (int)std::min<long>(64, (outs + NT - 1) / NT);
    hipLaunchKernelGGL(k_gram_reduce, dim3(gr, njobs), dim3(NT), 0, s, ja, scratch);
    return hipGetLastError();
}

// Y = beta Y + X Q (or Y = Y0 + X Q) over n rows; Q is a x c, column-major.
// Grid: (row blocks, jobs, 16-column chunks of Y).  Each thread owns one row
// and 16 outputs.  The workgroup stages its a x 16 block of Q in LDS (in
// passes of CQ rows when a is larger), so the coefficients are broadcast LDS
// reads; the loads of 8 X columns are issued together before their FMAs.
// The sum over k runs in order, the same for every launch shape.
constexpr int CJ = 16;    // output columns per register chunk
constexpr int CK = 8;     // X columns loaded together
constexpr int CQ = 256;   // Q rows staged in LDS per pass
__global__ __launch_bounds__(NT) void k_combo(const ComboArgs ca)
{
    __shared__ double qs[CQ * CJ];
    const ComboJob J = ca.jobs[blockIdx.y];
    const int a = J.a, c = J.c;
    const int j0 = blockIdx.z * CJ;
    if (j0 >= c) return;
    const int cu = c - j0 < CJ ? c - j0 : CJ;   // live columns of this chunk
    bool staged = false;
    for (long rb = blockIdx.x * (long)NT; rb < J.n; rb += (long)gridDim.x * NT) {
        const long r = rb + threadIdx.x;
        const bool live = r < J.n;
        double s[CJ];
#pragma unroll
        for (int u = 0; u < CJ; ++u) {
            double v = 0.0;
            if (live && u < cu) {
                if (J.Y0) v = gp(J.Y0)[r + (long)(j0 + u) * J.ldy0];
                else if (J.beta != 0.0) v = J.beta * gp(J.Y)[r + (long)(j0 + u) * J.ldy];
            }
            s[u] = v;
        }
        for (int kb = 0; kb < a; kb += CQ) {
            const int ka = a - kb < CQ ? a - kb : CQ;
            if (!(staged && a <= CQ)) {   // one pass covers Q: stage it once
                __syncthreads();
                for (int e = threadIdx.x; e < ka * CJ; e += NT) {
                    const int k = e / CJ, u = e % CJ;
                    const long qi = (kb + k) + (long)(j0 + u) * J.ldq;
                    qs[e] = u >= cu ? 0.0 : J.qoff >= 0 ? ca.q[J.qoff + qi] : gp(J.Q)[qi];
                }
                __syncthreads();
                staged = true;
            }
            if (live) {
                for (int k0 = 0; k0 < ka; k0 += CK) {
                    double xv[CK];
#pragma unroll
                    for (int t = 0; t < CK; ++t)
                        xv[t] = k0 + t < ka ? gp(J.X)[r + (long)(kb + k0 + t) * J.ldx] : 0.0;
#pragma unroll
                    for (int t = 0; t < CK; ++t) {
                        if (k0 + t < ka) {
                            const double *qk = qs + (k0 + t) * CJ;
#pragma unroll
                            for (int u = 0; u < CJ; ++u) s[u] = fma(xv[t], qk[u], s[u]);
                        }
                    }
                }
            }
        }
        if (live) {
#pragma unroll
            for (int u = 0; u < CJ; ++u)
                if (u < cu) gp(J.Y)[r + (long)(j0 + u) * J.ldy] = s[u];
        }
    }
}

hipError_t launch_combo(const ComboJob *jobs_dev, const ComboJob *jh, int njobs, hipStream_t s,
                        const double *const *qs)
{
    if (!jobs_dev && njobs > KJ) return hipErrorInvalidValue;
    ComboArgs ca;
    ca.jobs = make_jobs(jobs_dev, jh, njobs);
    if (!jobs_dev && qs) {
        int o = 0;
        for (int i = 0; i < njobs; ++i) {
            const int nq = jh[i].a * jh[i].c;   // column-major with ldq = a
            if (o + nq > KQ || (nq > 0 && jh[i].ldq != jh[i].a)) return hipErrorInvalidValue;
            if (nq == 0) continue;
            for (int k = 0; k < nq; ++k) ca.q[o + k] = qs[i][k];
            ca.jobs.inl[i].qoff = o;
            o += nq;
        }
    }
    long nmax = 1;
    int cch = 1;
    for (int i = 0; i < njobs; ++i) {
        if (jh[i].n > nmax) nmax = jh[i].n;
        cch = std::max(cch, (jh[i].c + CJ - 1) / CJ);
    }
    int gx = grid_for(nmax);
    if (gx > 2048) gx = 2048;
    hipLaunchKernelGGL(k_combo, dim3(gx, njobs, cch), dim3(NT), 0, s, ca);
    return hipGetLastError();
}

// ------------------------------------------------------ adjoint gradient --
// For m shifts (columns of X and Lam, stride ld):
//   dw_h = -sum_l gamma_l (D_h lam_l)(D_h x_l),  dw_v likewise,
//   dg_partial[chunk][l] = -sum_{pixels in chunk} [wh (D_h lam)(D_h x) + wv (D_v lam)(D_v x)].
__global__ __launch_bounds__(NT) void k_grad(const double *__restrict__ X, const double *__restrict__ L, long ld,
                                             const double *__restrict__ gam, int m,
                                             const double *__restrict__ wh, const double *__restrict__ wv,
                                             int ny, int nx, double *__restrict__ dwh, double *__restrict__ dwv,
                                             double *__restrict__ db, double *__restrict__ dgp)
{
    __shared__ double red[NT / 64];
    const long n = (long)ny * nx;
    const long per = (n + gridDim.x - 1) / gridDim.x;
    const long lo = blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    for (int l = 0; l < m; ++l) {
        const double *x = X + l * ld, *la = L + l * ld;
        double acc = 0.0;
        for (long gi = lo + threadIdx.x; gi < hi; gi += NT) {
            const int i = gi / nx, j = gi % nx;
            double ph = 0.0, pv = 0.0;
            if (j < nx - 1) ph = (la[gi + 1] - la[gi]) * (x[gi + 1] - x[gi]);
            if (i < ny - 1) pv = (la[gi + nx] - la[gi]) * (x[gi + nx] - x[gi]);
            acc += wh[gi] * ph + wv[gi] * pv;
        }
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) dgp[(long)blockIdx.x * m + l] = -(red[0] + red[1] + red[2] + red[3]);
        __syncthreads();
    }
    for (long gi = lo + threadIdx.x; gi < hi; gi += NT) {
        const int i = gi / nx, j = gi % nx;
        double sh = 0.0, sv = 0.0, sb = 0.0;
        for (int l = 0; l < m; ++l) {
            const double *x = X + l * ld, *la = L + l * ld;
            if (j < nx - 1) sh += gam[l] * (la[gi + 1] - la[gi]) * (x[gi + 1] - x[gi]);
            if (i < ny - 1) sv += gam[l] * (la[gi + nx] - la[gi]) * (x[gi + nx] - x[gi]);
            sb += la[gi];
        }
        dwh[gi] = -sh;
        dwv[gi] = -sv;
        if (db) db[gi] = sb;
    }
}

hipError_t launch_grad(const double *X, const double *Lam, long ld, const double *gammas_dev, int m,
                       const double *wh, const double *wv, int ny, int nx, double *dw_h, double *dw_v,
                       double *db, double *dg_partial, int nchunks, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad, dim3(nchunks), dim3(NT), 0, s, X, Lam, ld, gammas_dev, m, wh, wv, ny, nx, dw_h,
                       dw_v, db, dg_partial);
    return hipGetLastError();
}

}  // namespace rsr

namespace rsr {

// ------------------------------------------- graph-capturable shift-set solve --
// Plain CG of a shift set on one instance with every step on the device: the
// descriptors of the persistent CG launch are written by a kernel from the
// launch arguments, the tolerances come from norms of b computed on the device,
// and the last step x += alpha p, the true residual and the statistics are
// kernels too, so the whole sequence records into a HIP graph and replays.

// Fixed-order sum of one value per thread over the workgroup (result in thread 0).
__device__ double block_sum_fixed(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// stage 0: ZERO start (x = 0, r = b) and the partial sums of b^2;
// stage 1: r = b - r (GIVEN start, after r = B x);
// stage 2: x += alpha p with the step the CG kernel left (out_alpha);
// stage 3: partial sums of (b - rt)^2, rt = B x.
__global__ __launch_bounds__(NT) void k_async_elem(AsyncArgs a, int stage)
{
    __shared__ double red[NT / 64];
    const int i = blockIdx.y;
    const double *b = a.b + (size_t)i * a.ld_b;
    double *x = a.X + (size_t)i * a.ld_x;
    double *v = a.vec + (size_t)i * a.vstride;
    double *r = v, *pa = v + 8 * a.n, *rt = v + 7 * a.n;
    const double alpha = stage == 2 ? a.out_alpha[i] : 0.0;
    double acc = 0.0;
    for (long k = blockIdx.x * (long)NT + threadIdx.x; k < a.n; k += (long)gridDim.x * NT) {
        const double bk = b[k];
        if (stage == 0) {
            if (a.init == 0) {
                x[k] = 0.0;
                r[k] = bk;
            }
            acc = fma(bk, bk, acc);
        } else if (stage == 1) {
            r[k] = bk - r[k];
        } else if (stage == 2) {
            x[k] = fma(alpha, pa[k], x[k]);
        } else {
            const double e = bk - rt[k];
            acc = fma(e, e, acc);
        }
    }
    if (stage == 0 || stage == 3) {
        const double s = block_sum_fixed(acc, red);
        if (threadIdx.x == 0) a.part[(size_t)i * gridDim.x + blockIdx.x] = s;
    }
}

// One workgroup: ||b_i||^2 from the partials, the CG descriptors and the
// operator jobs of every system, and cleared barrier and output blocks.
__global__ __launch_bounds__(NT) void k_async_setup(AsyncArgs a)
{
    for (int i = threadIdx.x; i < a.m; i += NT) {
        double s = 0.0;
        for (int k = 0; k < a.nb; ++k) s += a.part[(size_t)i * a.nb + k];
        a.bn2[i] = s;
        double *v = a.vec + (size_t)i * a.vstride;
        SysDev d;
        memset(&d, 0, sizeof(d));
        d.inst = a.inst;
        d.q = 0;
        d.ntiles = a.ntiles;
        d.tile_base = i * a.ntiles;
        d.gamma = a.gam[i];
        d.tolabs = a.tol * sqrt(s);
        d.x = a.X + (size_t)i * a.ld_x;
        d.rb[0] = v;
        d.rb[1] = v + a.n;
        d.wb[0] = v + 2 * a.n;
        d.wb[1] = v + 3 * a.n;
        d.pb[0] = v + 4 * a.n;
        d.pb[1] = v + 5 * a.n;
        d.pa = v + 8 * a.n;
        d.cbuf = a.cbuf + (size_t)i * 2 * QMAX;
        d.ldw = a.n;
        a.sys[i] = d;
        // B x into r (GIVEN start) and, after the solve, B x into rt
        a.jobs[i] = ApplyJob{a.inst, 0, 1.0, a.gam[i], d.x, a.init == 0 ? v + 7 * a.n : v};
        a.jobs[a.m + i] = ApplyJob{a.inst, 0, 1.0, a.gam[i], d.x, v + 7 * a.n};
    }
    for (int k = threadIdx.x; k < a.clear_n; k += NT) a.clear[k] = 0.0;
}

// One workgroup: stats[i] = {iterations, kernel status, true relative
// residual, applications of B}.
__global__ __launch_bounds__(NT) void k_async_stats(AsyncArgs a, double *stats)
{
    for (int i = threadIdx.x; i < a.m; i += NT) {
        double s = 0.0;
        for (int k = 0; k < a.nb; ++k) s += a.part[(size_t)i * a.nb + k];
        const double bn2 = a.bn2[i];
        stats[4 * i + 0] = (double)a.out_iters[i];
        stats[4 * i + 1] = (double)a.out_status[i];
        stats[4 * i + 2] = bn2 > 0.0 ? sqrt(s / bn2) : 0.0;
        stats[4 * i + 3] = (double)(a.out_iters[i] + 1 + (a.init == 0 ? 0 : 1));
    }
}

hipError_t launch_async_elem(const AsyncArgs &a, int stage, hipStream_t s)
{
    hipLaunchKernelGGL(k_async_elem, dim3(a.nb, a.m), dim3(NT), 0, s, a, stage);
    return hipGetLastError();
}

hipError_t launch_async_setup(const AsyncArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_async_setup, dim3(1), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_async_stats(const AsyncArgs &a, double *stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_async_stats, dim3(1), dim3(NT), 0, s, a, stats);
    return hipGetLastError();
}

}  // namespace rsr
