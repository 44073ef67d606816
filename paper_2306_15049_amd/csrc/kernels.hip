// Device kernels of the recycled shifted solver (gfx950, FP64).
//
// The systems are (A + gamma E) x = b with A = K^T K (K: zero-boundary 2-D
// convolution by the PSF) and E = D^T W D (D: forward differences, W diagonal
// weights), Section 2.1 eq. blkeqn.  The unit of cost is one application of
// the shifted operator (Section 6), so the stencil that applies it is the
// centre of this file:
//
//   * tile_operator: one workgroup computes a TY x TX tile of
//     cA K^T K v + cE E v.  v is staged once into LDS with a 2r halo; K^T K is
//     applied as four 1-D passes (x conv, x corr, y conv, y corr) for a
//     rank-1 PSF, or as a direct 2-D conv + corr otherwise, with the
//     intermediate masked to the image after each forward pass (zero
//     boundary).  Each thread produces RB consecutive outputs per pass from a
//     register window, so an output costs (RB+S-1)/RB LDS reads instead of S.
//   * cg_persistent: all systems of a shift set advance together in one
//     cooperative launch.  Each iteration is two grid-wide phases:
//       phase 1: p = r + beta p - W mu (recomputed on the halo, ping-pong
//                buffers), w = B p, partial p.w;
//       phase 2: x += alpha p, r -= alpha w, partial r.r and Z^T r.
//     Per-system scalars are reduced from per-chunk partials in a fixed order
//     by every workgroup, so all workgroups take identical decisions and the
//     results are deterministic.  Converged systems drop out and the tile
//     list of the remaining ones is re-split evenly over the grid.
#include "internal.hpp"

#include <hip/hip_runtime.h>

namespace rsr {

// ---------------------------------------------------------------- helpers --
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ unsigned long long realtime()
{
    return __builtin_amdgcn_s_memrealtime();
}

// Tile geometry shared by host (LDS sizing) and device.
struct Geo {
    int ry, rx;        // PSF radii
    int hy, hx;        // halo of the staged input (2r, at least 1 for E)
    int oy, ox;        // hy - 2ry, hx - 2rx (0 or 1)
    int H0, W0, P0;    // staged input
    int W1, P1;        // after the x conv pass
    int P2;            // width-tx intermediates
    int H3;            // rows after the y conv pass
    int PE;            // pitch of the output accumulator
    int off1, offE, total;
};

__host__ __device__ inline Geo make_geo(int ty, int tx, int sy, int sx)
{
    Geo g;
    g.ry = sy / 2;
    g.rx = sx / 2;
    g.hy = 2 * g.ry > 1 ? 2 * g.ry : 1;
    g.hx = 2 * g.rx > 1 ? 2 * g.rx : 1;
    g.oy = g.hy - 2 * g.ry;
    g.ox = g.hx - 2 * g.rx;
    g.H0 = ty + 2 * g.hy;
    g.W0 = tx + 2 * g.hx;
    g.P0 = g.W0 | 1;
    g.W1 = tx + 2 * g.rx;
    g.P1 = g.W1 | 1;
    g.P2 = tx | 1;
    g.H3 = ty + 2 * g.ry;
    g.PE = tx | 1;
    int sz0 = g.H0 * g.P0;
    int sz1a = g.H0 * g.P1, sz1b = g.H3 * g.P2;
    int sz1 = sz1a > sz1b ? sz1a : sz1b;
    g.off1 = (sz0 + 1) & ~1;
    g.offE = (g.off1 + sz1 + 1) & ~1;
    g.total = g.offE + ty * g.PE;
    return g;
}

int tile_lds_doubles(int ty, int tx, int sy, int sx)
{
    Geo g = make_geo(ty, tx, sy, sx);
    int t = g.total;
    return t < 2048 ? 2048 : t;   // the persistent kernel reuses it as reduction scratch
}

// One 1-D stencil pass over `nlines` lines of `nout` outputs:
//   out[l][e] (=|+=) mask(e) * sum_c g[c] in[l][e + c],  g = f (corr) or reversed f (conv).
// Element e of line l lives at base + l*step_l + e*step_e.  Threads take
// (line, strip) items with consecutive threads on consecutive lines.
template <int S>
__device__ __forceinline__ void pass1d(const double *__restrict__ in, int in_e, int in_l, int nin,
                                       double *__restrict__ out, int out_e, int out_l, int nlines,
                                       int nout, const double *__restrict__ f, bool flip, bool acc,
                                       int lo, int hi)
{
    double g[S];
#pragma unroll
    for (int c = 0; c < S; ++c) g[c] = f[flip ? S - 1 - c : c];
    const int nstrip = (nout + RB - 1) / RB;
    const int total = nlines * nstrip;
    for (int it = threadIdx.x; it < total; it += NT) {
        const int l = it % nlines;
        const int e0 = (it / nlines) * RB;
        const double *src = in + l * in_l + e0 * in_e;
        const int kmax = nin - 1 - e0;   // last valid input element of this strip
        double win[RB + S - 1];
#pragma unroll
        for (int k = 0; k < RB + S - 1; ++k) win[k] = src[(k < kmax ? k : kmax) * in_e];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            double a = 0.0;
#pragma unroll
            for (int c = 0; c < S; ++c) a = fma(g[c], win[k + c], a);
            const int e = e0 + k;
            if (e < nout) {
                const double v = (e >= lo && e < hi) ? a : 0.0;
                double *d = out + l * out_l + e * out_e;
                if (acc) *d += v;
                else *d = v;
            }
        }
    }
}

// Runtime dispatch on the (odd) tap count.
__device__ void pass1d_any(int S, const double *in, int in_e, int in_l, int nin, double *out,
                           int out_e, int out_l, int nlines, int nout, const double *f, bool flip,
                           bool acc, int lo, int hi)
{
#define RSR_PASS(SS)                                                                          \
    case SS:                                                                                  \
        pass1d<SS>(in, in_e, in_l, nin, out, out_e, out_l, nlines, nout, f, flip, acc, lo, hi); \
        break;
    switch (S) {
        RSR_PASS(1) RSR_PASS(3) RSR_PASS(5) RSR_PASS(7) RSR_PASS(9) RSR_PASS(11) RSR_PASS(13)
        RSR_PASS(15) RSR_PASS(17) RSR_PASS(19) RSR_PASS(21) RSR_PASS(23) RSR_PASS(25)
        RSR_PASS(27) RSR_PASS(29) RSR_PASS(31)
    default: break;
    }
#undef RSR_PASS
}

// Direct 2-D pass: out[i][j] (=|+=) mask * sum_{a,c} g[a][c] in[i+a][j+c] with
// g = psf (corr) or the psf rotated by 180 degrees (conv).
__device__ void pass2d(const double *__restrict__ in, int pin, double *__restrict__ out, int pout,
                       int rows, int cols, const double *__restrict__ h, int sy, int sx, bool flip,
                       bool acc, int rlo, int rhi, int clo, int chi)
{
    const int nstrip = (cols + RB - 1) / RB;
    const int total = rows * nstrip;
    for (int it = threadIdx.x; it < total; it += NT) {
        const int i = it % rows;
        const int j0 = (it / rows) * RB;
        double a[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) a[k] = 0.0;
        const int jlast = cols + sx - 2;   // last valid input column of the row
        for (int ay = 0; ay < sy; ++ay) {
            const double *src = in + (i + ay) * pin;
            for (int cx = 0; cx < sx; ++cx) {
                const double gv = flip ? h[(sy - 1 - ay) * sx + (sx - 1 - cx)] : h[ay * sx + cx];
#pragma unroll
                for (int k = 0; k < RB; ++k) {
                    const int jj = j0 + k + cx;
                    a[k] = fma(gv, src[jj < jlast ? jj : jlast], a[k]);
                }
            }
        }
        const bool rin = (i >= rlo && i < rhi);
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int j = j0 + k;
            if (j < cols) {
                const double v = (rin && j >= clo && j < chi) ? a[k] : 0.0;
                double *d = out + i * pout + j;
                if (acc) *d += v;
                else *d = v;
            }
        }
    }
}

// cA * K^T K (buf0 -> ebuf, accumulated) for the tile whose top-left output is
// (y0, x0).  buf0 holds v on the (H0 x W0) staged window; it is overwritten.
__device__ void tile_A(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cA)
{
    double *buf0 = lds, *buf1 = lds + g.off1, *ebuf = lds + g.offE;
    const int ty = I.ty, tx = I.tx;
    if (I.sep) {
        // The A part is scaled once: fold cA into the last pass via a scaled copy of fy.
        // x conv: buf0 (cols from ox) -> buf1, mask to the image columns.
        pass1d_any(I.sx, buf0 + g.ox, 1, g.P0, g.W0 - g.ox, buf1, 1, g.P1, g.H0, g.W1, I.fx, true,
                   false, g.rx - x0, I.nx - x0 + g.rx);
        __syncthreads();
        // x corr: buf1 -> buf0 (pitch P2), tx outputs per row.
        pass1d_any(I.sx, buf1, 1, g.P1, g.W1, buf0, 1, g.P2, g.H0, tx, I.fx, false, false, 0, tx);
        __syncthreads();
        // y conv: buf0 rows from oy -> buf1 (H3 x tx, pitch P2), mask to the image rows.
        pass1d_any(I.sy, buf0 + g.oy * g.P2, g.P2, 1, g.H0 - g.oy, buf1, g.P2, 1, tx, g.H3, I.fy,
                   true, false, g.ry - y0, I.ny - y0 + g.ry);
        __syncthreads();
        if (cA != 1.0) {
            for (int k = threadIdx.x; k < g.H3 * g.P2; k += NT) buf1[k] *= cA;
            __syncthreads();
        }
        // y corr: buf1 -> ebuf (+=).
        pass1d_any(I.sy, buf1, g.P2, 1, g.H3, ebuf, g.PE, 1, tx, ty, I.fy, false, true, 0, ty);
    } else {
        // direct: K over (H3 x W1) with mask, then K^T into ebuf.
        pass2d(buf0 + g.oy * g.P0 + g.ox, g.P0, buf1, g.P1, g.H3, g.W1, I.psf, I.sy, I.sx, true,
               false, g.ry - y0, I.ny - y0 + g.ry, g.rx - x0, I.nx - x0 + g.rx);
        __syncthreads();
        if (cA != 1.0) {
            for (int k = threadIdx.x; k < g.H3 * g.P1; k += NT) buf1[k] *= cA;
            __syncthreads();
        }
        pass2d(buf1, g.P1, ebuf, g.PE, ty, tx, I.psf, I.sy, I.sx, false, true, 0, ty, 0, tx);
    }
    __syncthreads();
}

// ebuf = cE * E v on the tile (v staged in buf0).  Weight planes carry zeros
// where a difference does not exist, so only neighbours outside the image need
// a test.
__device__ void tile_E(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cE)
{
    const double *buf0 = lds;
    double *ebuf = lds + g.offE;
    const int ty = I.ty, tx = I.tx, nx = I.nx, ny = I.ny;
    for (int k = threadIdx.x; k < ty * tx; k += NT) {
        const int i = k / tx, j = k % tx;
        const int gy = y0 + i, gx = x0 + j;
        double e = 0.0;
        if (cE != 0.0 && gy < ny && gx < nx) {
            const long gi = (long)gy * nx + gx;
            const double *c = buf0 + (g.hy + i) * g.P0 + (g.hx + j);
            const double wc = I.wh[gi], wd = I.wv[gi];
            const double wl = gx > 0 ? I.wh[gi - 1] : 0.0;
            const double wu = gy > 0 ? I.wv[gi - nx] : 0.0;
            e = (wl + wc + wu + wd) * c[0] - wl * c[-1] - wc * c[1] - wu * c[-g.P0] - wd * c[g.P0];
            e *= cE;
        }
        ebuf[i * g.PE + j] = e;
    }
    __syncthreads();
}

// ---------------------------------------------------------- apply kernel --
// y = cA A v + cE E v for one tile per workgroup; blockIdx.y selects the job.
__global__ __launch_bounds__(NT) void k_apply(const InstDev *__restrict__ insts,
                                              const ApplyJob *__restrict__ jobs)
{
    extern __shared__ double lds[];
    const ApplyJob J = jobs[blockIdx.y];
    const InstDev I = insts[J.inst];
    const int ntile = I.nty * I.ntx;
    if ((int)blockIdx.x >= ntile) return;
    const int y0 = (blockIdx.x / I.ntx) * I.ty, x0 = (blockIdx.x % I.ntx) * I.tx;
    const Geo g = make_geo(I.ty, I.tx, I.sy, I.sx);
    for (int k = threadIdx.x; k < g.H0 * g.W0; k += NT) {
        const int li = k / g.W0, lj = k % g.W0;
        const int gy = y0 - g.hy + li, gx = x0 - g.hx + lj;
        double v = 0.0;
        if (gy >= 0 && gy < I.ny && gx >= 0 && gx < I.nx) v = J.v[(long)gy * I.nx + gx];
        lds[li * g.P0 + lj] = v;
    }
    __syncthreads();
    tile_E(I, g, lds, y0, x0, J.cE);
    if (J.cA != 0.0) tile_A(I, g, lds, y0, x0, J.cA);
    const double *ebuf = lds + g.offE;
    for (int k = threadIdx.x; k < I.ty * I.tx; k += NT) {
        const int i = k / I.tx, j = k % I.tx;
        const int gy = y0 + i, gx = x0 + j;
        if (gy < I.ny && gx < I.nx) J.y[(long)gy * I.nx + gx] = ebuf[i * g.PE + j];
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
                const double h = I.sep ? I.fy[a] * I.fx[c] : I.psf[a * I.sx + c];
                s = fma(h, J.v[(long)ii * I.nx + jj], s);
            }
        }
        J.y[gi] = s;
    }
}

hipError_t launch_apply(const InstDev *inst_dev, const InstDev &ih, const ApplyJob *jobs_dev, int njobs,
                        size_t lds, hipStream_t s)
{
    dim3 grid(ih.nty * ih.ntx, njobs);
    hipLaunchKernelGGL(k_apply, grid, dim3(NT), lds, s, inst_dev, jobs_dev);
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

// ------------------------------------------------ tall-skinny products --
// C = X^T Y for n x a and n x c panels.  Grid: (row chunks, output tiles of
// 16 x 16, jobs).  Each workgroup stages 64-row slabs of 16 X columns and 16 Y
// columns in LDS; each thread owns one output of the 16 x 16 tile and a
// quarter of the slab rows, then the four quarters are summed in a fixed
// order.  Chunk partials go to scratch and k_gram_reduce sums them in order.
constexpr int GT = 16;       // output tile edge
constexpr int GR = 64;       // rows per slab
constexpr int GCH = 4096;    // rows per chunk

__global__ __launch_bounds__(NT) void k_gram(const GramJob *__restrict__ jobs, double *__restrict__ scratch)
{
    __shared__ double xs[GR][GT + 1];
    __shared__ double ys[GR][GT + 1];
    const GramJob J = jobs[blockIdx.z];
    const int tiles_c = (J.c + GT - 1) / GT;
    const int tiles_a = (J.a + GT - 1) / GT;
    const int ot = blockIdx.y;
    if (ot >= tiles_a * tiles_c) return;
    const long nchunk = (J.n + GCH - 1) / GCH;
    if ((long)blockIdx.x >= nchunk) return;
    const int ia0 = (ot / tiles_c) * GT, jc0 = (ot % tiles_c) * GT;
    const long r0 = (long)blockIdx.x * GCH;
    const long r1 = r0 + GCH < J.n ? r0 + GCH : J.n;
    const int oi = threadIdx.x % GT, oj = (threadIdx.x / GT) % GT;   // output (oi, oj) ... 256 = 16x16
    double acc = 0.0;
    for (long rb = r0; rb < r1; rb += GR) {
        // stage slab: GR rows x GT cols of X and of Y (column-major panels)
        for (int k = threadIdx.x; k < GR * GT; k += NT) {
            const int rr = k % GR, cc = k / GR;
            const long row = rb + rr;
            const int xa = ia0 + cc, yc = jc0 + cc;
            xs[rr][cc] = (row < r1 && xa < J.a) ? J.X[row + (long)xa * J.ldx] : 0.0;
            ys[rr][cc] = (row < r1 && yc < J.c) ? J.Y[row + (long)yc * J.ldy] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < GR; ++rr) acc = fma(xs[rr][oi], ys[rr][oj], acc);
        __syncthreads();
    }
    const long off = J.sc_off + ((long)ot * nchunk + blockIdx.x) * (GT * GT);
    scratch[off + oi * GT + oj] = acc;
}

__global__ void k_gram_reduce(const GramJob *__restrict__ jobs, const double *__restrict__ scratch)
{
    const GramJob J = jobs[blockIdx.y];
    const int tiles_c = (J.c + GT - 1) / GT;
    const long nchunk = (J.n + GCH - 1) / GCH;
    const int total = J.a * J.c;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
        const int i = k / J.c, j = k % J.c;
        const int ot = (i / GT) * tiles_c + (j / GT);
        const double *src = scratch + J.sc_off + (long)ot * nchunk * (GT * GT) + (i % GT) * GT + (j % GT);
        double s = 0.0;
        for (long ch = 0; ch < nchunk; ++ch) s += src[ch * (GT * GT)];
        J.C[k] = s;
    }
}

size_t gram_scratch_doubles(const GramJob *jh, int njobs)
{
    size_t t = 0;
    for (int i = 0; i < njobs; ++i) {
        const long nchunk = (jh[i].n + GCH - 1) / GCH;
        const long ntiles = (long)((jh[i].a + GT - 1) / GT) * ((jh[i].c + GT - 1) / GT);
        t += (size_t)(nchunk * ntiles * GT * GT);
    }
    return t;
}

hipError_t launch_gram(const GramJob *jobs_dev, const GramJob *jh, int njobs, double *scratch,
                       size_t scratch_doubles, hipStream_t s)
{
    long maxchunk = 1, maxtiles = 1;
    for (int i = 0; i < njobs; ++i) {
        const long nchunk = (jh[i].n + GCH - 1) / GCH;
        const long ntiles = (long)((jh[i].a + GT - 1) / GT) * ((jh[i].c + GT - 1) / GT);
        if (nchunk > maxchunk) maxchunk = nchunk;
        if (ntiles > maxtiles) maxtiles = ntiles;
        if (jh[i].sc_off + (size_t)(nchunk * ntiles * GT * GT) > scratch_doubles) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_gram, dim3(maxchunk, maxtiles, njobs), dim3(NT), 0, s, jobs_dev, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce, dim3(8, njobs), dim3(NT), 0, s, jobs_dev, scratch);
    return hipGetLastError();
}

// Y = beta Y + X Q (or Y = Y0 + X Q) over n rows; Q is a x c, column-major.
constexpr int CJ = 16;   // output columns per register chunk
__global__ __launch_bounds__(NT) void k_combo(const ComboJob *__restrict__ jobs)
{
    const ComboJob J = jobs[blockIdx.y];
    const int a = J.a, c = J.c;
    for (long r = blockIdx.x * (long)NT + threadIdx.x; r < J.n; r += (long)gridDim.x * NT) {
        for (int j0 = 0; j0 < c; j0 += CJ) {
            double s[CJ];
#pragma unroll
            for (int u = 0; u < CJ; ++u) {
                const int j = j0 + u;
                double v = 0.0;
                if (j < c) {
                    if (J.Y0) v = J.Y0[r + (long)j * J.ldy0];
                    else if (J.beta != 0.0) v = J.beta * J.Y[r + (long)j * J.ldy];
                }
                s[u] = v;
            }
            for (int k = 0; k < a; ++k) {
                const double xv = J.X[r + (long)k * J.ldx];
                const double *qk = J.Q + k;
#pragma unroll
                for (int u = 0; u < CJ; ++u)
                    if (j0 + u < c) s[u] = fma(xv, qk[(long)(j0 + u) * J.ldq], s[u]);
            }
#pragma unroll
            for (int u = 0; u < CJ; ++u)
                if (j0 + u < c) J.Y[r + (long)(j0 + u) * J.ldy] = s[u];
        }
    }
}

hipError_t launch_combo(const ComboJob *jobs_dev, const ComboJob *jh, int njobs, hipStream_t s)
{
    long nmax = 1;
    for (int i = 0; i < njobs; ++i) if (jh[i].n > nmax) nmax = jh[i].n;
    int gx = grid_for(nmax);
    if (gx > 2048) gx = 2048;
    hipLaunchKernelGGL(k_combo, dim3(gx, njobs), dim3(NT), 0, s, jobs_dev);
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
                                             double *__restrict__ dgp)
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
        double sh = 0.0, sv = 0.0;
        for (int l = 0; l < m; ++l) {
            const double *x = X + l * ld, *la = L + l * ld;
            if (j < nx - 1) sh += gam[l] * (la[gi + 1] - la[gi]) * (x[gi + 1] - x[gi]);
            if (i < ny - 1) sv += gam[l] * (la[gi + nx] - la[gi]) * (x[gi + nx] - x[gi]);
        }
        dwh[gi] = -sh;
        dwv[gi] = -sv;
    }
}

hipError_t launch_grad(const double *X, const double *Lam, long ld, const double *gammas_dev, int m,
                       const double *wh, const double *wv, int ny, int nx, double *dw_h, double *dw_v,
                       double *dg_partial, int nchunks, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad, dim3(nchunks), dim3(NT), 0, s, X, Lam, ld, gammas_dev, m, wh, wv, ny, nx, dw_h,
                       dw_v, dg_partial);
    return hipGetLastError();
}

// ------------------------------------------------- persistent CG kernel --
// Grid barrier: a monotone arrival counter.  Barrier k completes when the
// counter reaches (k+1)*G.  The wait is bounded: past the time limit the
// waiting workgroup raises the abort flag and every workgroup leaves the
// kernel at its next barrier, so the grid always drains.
__device__ __forceinline__ bool grid_barrier(unsigned long long *bar, unsigned long long target,
                                             int *abort_flag, long long timeout, int *s_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long t0 = realtime();
        int ok = 1;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
            if ((long long)(realtime() - t0) > timeout) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// Exclusive scan of n <= 2*NT ints in LDS (in place); returns the total.
__device__ int block_excl_scan(int *v, int n, int *tmp /* NT/64 ints */)
{
    const int t = threadIdx.x;
    const int i0 = 2 * t, i1 = 2 * t + 1;
    const int a0 = i0 < n ? v[i0] : 0, a1 = i1 < n ? v[i1] : 0;
    int s = a0 + a1;
    // inclusive scan of s across the wave
    const int lane = t & 63, wid = t >> 6;
    int incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) tmp[wid] = incl;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wid) base += tmp[w];
        total += tmp[w];
    }
    const int excl = base + incl - s;
    if (i0 < n) v[i0] = excl;
    if (i1 < n) v[i1] = excl + a0;
    __syncthreads();
    return total;
}

// Work assignment of one phase: active systems in order, their tiles
// concatenated and split into G chunks of ipb items.
struct Assign {
    int *act;    // [MAXSYS] system ids
    int *pre;    // [MAXSYS+1] tile prefix
    int *foff;   // [MAXSYS+1] prefix of chunk counts (flat partial offsets)
    int *pos;    // [MAXSYS] system id -> position (-1 if inactive)
};

__device__ __forceinline__ int chunk_of_block(int b, int G)
{
    // XCD-aware: workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous run of chunks so neighbouring tiles share an L2.
    if (G % 8 == 0) return (b % 8) * (G / 8) + b / 8;
    return b;
}

__device__ __forceinline__ int nch_of(int pre_a, int nt, int ipb)
{
    return (pre_a + nt - 1) / ipb - pre_a / ipb + 1;
}

// Builds pre/foff for the systems listed in act[0..m) (act already filled).
__device__ void build_assign(const CGArgs &A, Assign &S, int m, int G, int *s_m, int *s_ipb, int *tmp)
{
    for (int k = threadIdx.x; k < m; k += NT) S.pre[k] = A.sys[S.act[k]].ntiles;
    __syncthreads();
    const int T = block_excl_scan(S.pre, m, tmp);
    if (threadIdx.x == 0) {
        S.pre[m] = T;
        *s_m = m;
        *s_ipb = T > 0 ? (T + G - 1) / G : 1;
    }
    __syncthreads();
    const int ipb = *s_ipb;
    for (int k = threadIdx.x; k < m; k += NT) S.foff[k] = nch_of(S.pre[k], A.sys[S.act[k]].ntiles, ipb);
    __syncthreads();
    const int F = block_excl_scan(S.foff, m, tmp);
    if (threadIdx.x == 0) S.foff[m] = F;
    for (int k = threadIdx.x; k < MAXSYS; k += NT) S.pos[k] = -1;
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += NT) S.pos[S.act[k]] = k;
    __syncthreads();
}

// Deterministic block-wide sum of cnt consecutive partial values of one
// system: part[(base + k) * nv + v0 + j] over k < nch.  Result in out[0..cnt).
__device__ void block_reduce_partials(const double *part, int base, int nch, int nv, int v0, int cnt,
                                      double *out, double *red)
{
    double acc[NVB];
#pragma unroll
    for (int j = 0; j < NVB; ++j) acc[j] = 0.0;
    for (int k = threadIdx.x; k < nch; k += NT) {
        const double *p = part + (long)(base + k) * nv + v0;
#pragma unroll
        for (int j = 0; j < NVB; ++j)
            if (j < cnt) acc[j] += p[j];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NVB; ++j)
        if (j < cnt) {
            const double s = wave_sum(acc[j]);
            if (lane == 0) red[wid * NVB + j] = s;
        }
    __syncthreads();
    if (threadIdx.x < cnt) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w * NVB + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

__global__ __launch_bounds__(NT) void k_cg(CGArgs A)
{
    extern __shared__ double smem[];
    double *tile = smem;                                    // stencil buffers / reduction scratch
    double *s_rho = smem + A.tile_lds;                      // [MAXSYS] current r.r
    double *s_rho_old = s_rho + MAXSYS;                     // [MAXSYS] previous r.r
    int *ib = (int *)(s_rho_old + MAXSYS);
    Assign S[2];
    for (int u = 0; u < 2; ++u) {
        S[u].act = ib; ib += MAXSYS;
        S[u].pre = ib; ib += MAXSYS + 1;
        S[u].foff = ib; ib += MAXSYS + 1;
        S[u].pos = ib; ib += MAXSYS;
    }
    __shared__ int s_m[2], s_ipb[2], s_tmp[NT / 64], s_flag;
    __shared__ double s_red[(NT / 64) * NVB];
    __shared__ double s_vals[NVB + 2];                      // scalars of the current system
    __shared__ double s_mu[QMAX];

    const int G = A.G;
    const int chunk = chunk_of_block(blockIdx.x, G);
    unsigned long long bar_target = 0;
    int cur = 0;   // S[cur] = assignment of the phase being executed

    // initial assignment: every system
    for (int k = threadIdx.x; k < A.nsys; k += NT) S[0].act[k] = k;
    __syncthreads();
    build_assign(A, S[0], A.nsys, G, &s_m[0], &s_ipb[0], s_tmp);

    // ---- phase R: partials of r.r and Z^T r for the initial residuals
    // (shared with phase 2 below through the lambda-free helper macro body)
    auto run_phase2 = [&](const Assign &As, int m, int ipb, bool update, int it) {
        const int T = As.pre[m];
        const int lo = chunk * ipb;
        const int hi = lo + ipb < T ? lo + ipb : T;
        if (lo >= hi) return;
        // locate the first system
        int a = 0;
        {
            int l = 0, h = m - 1;
            while (l < h) { const int md = (l + h + 1) >> 1; if (As.pre[md] <= lo) l = md; else h = md - 1; }
            a = l;
        }
        int cur_sys = -1;
        double racc[NVB];
        double alpha = 0.0;
        int q = 0;
        const double *Zp = nullptr;
        long ldw = 0;
        for (int item = lo; item < hi; ++item) {
            while (item >= As.pre[a + 1]) ++a;
            const int s = As.act[a];
            if (s != cur_sys) {
                if (cur_sys >= 0) {
                    // flush partials of the previous system
                    const int pa = As.pos[cur_sys];
                    const int slot = chunk - As.pre[pa] / ipb;
                    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
                    for (int j = 0; j < NVB; ++j)
                        if (j < 1 + q) {
                            const double sm = wave_sum(racc[j]);
                            if (lane == 0) s_red[wid * NVB + j] = sm;
                        }
                    __syncthreads();
                    if (threadIdx.x < 1 + q) {
                        double sm = 0.0;
                        for (int w = 0; w < NT / 64; ++w) sm += s_red[w * NVB + threadIdx.x];
                        A.partB[(long)(A.sys[cur_sys].tile_base + slot) * NVB + threadIdx.x] = sm;
                    }
                    __syncthreads();
                }
                cur_sys = s;
                q = A.sys[s].q;
                Zp = A.sys[s].Z;
                ldw = A.sys[s].ldw;
#pragma unroll
                for (int j = 0; j < NVB; ++j) racc[j] = 0.0;
                if (update) {
                    // alpha = rho / p.w with p.w reduced from this assignment's partials
                    block_reduce_partials(A.partA, A.sys[s].tile_base, As.foff[a + 1] - As.foff[a], 1, 0, 1,
                                          s_vals, s_red);
                    const double pw = s_vals[0];
                    alpha = (pw > 0.0 && isfinite(pw)) ? s_rho[s] / pw : 0.0;
                    if (!(pw > 0.0 && isfinite(pw))) alpha = -1.0;  // marker: breakdown
                }
            }
            const SysDev &Y = A.sys[s];
            const InstDev &I = A.inst[Y.inst];
            const int t = item - As.pre[a];
            const int y0 = (t / I.ntx) * I.ty, x0 = (t % I.ntx) * I.tx;
            const double *pnew = ((it + 1) & 1) ? Y.p1 : Y.p0;
            for (int k = threadIdx.x; k < I.ty * I.tx; k += NT) {
                const int gy = y0 + k / I.tx, gx = x0 + k % I.tx;
                if (gy >= I.ny || gx >= I.nx) continue;
                const long gi = (long)gy * I.nx + gx;
                double rn = Y.r[gi];
                if (update && alpha >= 0.0) {
                    Y.x[gi] = fma(alpha, pnew[gi], Y.x[gi]);
                    rn = fma(-alpha, Y.w[gi], rn);
                    Y.r[gi] = rn;
                }
                racc[0] = fma(rn, rn, racc[0]);
#pragma unroll
                for (int j = 0; j < QMAX; ++j)
                    if (j < q) racc[1 + j] = fma(Zp[j * ldw + gi], rn, racc[1 + j]);
            }
            if (update && alpha < 0.0) racc[0] = -1e300 / (double)NT;   // propagate breakdown
        }
        if (cur_sys >= 0) {
            const int pa = As.pos[cur_sys];
            const int slot = chunk - As.pre[pa] / ipb;
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
            for (int j = 0; j < NVB; ++j)
                if (j < 1 + q) {
                    const double sm = wave_sum(racc[j]);
                    if (lane == 0) s_red[wid * NVB + j] = sm;
                }
            __syncthreads();
            if (threadIdx.x < 1 + q) {
                double sm = 0.0;
                for (int w = 0; w < NT / 64; ++w) sm += s_red[w * NVB + threadIdx.x];
                A.partB[(long)(A.sys[cur_sys].tile_base + slot) * NVB + threadIdx.x] = sm;
            }
            __syncthreads();
        }
    };

    run_phase2(S[0], s_m[0], s_ipb[0], false, -1);
    int nbar = 0;
    if (!grid_barrier(A.bar, (unsigned long long)(++nbar) * G, A.abort_flag, A.timeout_ticks, &s_flag)) return;

    for (int it = 0;; ++it) {
        // ---- reduce r.r of every active system (assignment S[cur]) and decide
        Assign &O = S[cur];
        const int mo = s_m[cur], ipbo = s_ipb[cur];
        const int F = O.foff[mo];
        double *flat = tile;
        for (int f = threadIdx.x; f < F; f += NT) {
            int l = 0, h = mo - 1;
            while (l < h) { const int md = (l + h + 1) >> 1; if (O.foff[md] <= f) l = md; else h = md - 1; }
            const int k = f - O.foff[l];
            flat[f] = A.partB[(long)(A.sys[O.act[l]].tile_base + k) * NVB];
        }
        __syncthreads();
        Assign &N = S[cur ^ 1];
        int *keep = N.pos;   // scratch flags, rebuilt by build_assign
        if (mo <= 16) {
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
            for (int a = wid; a < mo; a += NT / 64) {
                double v = 0.0;
                for (int k = O.foff[a] + lane; k < O.foff[a + 1]; k += 64) v += flat[k];
                v = wave_sum(v);
                if (lane == 0) flat[F + a] = v;
            }
        } else {
            for (int a = threadIdx.x; a < mo; a += NT) {
                double v = 0.0;
                for (int k = O.foff[a]; k < O.foff[a + 1]; ++k) v += flat[k];
                flat[F + a] = v;
            }
        }
        __syncthreads();
        for (int a = threadIdx.x; a < mo; a += NT) {
            const int s = O.act[a];
            const double rho = flat[F + a];
            int st = 0;
            if (!isfinite(rho)) st = -3;
            else if (rho < 0.0) st = -4;
            else if (sqrt(rho) <= A.sys[s].tolabs) st = 1;
            else if (it >= A.maxit) st = 2;
            s_rho_old[s] = s_rho[s];
            s_rho[s] = rho;
            keep[a] = (st == 0);
            if (st != 0 && blockIdx.x == 0) {
                A.out_status[s] = st;
                A.out_iters[s] = it;
                A.out_rho[s] = rho;
            }
        }
        __syncthreads();
        // compact the active list
        int *newpos = N.foff;   // scratch
        for (int a = threadIdx.x; a < mo; a += NT) newpos[a] = keep[a];
        __syncthreads();
        const int mn = block_excl_scan(newpos, mo, s_tmp);
        for (int a = threadIdx.x; a < mo; a += NT)
            if (keep[a]) N.act[newpos[a]] = O.act[a];
        __syncthreads();
        if (mn == 0) break;
        build_assign(A, N, mn, G, &s_m[cur ^ 1], &s_ipb[cur ^ 1], s_tmp);
        const int ipbn = s_ipb[cur ^ 1];

        // ---- phase 1 under N: p = r + beta p - W mu, w = B p, partial p.w
        {
            const int T = N.pre[mn];
            const int lo = chunk * ipbn;
            const int hi = lo + ipbn < T ? lo + ipbn : T;
            int a = 0;
            if (lo < hi) {
                int l = 0, h = mn - 1;
                while (l < h) { const int md = (l + h + 1) >> 1; if (N.pre[md] <= lo) l = md; else h = md - 1; }
                a = l;
            }
            int cur_sys = -1;
            double pacc = 0.0;
            for (int item = lo; item < hi; ++item) {
                while (item >= N.pre[a + 1]) ++a;
                const int s = N.act[a];
                const SysDev &Y = A.sys[s];
                if (s != cur_sys) {
                    if (cur_sys >= 0) {
                        const double sm = wave_sum(pacc);
                        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = sm;
                        __syncthreads();
                        if (threadIdx.x == 0) {
                            const int pa = N.pos[cur_sys];
                            A.partA[A.sys[cur_sys].tile_base + (chunk - N.pre[pa] / ipbn)] =
                                s_red[0] + s_red[1] + s_red[2] + s_red[3];
                        }
                        __syncthreads();
                    }
                    cur_sys = s;
                    pacc = 0.0;
                    // mu = Ginv (Z^T r) from the previous assignment's partials
                    if (Y.q > 0) {
                        const int po = O.pos[s];
                        block_reduce_partials(A.partB, Y.tile_base, O.foff[po + 1] - O.foff[po], NVB, 1, Y.q,
                                              s_vals, s_red);
                        if (threadIdx.x < Y.q) {
                            double m = 0.0;
                            for (int j = 0; j < Y.q; ++j) m += Y.Ginv[threadIdx.x * QMAX + j] * s_vals[j];
                            s_mu[threadIdx.x] = m;
                        }
                        __syncthreads();
                    }
                }
                const double beta = it > 0 ? s_rho[s] / s_rho_old[s] : 0.0;
                const InstDev &I = A.inst[Y.inst];
                const Geo g = make_geo(I.ty, I.tx, I.sy, I.sx);
                const int t = item - N.pre[a];
                const int y0 = (t / I.ntx) * I.ty, x0 = (t % I.ntx) * I.tx;
                const double *pold = (it & 1) ? Y.p1 : Y.p0;
                double *pnew = (it & 1) ? Y.p0 : Y.p1;
                const int q = Y.q;
                for (int k = threadIdx.x; k < g.H0 * g.W0; k += NT) {
                    const int li = k / g.W0, lj = k % g.W0;
                    const int gy = y0 - g.hy + li, gx = x0 - g.hx + lj;
                    double v = 0.0;
                    if (gy >= 0 && gy < I.ny && gx >= 0 && gx < I.nx) {
                        const long gi = (long)gy * I.nx + gx;
                        v = Y.r[gi];
                        if (it > 0) v = fma(beta, pold[gi], v);
                        for (int j = 0; j < q; ++j) v = fma(-s_mu[j], Y.W[j * Y.ldw + gi], v);
                        if (li >= g.hy && li < g.hy + I.ty && lj >= g.hx && lj < g.hx + I.tx) pnew[gi] = v;
                    }
                    tile[li * g.P0 + lj] = v;
                }
                __syncthreads();
                tile_E(I, g, tile, y0, x0, Y.gamma);
                tile_A(I, g, tile, y0, x0, 1.0);
                const double *ebuf = tile + g.offE;
                for (int k = threadIdx.x; k < I.ty * I.tx; k += NT) {
                    const int i = k / I.tx, j = k % I.tx;
                    const int gy = y0 + i, gx = x0 + j;
                    if (gy < I.ny && gx < I.nx) {
                        const long gi = (long)gy * I.nx + gx;
                        const double y = ebuf[i * g.PE + j];
                        Y.w[gi] = y;
                        pacc = fma(pnew[gi], y, pacc);
                    }
                }
                __syncthreads();
            }
            if (cur_sys >= 0) {
                const double sm = wave_sum(pacc);
                if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = sm;
                __syncthreads();
                if (threadIdx.x == 0) {
                    const int pa = N.pos[cur_sys];
                    A.partA[A.sys[cur_sys].tile_base + (chunk - N.pre[pa] / ipbn)] =
                        s_red[0] + s_red[1] + s_red[2] + s_red[3];
                }
                __syncthreads();
            }
        }
        if (!grid_barrier(A.bar, (unsigned long long)(++nbar) * G, A.abort_flag, A.timeout_ticks, &s_flag)) return;
        // ---- phase 2 under N
        run_phase2(N, mn, ipbn, true, it);
        if (!grid_barrier(A.bar, (unsigned long long)(++nbar) * G, A.abort_flag, A.timeout_ticks, &s_flag)) return;
        cur ^= 1;
        (void)ipbo;
    }
}

int tile_lds_doubles_min() { return 2048; }

size_t cg_lds_bytes(int tile_lds)
{
    size_t d = (size_t)tile_lds + 2 * MAXSYS;                    // tile + rho arrays
    size_t ints = 2 * (size_t)(MAXSYS + (MAXSYS + 1) + (MAXSYS + 1) + MAXSYS);
    return d * sizeof(double) + ints * sizeof(int);
}

int cg_max_blocks_per_cu(size_t lds)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cg, NT, lds) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_cg(const CGArgs &a, int G, size_t lds, hipStream_t s, bool cooperative)
{
    if (cooperative) {
        void *args[] = {(void *)&a};
        return hipLaunchCooperativeKernel((const void *)k_cg, dim3(G), dim3(NT), args, (unsigned)lds, s);
    }
    hipLaunchKernelGGL(k_cg, dim3(G), dim3(NT), lds, s, a);
    return hipGetLastError();
}

}  // namespace rsr
