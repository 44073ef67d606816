// LDS-tiled application of the shifted operator on one output tile.
//
// The operator is B = cA K^T K + cE E with K a zero-boundary 2-D convolution
// by the PSF and E = D^T W D (Section 2.1, eq. blkeqn).  A workgroup stages
// its input on a (TY + 2hy) x (TX + 2hx) window in LDS (hy = 2 ry: K^T K
// reaches two PSF radii) and then:
//   * rank-1 PSF h = fy fx^T (square after zero padding, S taps): four 1-D
//     passes -- x conv, x corr, y conv, y corr.  K^T K = (Ty^T Ty) (x) (Tx^T Tx)
//     because the x and y factors commute; the forward pass output is masked
//     to the image before its transpose reads it (zero boundary);
//   * any other PSF: a direct 2-D conv then corr, masked in between;
//   * E on the tile from the 5-point neighbourhood and the weight planes.
// Each thread of a pass produces R consecutive outputs from a window of
// R + S - 1 registers, so an output costs (R + S - 1) / R LDS reads and S FMAs.
#pragma once
#include "internal.hpp"

namespace rsr {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Staged-window traversal without integer division: a row of the window is
// covered by LW consecutive threads (LW = 64 or 128 >= window width), the
// NT / LW thread rows step down the window.
struct WinMap {
    int lw_log;   // log2(LW)
    int rs;       // window rows per step (NT / LW)
};
__host__ __device__ inline WinMap win_map(int W0) { return W0 <= 64 ? WinMap{6, NT / 64} : WinMap{7, NT / 128}; }

// Tile geometry shared by host (LDS sizing) and device.
struct Geo {
    int ry, rx;        // PSF radii
    int hy, hx;        // halo of the staged input (2r, at least 1 for E)
    int oy, ox;        // hy - 2ry, hx - 2rx (0 or 1)
    int H0, W0, P0;    // staged input
    int W1, P1;        // after the x conv pass
    int P2;            // width-tx intermediates
    int H3;            // rows after the y conv pass
    int PE;            // pitch of the output accumulator / interior copies
    int off1, offE, offP, total;
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
    // Passes read up to RB-1 elements past the end of a line (row passes) or
    // RB-1 lines past the last one (column passes); those values feed only
    // outputs beyond the line, which are never stored, so the buffers are padded
    // instead of clamping every window load.
    const int pad = RB * (g.P0 > g.P1 ? g.P0 : g.P1) + RB;
    const int sz0 = g.H0 * g.P0 + pad;
    const int sz1a = g.H0 * g.P1, sz1b = g.H3 * g.P2;
    const int sz1 = (sz1a > sz1b ? sz1a : sz1b) + pad;
    g.off1 = (sz0 + 1) & ~1;
    g.offE = (g.off1 + sz1 + 1) & ~1;
    g.offP = (g.offE + ty * g.PE + 1) & ~1;
    g.total = g.offP + ty * g.PE;
    return g;
}

// out[l][e] (=|+=) mask(e) * sum_c g[c] in[l][e + c] over nlines lines of nout
// outputs; g = f (corr) or reversed f (conv).  Element e of line l is at
// base + l*step_l + e*step_e.  Consecutive threads take consecutive lines.
template <int S, int R>
__device__ __forceinline__ void pass1d(const double *__restrict__ in, int in_e, int in_l, int /*nin*/,
                                       double *__restrict__ out, int out_e, int out_l, int nlines,
                                       int nout, const double *__restrict__ f, bool flip, bool acc,
                                       int lo, int hi)
{
    double g[S];
#pragma unroll
    for (int c = 0; c < S; ++c) g[c] = f[flip ? S - 1 - c : c];
    const int nstrip = (nout + R - 1) / R;
    const int total = nlines * nstrip;
    for (int it = threadIdx.x; it < total; it += NT) {
        const int l = it % nlines;
        const int e0 = (it / nlines) * R;
        const double *src = in + l * in_l + e0 * in_e;
        double win[R + S - 1];   // elements past nin land in the buffer padding
#pragma unroll
        for (int k = 0; k < R + S - 1; ++k) win[k] = src[k * in_e];
#pragma unroll
        for (int k = 0; k < R; ++k) {
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

// cA K^T K for a rank-1 square PSF of S taps: buf0 (staged input) -> ebuf (+=).
template <int S>
__device__ void tile_A_sep(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cA)
{
    constexpr int R = S <= 15 ? 8 : 4;
    double *buf0 = lds, *buf1 = lds + g.off1, *ebuf = lds + g.offE;
    const int ty = I.ty, tx = I.tx;
    // x conv: buf0 (cols from ox) -> buf1, masked to the image columns
    pass1d<S, R>(buf0 + g.ox, 1, g.P0, g.W0 - g.ox, buf1, 1, g.P1, g.H0, g.W1, I.fx, true, false,
                 g.rx - x0, I.nx - x0 + g.rx);
    __syncthreads();
    // x corr: buf1 -> buf0 (pitch P2)
    pass1d<S, R>(buf1, 1, g.P1, g.W1, buf0, 1, g.P2, g.H0, tx, I.fx, false, false, 0, tx);
    __syncthreads();
    // y conv: buf0 rows from oy -> buf1 (H3 x tx), masked to the image rows
    pass1d<S, R>(buf0 + g.oy * g.P2, g.P2, 1, g.H0 - g.oy, buf1, g.P2, 1, tx, g.H3, I.fy, true, false,
                 g.ry - y0, I.ny - y0 + g.ry);
    __syncthreads();
    if (cA != 1.0) {
        for (int k = threadIdx.x; k < g.H3 * g.P2; k += NT) buf1[k] *= cA;
        __syncthreads();
    }
    // y corr: buf1 -> ebuf (+=)
    pass1d<S, R>(buf1, g.P2, 1, g.H3, ebuf, g.PE, 1, tx, ty, I.fy, false, true, 0, ty);
    __syncthreads();
}

// Direct 2-D pass: out[i][j] (=|+=) mask * sum_{a,c} g[a][c] in[i+a][j+c] with
// g = psf (corr) or the psf rotated by 180 degrees (conv).
__device__ inline void pass2d(const double *__restrict__ in, int pin, double *__restrict__ out, int pout,
                              int rows, int cols, const double *__restrict__ h, int sy, int sx, bool flip,
                              bool acc, int rlo, int rhi, int clo, int chi)
{
    constexpr int R = 4;
    const int nstrip = (cols + R - 1) / R;
    const int total = rows * nstrip;
    for (int it = threadIdx.x; it < total; it += NT) {
        const int i = it % rows;
        const int j0 = (it / rows) * R;
        double a[R];
#pragma unroll
        for (int k = 0; k < R; ++k) a[k] = 0.0;
        const int jlast = cols + sx - 2;   // last valid input column of the row
        for (int ay = 0; ay < sy; ++ay) {
            const double *src = in + (i + ay) * pin;
            for (int cx = 0; cx < sx; ++cx) {
                const double gv = flip ? h[(sy - 1 - ay) * sx + (sx - 1 - cx)] : h[ay * sx + cx];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int jj = j0 + k + cx;
                    a[k] = fma(gv, src[jj < jlast ? jj : jlast], a[k]);
                }
            }
        }
        const bool rin = (i >= rlo && i < rhi);
#pragma unroll
        for (int k = 0; k < R; ++k) {
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

__device__ inline void tile_A_direct(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cA)
{
    double *buf0 = lds, *buf1 = lds + g.off1, *ebuf = lds + g.offE;
    pass2d(buf0 + g.oy * g.P0 + g.ox, g.P0, buf1, g.P1, g.H3, g.W1, I.psf, I.sy, I.sx, true, false, g.ry - y0,
           I.ny - y0 + g.ry, g.rx - x0, I.nx - x0 + g.rx);
    __syncthreads();
    if (cA != 1.0) {
        for (int k = threadIdx.x; k < g.H3 * g.P1; k += NT) buf1[k] *= cA;
        __syncthreads();
    }
    pass2d(buf1, g.P1, ebuf, g.PE, I.ty, I.tx, I.psf, I.sy, I.sx, false, true, 0, I.ty, 0, I.tx);
    __syncthreads();
}

// ebuf += cA K^T K (staged input in buf0, which is overwritten).
__device__ inline void tile_A(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cA)
{
    if (!I.sep) {
        tile_A_direct(I, g, lds, y0, x0, cA);
        return;
    }
#define RSR_SEP(SS) \
    case SS: tile_A_sep<SS>(I, g, lds, y0, x0, cA); break;
    switch (I.sy) {
        RSR_SEP(1) RSR_SEP(3) RSR_SEP(5) RSR_SEP(7) RSR_SEP(9) RSR_SEP(11) RSR_SEP(13) RSR_SEP(15)
        RSR_SEP(17) RSR_SEP(19) RSR_SEP(21) RSR_SEP(23) RSR_SEP(25) RSR_SEP(27) RSR_SEP(29) RSR_SEP(31)
    default: break;
    }
#undef RSR_SEP
}

// ebuf = cE * E v on the tile (v staged in buf0).  Weight planes carry zeros
// where a difference does not exist, so only neighbours outside the image need
// a test.
__device__ inline void tile_E(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cE)
{
    constexpr int NE = 4;   // outputs per thread whose weight loads are issued together
    const double *buf0 = lds;
    double *ebuf = lds + g.offE;
    const int ty = I.ty, tx = I.tx, nx = I.nx, ny = I.ny, ne = ty * tx;
    for (int base = 0; base < ne; base += NT * NE) {
        long gi[NE];
        bool ok[NE];
        int gx[NE], gy[NE];
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int k = base + u * NT + threadIdx.x;
            gy[u] = y0 + (k >> I.ltx);
            gx[u] = x0 + (k & (tx - 1));
            ok[u] = cE != 0.0 && k < ne && gy[u] < ny && gx[u] < nx;
            gi[u] = ok[u] ? (long)gy[u] * nx + gx[u] : 0;
        }
        double wc[NE], wd[NE], wl[NE], wu[NE];
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            wc[u] = ok[u] ? I.wh[gi[u]] : 0.0;
            wd[u] = ok[u] ? I.wv[gi[u]] : 0.0;
            wl[u] = (ok[u] && gx[u] > 0) ? I.wh[gi[u] - 1] : 0.0;
            wu[u] = (ok[u] && gy[u] > 0) ? I.wv[gi[u] - nx] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int k = base + u * NT + threadIdx.x;
            if (k < ne) {
                const int i = k >> I.ltx, j = k & (tx - 1);
                double e = 0.0;
                if (ok[u]) {
                    const double *c = buf0 + (g.hy + i) * g.P0 + (g.hx + j);
                    e = (wl[u] + wc[u] + wu[u] + wd[u]) * c[0] - wl[u] * c[-1] - wc[u] * c[1] - wu[u] * c[-g.P0] -
                        wd[u] * c[g.P0];
                    e *= cE;
                }
                ebuf[i * g.PE + j] = e;
            }
        }
    }
    __syncthreads();
}

}  // namespace rsr
