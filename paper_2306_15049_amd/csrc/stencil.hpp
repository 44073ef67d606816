// LDS-tiled application of the shifted operator on one output tile.
//
// The operator is B = cA K^T K + cE E with K a zero-boundary 2-D convolution
// by the PSF and E = D^T W D (Section 2.1, eq. blkeqn).  A workgroup stages
// its input on a (TY + 2hy) x (TX + 2hx) window in LDS (hy = 2 ry: K^T K
// reaches two PSF radii) and then:
//   * rank-1 PSF h = fy fx^T (square after zero padding, S = 2r + 1 taps):
//     K^T K = (Ty^T Ty) (x) (Tx^T Tx), and each factor T^T T is a band of
//     4r + 1 diagonals (the autocorrelation of the 1-D factor) except for an
//     r x r correction at each end of a line (the terms of the zero boundary).
//     So two banded passes -- along x over all window rows, then along y into
//     the tile -- plus the end corrections on tiles that touch the image edge;
//   * any other PSF: a direct 2-D conv then corr, masked in between;
//   * E on the tile from the 5-point neighbourhood and the weight planes.
// Each thread of a banded pass produces R consecutive outputs from a sliding
// register window, so an output costs (R + taps - 1) / R LDS reads.
#pragma once
#include "internal.hpp"

namespace rsr {

// Lane move of a double by a DPP pattern (two 32-bit moves); lanes outside
// ROWS, and lanes whose source does not exist, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane.
// DPP moves instead of LDS-crossbar shuffles: two quad swaps and the half-row
// and row mirrors leave each 16-lane row's sum in all its lanes, the row-15
// and row-31 broadcasts then accumulate the rows so that lane 63 holds the
// total, which is read out as a scalar.  The order of the additions is fixed.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_mov<0xB1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141, 0xf>(v);   // row_half_mirror
    v += dpp_mov<0x140, 0xf>(v);   // row_mirror
    v += dpp_mov<0x142, 0xa>(v);   // row_bcast15 into rows 1 and 3
    v += dpp_mov<0x143, 0xc>(v);   // row_bcast31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums over the 64 lanes of up to 16 values at once (all lanes active).  The
// values are transposed while they are reduced: at each of four DPP steps a
// lane keeps half of its remaining values, adds its partner's copy of that
// half and hands the other half over (partners: row mirror, half-row mirror,
// lane ^ 3, lane ^ 1), so 8 + 4 + 2 + 1 moves leave lane i of every 16-lane
// row with the row's sum of value i; two exchanges across rows (lane ^ 16,
// lane ^ 32) finish the sums.  Returns, in every lane, the wave total of value
// (lane & 15), 0 past NV.  Sixteen separate wave_sum calls would take 96
// moves.  The order of the additions is fixed.
template <int NV>
__device__ __forceinline__ double wave_sum16(const double (&v)[NV])
{
    static_assert(NV <= 16, "at most 16 values");
    const int i = threadIdx.x & 15;
    auto val = [&](int k) { return k < NV ? v[k] : 0.0; };
    double a[8], b[4], c[2];
    const bool hA = i & 8, hB = i & 4, hC = i & 2, hD = i & 1;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        a[k] = (hA ? val(k + 8) : val(k)) + dpp_mov<0x140, 0xf>(hA ? val(k) : val(k + 8));   // row_mirror
#pragma unroll
    for (int k = 0; k < 4; ++k)
        b[k] = (hB ? a[k + 4] : a[k]) + dpp_mov<0x141, 0xf>(hB ? a[k] : a[k + 4]);   // row_half_mirror
#pragma unroll
    for (int k = 0; k < 2; ++k)
        c[k] = (hC ? b[k + 2] : b[k]) + dpp_mov<0x1B, 0xf>(hC ? b[k] : b[k + 2]);   // quad_perm [3,2,1,0]
    double d = (hD ? c[1] : c[0]) + dpp_mov<0xB1, 0xf>(hD ? c[0] : c[1]);       // quad_perm [1,0,3,2]
    d += __shfl_xor(d, 16, 64);
    d += __shfl_xor(d, 32, 64);
    return d;
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
    int W1, P1;        // after the conv pass (direct path)
    int P2;            // pitch of width-tx intermediates (banded x output)
    int H3;            // rows after the conv pass (direct path)
    int PE;            // pitch of the output accumulator / interior copies
    int off1, offE, offP, offR, offT, total;   // offP/offR: interior copies; offT: a slot per thread
                                               // for discarded stores
    int offK;          // rank-R path: K v on the tile and its PSF-radius halo
};


__host__ __device__ inline Geo make_geo(int ty, int tx, int sy, int sx, int sep)
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
    // The banded passes read up to RB - 1 elements past the end of a line (the x
    // pass, when RB does not divide tx) or RB - 1 lines past the last one (the y
    // pass, when RB does not divide ty); those values feed only outputs beyond
    // the line, which are never stored, so the buffers are padded instead of
    // clamping every window load.  The direct path clamps its reads.
    const int sz0 = g.H0 * g.P0 + RB;
    // sep 1: x-band output; sep 2 (rank R): the x-pass output of one term (read
    // RMAX rows past its end by the strips of the y-pass) and then K v on the
    // tile plus halo; sep 0: the conv output
    const int sz1 = sep == 1 ? g.H0 * g.P2 + RB * g.P2 + RB
                  : sep == 2 ? (g.H0 + RMAX) * g.P1 + RMAX + (g.H3 + RMAX) * g.P1 + RMAX
                             : g.H3 * g.P1;
    g.off1 = (sz0 + 1) & ~1;
    g.offK = sep == 2 ? ((g.off1 + (g.H0 + RMAX) * g.P1 + RMAX + 1) & ~1) : g.off1;
    g.offE = (g.off1 + sz1 + 1) & ~1;
    g.offP = (g.offE + ty * g.PE + 1) & ~1;
    g.offR = g.offP + ty * g.PE;
    g.offT = g.offR + ty * g.PE;
    g.total = g.offT + NT;
    return g;
}

// LDS of an instance's separable-path constants, kept apart from the tile
// buffers: the x band at 0, the y band at TAPS, then the four r x r end
// corrections Lx, Rx, Ly, Ry (the layout of InstDev::band after its bands).
__host__ __device__ inline int taps_doubles(int s, int sep)
{
    return sep == 1 ? 2 * TAPS + 4 * (s / 2) * (s / 2) : sep == 2 ? 4 * RMAX * MAXS : 0;
}

// Copy the bands and end corrections into LDS (read as broadcasts by the
// passes and the end fixes).
__device__ __forceinline__ void stage_taps(const InstDev &I, double *taps)
{
    if (I.sep == 2) {   // rank-R factors: per term [fy reversed][fx reversed][fy][fx]
        const int nt = 2 * I.rank * (I.sy + I.sx);
        const gdbl *src = gp(I.band);
        for (int k = threadIdx.x; k < nt; k += NT) taps[k] = src[k];
        return;
    }
    if (!I.sep) return;
    const int r = I.sx / 2, nb = 4 * r + 1, nc = 4 * r * r;
    const gdbl *src = gp(I.band);
    for (int k = threadIdx.x; k < nb; k += NT) {
        taps[k] = src[k];
        taps[TAPS + k] = src[nb + k];
    }
    for (int k = threadIdx.x; k < nc; k += NT) taps[2 * TAPS + k] = src[2 * nb + k];
}

// out[l][e] (=|+=) sum_t b[t] in[l][e + t], t < NT_, over nlines lines of nout
// outputs.  Element e of line l is at base + l*step_l + e*step_e; consecutive
// threads take consecutive lines.  The taps are applied in chunks of CT so
// that the register window stays at R + CT - 1 values.  The R accumulators are
// independent FMA chains; stores past the end of a line go to the thread's
// slot in `trash` instead of being skipped, so that no branch separates the
// chains (a guarded store lets the compiler sink each chain into its own
// block, which serialises them).
template <int NT_, int R, int CT>
__device__ __forceinline__ void pass_band(const double *__restrict__ in, int in_e, int in_l,
                                          double *__restrict__ out, int out_e, int out_l, int nlines,
                                          int nout, const double *__restrict__ b, bool acc,
                                          double *__restrict__ trash)
{
    const int nstrip = (nout + R - 1) / R;
    const int total = nlines * nstrip;
    for (int it = threadIdx.x; it < total; it += NT) {
        const int l = it % nlines;
        const int e0 = (it / nlines) * R;
        const double *src = in + l * in_l + e0 * in_e;
        double a[R];
#pragma unroll
        for (int k = 0; k < R; ++k) a[k] = 0.0;
#pragma unroll
        for (int c0 = 0; c0 < NT_; c0 += CT) {
            constexpr int W = R + CT - 1;
            double win[W];   // elements past the line land in the buffer padding
#pragma unroll
            for (int k = 0; k < W; ++k) win[k] = (c0 + k < NT_ + R - 1) ? src[(c0 + k) * in_e] : 0.0;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c0 + c < NT_) {
                    const double t = b[c0 + c];
#pragma unroll
                    for (int k = 0; k < R; ++k) a[k] = fma(t, win[k + c], a[k]);
                }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = e0 + k;
            double *d = e < nout ? out + l * out_l + e * out_e : trash + threadIdx.x;
            if (acc) *d += a[k];
            else *d = a[k];
        }
    }
}

// Image positions of a tile's span [a0, a0 + len) that need an end correction
// of a band of radius r on a line of n: the left range [la, lb) (positions < r)
// and the right range [ra, rb) (positions >= n - r, not already in the left
// range), so every position appears once.
struct EndSpan {
    int la, nl, ra, nc;
};
__device__ __forceinline__ EndSpan end_span(int a0, int len, int n, int r)
{
    const int end = min(a0 + len, n);
    const int lb = min(end, r);
    const int nl = max(0, lb - a0);
    const int ra = max(max(n - r, a0), a0 + nl);
    const int nr = max(0, end - ra);
    return EndSpan{a0, nl, ra, nl + nr};
}

// End corrections of the x band on the x-pass output (buf1 = H0 x tx): for
// image columns j < r subtract (Lx v)[j], for j >= nx - r subtract (Rx v)[..],
// v being the staged window row (zeros outside the image).  Items run over the
// window rows times the tile's end columns only.
template <int r>
__device__ __forceinline__ void band_fix_x(const InstDev &I, const Geo &g, const double *buf0, double *buf1, int x0,
                                           const double *Lx)
{
    constexpr int rr = r * r;
    const int nx = I.nx;
    const double *Rx = Lx + rr;
    const EndSpan sp = end_span(x0, I.tx, nx, r);
    const int total = g.H0 * sp.nc;
    // two items per thread per round, their loads in flight together (a 16-row
    // tile at r = 7 has 44 x 7 items: one round instead of two)
    for (int it0 = threadIdx.x; it0 < total; it0 += 2 * NT) {
        double s[2];
        int dst[2];
        bool val[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int it = it0 + h * NT;
            val[h] = it < total;
            const int itc = val[h] ? it : it0;
            const int l = itc / sp.nc, c = itc - l * sp.nc;
            const int j = c < sp.nl ? sp.la + c : sp.ra + (c - sp.nl);
            const double *row = buf0 + l * g.P0 + g.hx - x0;   // row[i] = v at image column i
            double s0 = 0.0, s1 = 0.0;
            if (j < r) {
#pragma unroll
                for (int i = 0; i < r; ++i) s0 = fma(Lx[j * r + i], row[i], s0);
            }
            if (j >= nx - r) {
                const int p = j - (nx - r);
#pragma unroll
                for (int q = 0; q < r; ++q) s1 = fma(Rx[p * r + q], row[nx - r + q], s1);
            }
            s[h] = s0 + s1;
            dst[h] = l * g.P2 + (j - x0);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (val[h]) buf1[dst[h]] -= s[h];
    }
}

// End corrections of the y band, subtracted from the tile accumulator; the
// inputs are the x-pass output rows (buf1 row k = image row y0 - hy + k).
template <int r>
__device__ __forceinline__ void band_fix_y(const InstDev &I, const Geo &g, const double *buf1, double *ebuf, int y0,
                                           const double *Ly)
{
    constexpr int rr = r * r;
    const int tx = I.tx, ny = I.ny;
    const double *Ry = Ly + rr;
    const EndSpan sp = end_span(y0, I.ty, ny, r);
    for (int it = threadIdx.x; it < sp.nc * tx; it += NT) {
        const int c = it >> I.ltx, e = it & (tx - 1);
        const int gy = c < sp.nl ? sp.la + c : sp.ra + (c - sp.nl);
        const double *col = buf1 + (g.hy - y0) * g.P2 + e;   // col[k * P2] = value at image row k
        double s0 = 0.0, s1 = 0.0;
        if (gy < r) {
#pragma unroll
            for (int k = 0; k < r; ++k) s0 = fma(Ly[gy * r + k], col[k * g.P2], s0);
        }
        if (gy >= ny - r) {
            const int p = gy - (ny - r);
#pragma unroll
            for (int q = 0; q < r; ++q) s1 = fma(Ry[p * r + q], col[(ny - r + q) * g.P2], s1);
        }
        ebuf[(gy - y0) * g.PE + e] -= s0 + s1;
    }
}

// ebuf += cA K^T K v for a rank-1 square PSF of S = 2r + 1 taps (v staged in
// buf0, bands and end corrections staged in taps by stage_taps).
template <int S>
__device__ __forceinline__ void tile_A_sep(const InstDev &I, const Geo &g, double *lds, const double *taps, int y0,
                                           int x0, double cA)
{
    constexpr int r = S / 2, NB = 4 * r + 1;
    constexpr int R = NB <= 29 ? RB : 4;
    constexpr int CT = NB <= 29 ? NB : 16;
    double *buf0 = lds, *buf1 = lds + g.off1, *ebuf = lds + g.offE, *trash = lds + g.offT;
    const double *bx = taps, *by = taps + TAPS;
    const int ty = I.ty, tx = I.tx;
    // x band over every window row: buf0 (from column ox) -> buf1 (H0 x tx)
    pass_band<NB, R, CT>(buf0 + g.ox, 1, g.P0, buf1, 1, g.P2, g.H0, tx, bx, false, trash);
    __syncthreads();
    if (r > 0 && (x0 < r || x0 + tx > I.nx - r)) {
        band_fix_x<r>(I, g, buf0, buf1, x0, taps + 2 * TAPS);
        __syncthreads();
    }
    if (cA != 1.0) {
        for (int k = threadIdx.x; k < g.H0 * g.P2; k += NT) buf1[k] *= cA;
        __syncthreads();
    }
    // y band: buf1 (from row oy) -> ebuf (+=).  Its lines are the tile's tx
    // columns of ty outputs: with R outputs per thread a 16 x 32 tile would
    // occupy one wave, so columns are cut into strips of 4 (or 2) outputs to
    // keep every wave busy; the pass is bound by the latency of its FMA chains,
    // not by the extra window reads.
    constexpr int RY = R < 4 ? R : 4;
    if (tx * ((ty + RY - 1) / RY) >= NT)
        pass_band<NB, RY, CT>(buf1 + g.oy * g.P2, g.P2, 1, ebuf, g.PE, 1, tx, ty, by, true, trash);
    else
        pass_band<NB, 2, CT>(buf1 + g.oy * g.P2, g.P2, 1, ebuf, g.PE, 1, tx, ty, by, true, trash);
    __syncthreads();
    if (r > 0 && (y0 < r || y0 + ty > I.ny - r)) {
        band_fix_y<r>(I, g, buf1, ebuf, y0, taps + 2 * TAPS + 2 * r * r);
        __syncthreads();
    }
}

// Direct 2-D pass: out[i][j] (=|+=) mask * sum_{a,c} g[a][c] in[i+a][j+c] with
// g = psf (corr) or the psf rotated by 180 degrees (conv).
__device__ __forceinline__ void pass2d(const double *__restrict__ in, int pin, double *__restrict__ out, int pout,
                              int rows, int cols, const double *__restrict__ h, int sy, int sx, bool flip,
                              bool acc, int rlo, int rhi, int clo, int chi, double *__restrict__ trash)
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
                const double gv = flip ? gp(h)[(sy - 1 - ay) * sx + (sx - 1 - cx)] : gp(h)[ay * sx + cx];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int jj = j0 + k + cx;
                    a[k] = fma(gv, src[jj < jlast ? jj : jlast], a[k]);
                }
            }
        }
        const bool rin = (i >= rlo && i < rhi);
#pragma unroll
        for (int k = 0; k < R; ++k) {   // branch-free stores (see pass_band)
            const int j = j0 + k;
            const double v = (rin && j >= clo && j < chi) ? a[k] : 0.0;
            double *d = j < cols ? out + i * pout + j : trash + threadIdx.x;
            if (acc) *d += v;
            else *d = v;
        }
    }
}

__device__ __forceinline__ void tile_A_direct(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cA)
{
    double *buf0 = lds, *buf1 = lds + g.off1, *ebuf = lds + g.offE, *trash = lds + g.offT;
    pass2d(buf0 + g.oy * g.P0 + g.ox, g.P0, buf1, g.P1, g.H3, g.W1, I.psf, I.sy, I.sx, true, false, g.ry - y0,
           I.ny - y0 + g.ry, g.rx - x0, I.nx - x0 + g.rx, trash);
    __syncthreads();
    if (cA != 1.0) {
        for (int k = threadIdx.x; k < g.H3 * g.P1; k += NT) buf1[k] *= cA;
        __syncthreads();
    }
    pass2d(buf1, g.P1, ebuf, g.PE, I.ty, I.tx, I.psf, I.sy, I.sx, false, true, 0, I.ty, 0, I.tx, trash);
    __syncthreads();
}

// out[l][e] (=|+=) sum_{t < nt} b[t] in[l][e + t] over nlines lines of nout
// outputs, a runtime tap count (the rank-R path); R outputs per thread, stores
// past a line's end to the thread's trash slot (see pass_band).
template <int R>
__device__ __forceinline__ void pass_line(const double *__restrict__ in, int in_e, int in_l, double *__restrict__ out,
                                          int out_e, int out_l, int nlines, int nout, const double *__restrict__ b,
                                          int nt, bool acc, double *__restrict__ trash)
{
    const int nstrip = (nout + R - 1) / R;
    const int total = nlines * nstrip;
    for (int it = threadIdx.x; it < total; it += NT) {
        const int l = it % nlines;
        const int e0 = (it / nlines) * R;
        const double *src = in + l * in_l + e0 * in_e;
        double a[R];
#pragma unroll
        for (int k = 0; k < R; ++k) a[k] = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double bt = b[t];
#pragma unroll
            for (int k = 0; k < R; ++k) a[k] = fma(bt, src[(t + k) * in_e], a[k]);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = e0 + k;
            double *d = e < nout ? out + l * out_l + e * out_e : trash + threadIdx.x;
            if (acc) *d += a[k];
            else *d = a[k];
        }
    }
}

// ebuf += cA K^T K v for a PSF of rank R = I.rank (2..RMAX): h = sum_k fy_k fx_k^T,
// so K v = sum_k (Ty_k (x) Tx_k) v, each term a row pass then a column pass.
// K v is formed on the tile and its PSF-radius halo (the conv of the direct
// path, term by term), masked to the image, scaled by cA, and K^T applied to it
// on the tile (the corr, term by term) -- 2 (sy + sx) taps per output and term
// instead of the 2 sy sx of the direct stencil.
__device__ __forceinline__ void tile_A_rank(const InstDev &I, const Geo &g, double *lds, const double *taps, int y0,
                                            int x0, double cA)
{
    double *buf0 = lds, *xb = lds + g.off1, *kb = lds + g.offK, *ebuf = lds + g.offE, *trash = lds + g.offT;
    const int sy = I.sy, sx = I.sx, R = I.rank, per = 2 * (sy + sx);
    const int xrows = g.H3 + sy - 1;   // input rows of the conv column pass
    for (int k = 0; k < R; ++k) {
        const double *fyr = taps + k * per, *fxr = fyr + sy;
        pass_line<4>(buf0 + g.oy * g.P0 + g.ox, 1, g.P0, xb, 1, g.P1, xrows, g.W1, fxr, sx, false, trash);
        __syncthreads();
        pass_line<4>(xb, g.P1, 1, kb, g.P1, 1, g.W1, g.H3, fyr, sy, k > 0, trash);
        __syncthreads();
    }
    // K v exists on the image only (zero boundary), then the scale
    for (int e = threadIdx.x; e < g.H3 * g.W1; e += NT) {
        const int i = e / g.W1, j = e - i * g.W1;
        const int gy = y0 - g.ry + i, gx = x0 - g.rx + j;
        double *d = kb + i * g.P1 + j;
        *d = (gy >= 0 && gy < I.ny && gx >= 0 && gx < I.nx) ? cA * *d : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < R; ++k) {
        const double *fy = taps + k * per + sy + sx, *fx = fy + sy;
        pass_line<4>(kb, 1, g.P1, xb, 1, g.P2, g.H3, I.tx, fx, sx, false, trash);
        __syncthreads();
        pass_line<4>(xb, g.P2, 1, ebuf, g.PE, 1, I.tx, I.ty, fy, sy, true, trash);
        __syncthreads();
    }
}

// ebuf += cA K^T K (staged input in buf0, which is overwritten).
__device__ __forceinline__ void tile_A(const InstDev &I, const Geo &g, double *lds, const double *taps, int y0,
                                       int x0, double cA)
{
    if (I.sep == 2) {
        tile_A_rank(I, g, lds, taps, y0, x0, cA);
        return;
    }
    if (!I.sep) {
        tile_A_direct(I, g, lds, y0, x0, cA);
        return;
    }
#define RSR_SEP(SS) \
    case SS: tile_A_sep<SS>(I, g, lds, taps, y0, x0, cA); break;
    switch (I.sy) {
        RSR_SEP(1) RSR_SEP(3) RSR_SEP(5) RSR_SEP(7) RSR_SEP(9) RSR_SEP(11) RSR_SEP(13) RSR_SEP(15)
        RSR_SEP(17) RSR_SEP(19) RSR_SEP(21) RSR_SEP(23) RSR_SEP(25) RSR_SEP(27) RSR_SEP(29) RSR_SEP(31)
    default: break;
    }
#undef RSR_SEP
}

// E v on the tile in two steps so that the weight loads travel with the
// window loads: tile_E_load fetches the four weights of each output pixel
// (w_h at the pixel and its left neighbour, w_v at the pixel and the one above)
// into registers, tile_E_apply combines them with the staged window.  Weight
// planes carry zeros where a difference does not exist, so only neighbours
// outside the image need a test.  Tiles of more than NT * NE pixels load
// their weights in tile_E_apply.
constexpr int NE = 4;   // output pixels per thread whose weights are held in registers

struct EWts {
    double c[NE], d[NE], l[NE], u[NE];
};

__device__ __forceinline__ void tile_E_load(const InstDev &I, int y0, int x0, int kbase, double cE, EWts &w)
{
    const int tx = I.tx, nx = I.nx, ny = I.ny, ne = I.ty * I.tx;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int k = kbase + u * NT + threadIdx.x;
        const int gy = y0 + (k >> I.ltx), gx = x0 + (k & (tx - 1));
        const bool ok = cE != 0.0 && k < ne && gy < ny && gx < nx;
        const bool okl = ok && gx > 0, oku = ok && gy > 0;
        // branch-free: masked lanes load element 0 and discard it
        const long gi = ok ? (long)gy * nx + gx : 0;
        const double c = gp(I.wh)[gi], d = gp(I.wv)[gi];
        const double l = gp(I.wh)[okl ? gi - 1 : 0], up = gp(I.wv)[oku ? gi - nx : 0];
        w.c[u] = ok ? c : 0.0;
        w.d[u] = ok ? d : 0.0;
        w.l[u] = okl ? l : 0.0;
        w.u[u] = oku ? up : 0.0;
    }
}

// ebuf (=) cE * E v for the NT * NE pixels from kbase, weights in w.
__device__ __forceinline__ void tile_E_apply(const InstDev &I, const Geo &g, double *lds, int y0, int x0, int kbase,
                                             double cE, const EWts &w)
{
    const double *buf0 = lds;
    double *ebuf = lds + g.offE;
    const int tx = I.tx, nx = I.nx, ny = I.ny, ne = I.ty * I.tx;
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int k = kbase + u * NT + threadIdx.x;
        if (k < ne) {
            const int i = k >> I.ltx, j = k & (tx - 1);
            const bool ok = cE != 0.0 && y0 + i < ny && x0 + j < nx;
            double e = 0.0;
            if (ok) {
                const double *c = buf0 + (g.hy + i) * g.P0 + (g.hx + j);
                e = (w.l[u] + w.c[u] + w.u[u] + w.d[u]) * c[0] - w.l[u] * c[-1] - w.c[u] * c[1] - w.u[u] * c[-g.P0] -
                    w.d[u] * c[g.P0];
                e *= cE;
            }
            ebuf[i * g.PE + j] = e;
        }
    }
}

// ebuf = cE * E v on the whole tile (v staged in buf0); w holds the weights
// of the first NT * NE pixels (loaded beforehand by tile_E_load).
__device__ __forceinline__ void tile_E(const InstDev &I, const Geo &g, double *lds, int y0, int x0, double cE, const EWts &w)
{
    const int ne = I.ty * I.tx;
    tile_E_apply(I, g, lds, y0, x0, 0, cE, w);
    for (int base = NT * NE; base < ne; base += NT * NE) {
        EWts v;
        tile_E_load(I, y0, x0, base, cE, v);
        tile_E_apply(I, g, lds, y0, x0, base, cE, v);
    }
    __syncthreads();
}

}  // namespace rsr
