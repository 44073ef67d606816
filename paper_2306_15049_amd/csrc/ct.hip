// Parallel-beam CT projector of the second example (Sec. 8): K = C / ||C||_F
// with C[(a, k), (i, j)] the length of ray (a, k) inside pixel (i, j) (the
// geometry is stated with CtDev in internal.hpp).
//
//   * k_ct_fwd: CT_SUB lanes per ray.  The ray is walked along the axis it is
//     closer to (rows when |cos| >= |sin|, columns otherwise), the lanes taking
//     every CT_SUB-th row; in each row (column) the ray crosses at most two
//     pixels, found from its extent over the row's slab, and each is clipped
//     exactly.  The lanes' sums are combined in a fixed order.
//   * k_ct_back: CT_SUB lanes per pixel, taking every CT_SUB-th angle.  For an
//     angle, the rays that can meet the pixel lie within half the pixel's
//     projected width of its centre; each is clipped against the pixel with
//     the same routine and the same per-angle constants, so every entry of K^T
//     is bitwise the entry of K (only the summation order differs).
//     The back-projection also applies cE E v at the pixel (E = D^T W D), so
//     B v = (K^T K + gamma E) v is a forward and a backward launch.
//
// Both kernels take a batch of jobs (blockIdx.y), one per vector, as the
// stencil path does; the projections are bound by the clip arithmetic and the
// gathers (about 4 (ny + nx) clips per ray), not by HBM.
#include "internal.hpp"

#include <hip/hip_runtime.h>

namespace rsr {

namespace {

constexpr int CT_NT = 256;
constexpr int CT_SUB = 4;   // lanes that share one ray (forward) or one pixel (backward)

// Per-angle constants: cos, sin and the reciprocals of the direction (-sin, cos)
// of the ray's parametrisation (0 where a component is 0).
struct Dir {
    double c, s, idx, idy;
};
__device__ __forceinline__ Dir load_dir(const CtDev &I, int a)
{
    const gdbl *p = gp(I.cs) + 4 * a;
    return Dir{p[0], p[1], p[2], p[3]};
}

// Length of the line x c + y s = t inside [x0, x1] x [y0, y1]: with the line
// parametrised at unit speed as P(u) = t (c, s) + u (-s, c), each axis bounds
// u to an interval (an axis the line does not move along keeps all of it when
// the line's coordinate is inside the box, none of it otherwise).
__device__ __forceinline__ double ray_len(const Dir &d, double t, double x0, double x1, double y0, double y1)
{
    const double px = t * d.c, py = t * d.s;
    double lo = -INFINITY, hi = INFINITY;
    if (d.idx == 0.0) {
        if (!(px >= x0 && px <= x1)) return 0.0;
    } else {
        const double u1 = (x0 - px) * d.idx, u2 = (x1 - px) * d.idx;
        lo = fmax(lo, fmin(u1, u2));
        hi = fmin(hi, fmax(u1, u2));
    }
    if (d.idy == 0.0) {
        if (!(py >= y0 && py <= y1)) return 0.0;
    } else {
        const double u1 = (y0 - py) * d.idy, u2 = (y1 - py) * d.idy;
        lo = fmax(lo, fmin(u1, u2));
        hi = fmin(hi, fmax(u1, u2));
    }
    return fmax(hi - lo, 0.0);
}

// Sum over the CT_SUB consecutive lanes of a group, the same in every lane
// (pairs first, then the two pair sums).
__device__ __forceinline__ double sub_sum(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
}

__device__ __forceinline__ bool fwd_job(const CtJob &J) { return J.op == 3 || J.op == 5 || (J.op == 0 && J.cA != 0.0); }

__global__ __launch_bounds__(CT_NT) void k_ct_fwd(const CtDev *__restrict__ insts, const CtJob *__restrict__ jobs)
{
    const CtJob J = jobs[blockIdx.y];
    if (!fwd_job(J)) return;
    const CtDev I = insts[J.inst];
    const int sub = threadIdx.x & (CT_SUB - 1);
    const int ray0 = blockIdx.x * (CT_NT / CT_SUB) + (threadIdx.x / CT_SUB);
    const bool live = ray0 < I.na * I.nd;
    const int ray = live ? ray0 : 0;   // dead lanes follow ray 0 and store nothing (the group sum stays in step)
    const int a = ray / I.nd, k = ray - a * I.nd;
    const Dir dr = load_dir(I, a);
    const double c = dr.c, s = dr.s;
    const double t = (k - 0.5 * (I.nd - 1)) * I.spacing;
    const double hx = 0.5 * (I.nx - 1), hy = 0.5 * (I.ny - 1);
    const bool sq = J.op == 5;
    const gdbl *__restrict__ v = gp(J.v);
    double acc = 0.0;
    if (fabs(c) >= fabs(s)) {
        // row i spans y in [yc - 1/2, yc + 1/2]; there the ray has x = (t - y s) / c
        for (int i = sub; i < I.ny; i += CT_SUB) {
            const double yc = hy - i;
            const double xa = (t - (yc - 0.5) * s) / c, xb = (t - (yc + 0.5) * s) / c;
            int j0 = (int)floor(fmin(xa, xb) + hx + 0.5) - 1, j1 = (int)floor(fmax(xa, xb) + hx + 0.5) + 1;
            j0 = j0 < 0 ? 0 : j0;
            j1 = j1 > I.nx - 1 ? I.nx - 1 : j1;
            for (int j = j0; j <= j1; ++j) {
                const double xc = j - hx;
                const double L = ray_len(dr, t, xc - 0.5, xc + 0.5, yc - 0.5, yc + 0.5);
                if (L > 0.0) acc = sq ? fma(L, L, acc) : fma(L, v[(long)i * I.nx + j], acc);
            }
        }
    } else {
        // column j spans x in [xc - 1/2, xc + 1/2]; there the ray has y = (t - x c) / s
        for (int j = sub; j < I.nx; j += CT_SUB) {
            const double xc = j - hx;
            const double ya = (t - (xc - 0.5) * c) / s, yb = (t - (xc + 0.5) * c) / s;
            int i0 = (int)floor(hy - fmax(ya, yb) + 0.5) - 1, i1 = (int)floor(hy - fmin(ya, yb) + 0.5) + 1;
            i0 = i0 < 0 ? 0 : i0;
            i1 = i1 > I.ny - 1 ? I.ny - 1 : i1;
            for (int i = i0; i <= i1; ++i) {
                const double yc = hy - i;
                const double L = ray_len(dr, t, xc - 0.5, xc + 0.5, yc - 0.5, yc + 0.5);
                if (L > 0.0) acc = sq ? fma(L, L, acc) : fma(L, v[(long)i * I.nx + j], acc);
            }
        }
    }
    acc = sub_sum(acc);
    if (!live || sub != 0) return;
    if (sq) gp(J.sino)[ray] = acc;
    else if (J.op == 3) gp(J.y)[ray] = I.scale * acc;
    else gp(J.sino)[ray] = I.scale * acc;
}

__global__ __launch_bounds__(CT_NT) void k_ct_back(const CtDev *__restrict__ insts, const CtJob *__restrict__ jobs)
{
    const CtJob J = jobs[blockIdx.y];
    if (!(J.op == 0 || J.op == 4)) return;
    const CtDev I = insts[J.inst];
    const long n = (long)I.ny * I.nx;
    const int sub = threadIdx.x & (CT_SUB - 1);
    const long p0 = (long)blockIdx.x * (CT_NT / CT_SUB) + (threadIdx.x / CT_SUB);
    const bool live = p0 < n;
    const long p = live ? p0 : 0;      // dead lanes follow pixel 0 and store nothing
    const int i = (int)(p / I.nx), j = (int)(p - (long)i * I.nx);
    const double hx = 0.5 * (I.nx - 1), hy = 0.5 * (I.ny - 1);
    const double xc = j - hx, yc = hy - i;
    double out = 0.0;
    if (J.op == 4 || J.cA != 0.0) {
        const gdbl *__restrict__ sg = gp(J.op == 4 ? J.v : (const double *)J.sino);
        const double kc = 0.5 * (I.nd - 1);
        double acc = 0.0;
        for (int a = sub; a < I.na; a += CT_SUB) {
            const Dir dr = load_dir(I, a);
            const double c = dr.c, s = dr.s;
            const double tc = xc * c + yc * s, h = 0.5 * (fabs(c) + fabs(s));
            int k0 = (int)ceil((tc - h) / I.spacing + kc) - 1, k1 = (int)floor((tc + h) / I.spacing + kc) + 1;
            k0 = k0 < 0 ? 0 : k0;
            k1 = k1 > I.nd - 1 ? I.nd - 1 : k1;
            for (int k = k0; k <= k1; ++k) {
                const double t = (k - kc) * I.spacing;
                const double L = ray_len(dr, t, xc - 0.5, xc + 0.5, yc - 0.5, yc + 0.5);
                if (L > 0.0) acc = fma(L, sg[(long)a * I.nd + k], acc);
            }
        }
        out = I.scale * sub_sum(acc);
        if (J.op == 0) out *= J.cA;
    }
    if (!live || sub != 0) return;
    if (J.op == 0 && J.cE != 0.0) {
        // (D^T W D v) at the pixel: w_h[i,j] weights v[i,j+1] - v[i,j], w_v[i,j] weights v[i+1,j] - v[i,j]
        const gdbl *__restrict__ v = gp(J.v);
        const gdbl *__restrict__ wh = gp(I.wh);
        const gdbl *__restrict__ wv = gp(I.wv);
        const double vc = v[p];
        double e = 0.0;
        if (j > 0) e = fma(wh[p - 1], vc - v[p - 1], e);
        if (j < I.nx - 1) e = fma(-wh[p], v[p + 1] - vc, e);
        if (i > 0) e = fma(wv[p - I.nx], vc - v[p - I.nx], e);
        if (i < I.ny - 1) e = fma(-wv[p], v[p + I.nx] - vc, e);
        out = fma(J.cE, e, out);
    }
    gp(J.y)[p] = out;
}

}  // namespace

hipError_t launch_ct_fwd(const CtDev *inst_dev, const CtJob *jobs_dev, int njobs, int max_rays, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    constexpr int per = CT_NT / CT_SUB;
    hipLaunchKernelGGL(k_ct_fwd, dim3((max_rays + per - 1) / per, njobs), dim3(CT_NT), 0, s, inst_dev, jobs_dev);
    return hipGetLastError();
}

hipError_t launch_ct_back(const CtDev *inst_dev, const CtJob *jobs_dev, int njobs, long max_px, hipStream_t s)
{
    if (njobs <= 0) return hipSuccess;
    constexpr int per = CT_NT / CT_SUB;
    hipLaunchKernelGGL(k_ct_back, dim3((unsigned)((max_px + per - 1) / per), njobs), dim3(CT_NT), 0, s,
                       inst_dev, jobs_dev);
    return hipGetLastError();
}

}  // namespace rsr
