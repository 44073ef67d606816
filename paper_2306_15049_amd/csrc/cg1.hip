// Persistent deflated CG of one system whose tiles fit the grid (gfx950, FP64).
//
// The launches of the sequential mode (one shift at a time) hold a single
// system, and at the benchmark's 256 x 256 that is 128 tiles: one per
// workgroup, an iteration being a chain of dependent steps (partial sums,
// decisions, window loads, stencil, epilogue, barrier) rather than a stream of
// bytes.  This kernel is k_cg (cg.hip) with the generality that chain does not
// need taken out:
//   * each workgroup owns the same tile for the whole launch, so the tile's
//     x, p and its columns of W and Z live in registers; only r, w and ph,
//     which the neighbours' windows read, go to memory each iteration (x and
//     p once, at the end);
//   * there is no work assignment, no system switch and no grid shrink: the
//     top of an iteration reduces one system's partials, and every workgroup
//     forms c_j itself from them;
//   * what other workgroups read (r, ph, w and the partial sums) is stored
//     write-through, so publishing a step needs no L2 write-back (wst below),
//     and the steps are ordered by per-tile flags rather than a grid barrier
//     (step_sync below);
//   * a launch that records CG-Lanczos data (the LZ instantiations) stores r_j
//     and the step's coefficients as k_cg does;
//   * the step j-1 vectors on the window are loaded at the top of the
//     iteration, behind the partial sums, and their latency overlaps the
//     reductions that decide alpha and beta; the weights of E stay in
//     registers for the whole launch.
// Iteration j is otherwise the fused iteration of k_cg with coherent loads:
// the same recomputation of r_j and ph_j on the window, the same stencil, the
// same partial sums in the same slots and the same reduction order, so the
// iterates are those of k_cg.
#include "cgcore.hpp"

namespace rsr {

namespace {

// Write-through publication, the cheaper barrier for a kernel that knows the
// few arrays its neighbours read.  An agent-scope store (sc1) is written
// through the XCD's L2 to the device coherence point, and it counts as done
// (vmcnt) only once it is there.  When every such store of every wave has
// completed before the workgroup meets at the barrier, nothing written for
// other workgroups sits dirty in the L2, so the arrival needs no release: a
// release writes back the whole L2 on the barrier's critical path.  Stores
// that only this workgroup reads back (its own x and p at the end) stay plain.
__device__ __forceinline__ void wst(gdbl *p, double v)
{
    typedef __attribute__((address_space(1))) unsigned long long gu64;
    __hip_atomic_store((gu64 *)p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wst(double *p, double v) { wst(gp(p), v); }

// Step flags in place of a grid barrier.  Each workgroup publishes the end of
// its step k by writing k into its tile's flag, once its write-through stores
// have completed (every wave waits for its own before the workgroup meets),
// and then waits until every tile's flag has reached k.  That is one write and
// one poll round trip, where a counter barrier takes an arrival, a release and
// the polls of both.  The flags start at zero and only grow, so the wait for
// step k cannot be met by an older step.  Every wait is bounded as in
// grid_barrier (cgcore.hpp): past the time limit the abort flag is raised, and
// a workgroup that sees it leaves at its next wait.
__device__ __forceinline__ bool step_sync(unsigned long long *flags, int nflags, int own, bool has,
                                          unsigned long long k, int *abort_flag, long long timeout)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0 && has) __hip_atomic_store(flags + own, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool ok = true;
    if ((int)threadIdx.x < nflags) {
        // spin_until without the sleep between polls: the flags are written once per
        // step, and a poll round trip already takes a microsecond
        unsigned long long *word = flags + threadIdx.x;
        const unsigned long long t0 = realtime();
        while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = false;
                break;
            }
            if ((long long)(realtime() - t0) > timeout) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = false;
                break;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return __syncthreads_or(ok ? 0 : 1) == 0;
}

// A tile's partial sums into its slot: block_accumulate (cgcore.hpp) onto
// zeroed accumulators, each value stored by the thread that forms it (no
// second workgroup barrier; 0.0 + s keeps the rounding, and the sign of a zero,
// of accumulating onto zero).
template <int NV>
__device__ __forceinline__ void block_sum_to_slot(const double (&v)[NV], double *red, gdbl *dst, int ps, int slot)
{
    wave_partials<NV>(v, NV, red + ((int)threadIdx.x >> 6) * NVP);
    __syncthreads();
    if (threadIdx.x < NVP) {
        double val = 0.0;
        if (threadIdx.x < NV) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w * NVP + threadIdx.x];
            val = 0.0 + s;
        }
        wst(dst + (int)threadIdx.x * ps + slot, val);
    }
}

constexpr int NPX = 4;   // own pixels per thread: tiles of up to 4 NT pixels
// window rows per thread loaded at the top of an iteration (fewer for the widest
// local spaces, whose registers would spill)
template <int QT> constexpr int nbp() { return QT >= 8 ? 6 : 12; }

template <int QT, bool LZ>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1))) void k_cg1(CGArgs A, SysDev S1)
{
    constexpr int NVT = 4 + 2 * QT;   // used values per partial slot
    constexpr int NBP = nbp<QT>();
    constexpr int QW = QT > 0 ? QT : 1;
    extern __shared__ double smem[];
    double *tile = smem;                          // stencil buffers / reduction scratch
    double *taps = smem + A.tile_lds;             // bands and end corrections of the instance
    // one flag per tile after the barrier block (zero at launch)
    unsigned long long *flags = (unsigned long long *)((char *)A.bar + BAR_BYTES);
    __shared__ double s_red[(NT / 64) * NVP];
    __shared__ double s_vals[NVP];
    __shared__ double s_dec[3];                   // alpha_{j-1}, beta_j, status of iteration j
    __shared__ double s_z[QMAX];
    __shared__ double s_c[QMAX];                  // c_j (c_{-1} = 0)
    __shared__ SysDev s_sd;
    __shared__ InstDev s_id;

    {
        static_assert(sizeof(SysDev) % 8 == 0 && sizeof(InstDev) % 8 == 0, "descriptor size");
        constexpr int NSD = (int)(sizeof(SysDev) / 8), NID = (int)(sizeof(InstDev) / 8);
        if (threadIdx.x < NSD)
            ((unsigned long long *)&s_sd)[threadIdx.x] =
                A.sys ? ((const unsigned long long *)A.sys)[threadIdx.x]
                      : reinterpret_cast<const unsigned long long *>(&S1)[threadIdx.x];
        __syncthreads();
        const unsigned long long *isrc = (const unsigned long long *)(A.inst + s_sd.inst);
        if (threadIdx.x < NID) ((unsigned long long *)&s_id)[threadIdx.x] = isrc[threadIdx.x];
        if (threadIdx.x < QMAX) s_c[threadIdx.x] = 0.0;
        __syncthreads();
        stage_taps(s_id, taps);
        __syncthreads();
    }
    const SysDev &Y = s_sd;
    const InstDev &I = s_id;
    const int PS = A.pstride;
    const int q = Y.q;
    const double tol2 = Y.tolabs * Y.tolabs;      // compared with rho = ||r||^2
    const int F = Y.ntiles;                       // chunks of the system: one tile each
    const int chunk = chunk_of_block(blockIdx.x, A.G);
    const bool has = chunk < F;                   // workgroups past the tiles only reduce and wait
    const int slot = Y.tile_base + chunk;
    const int t = has ? chunk : 0;
    const int y0 = (t / I.ntx) * I.ty, x0 = (t % I.ntx) * I.tx;
    const int ne = I.ty * I.tx;
    const long ldw = Y.ldw;
    const Geo g = make_geo(I.ty, I.tx, I.sy, I.sx, I.sep);

    // own pixels k = i * NT + threadIdx.x (the order of k_cg's interior loop)
    int gi[NPX];
    bool ok[NPX];
    double xr[NPX], pr[NPX], wl[NPX][QW], zl[NPX][QW];
#pragma unroll
    for (int i = 0; i < NPX; ++i) {
        const int k = i * NT + threadIdx.x;
        const int gy = y0 + (k >> I.ltx), gx = x0 + (k & (I.tx - 1));
        ok[i] = has && k < ne && gy < I.ny && gx < I.nx;
        gi[i] = ok[i] ? gy * I.nx + gx : 0;
        xr[i] = ok[i] ? gp(Y.x)[gi[i]] : 0.0;
        pr[i] = 0.0;
#pragma unroll
        for (int j = 0; j < QT; ++j) {
            wl[i][j] = (j < q && ok[i]) ? gp(Y.W)[j * ldw + gi[i]] : 0.0;
            zl[i][j] = (j < q && ok[i]) ? gp(Y.Z)[j * ldw + gi[i]] : 0.0;
        }
    }

    // window cells of this thread: column lj, rows lbase + u * rs; the first NBP
    // of them are loaded at the top of each iteration
    const WinMap wm = win_map(g.W0);
    const int lj = threadIdx.x & ((1 << wm.lw_log) - 1);
    const int lbase = (int)threadIdx.x >> wm.lw_log;
    const int gxw = x0 - g.hx + lj;
    const bool colok = lj < g.W0 && gxw >= 0 && gxw < I.nx;
    const bool colown = lj >= g.hx && lj < g.hx + I.tx;
    int wiP[NBP];
    bool wokP[NBP], ownP[NBP];
#pragma unroll
    for (int u = 0; u < NBP; ++u) {
        const int li = lbase + u * wm.rs;
        const int gy = y0 - g.hy + li;
        wokP[u] = has && colok && li < g.H0 && gy >= 0 && gy < I.ny;
        ownP[u] = colown && li >= g.hy && li < g.hy + I.ty;
        wiP[u] = wokP[u] ? gy * I.nx + gxw : 0;
    }

    // ---- initial pass: r_0.r_0 and Z^T r_0 into the slots read by iteration 0
    {
        __syncthreads();
        double v[NVT];
#pragma unroll
        for (int j = 0; j < NVT; ++j) v[j] = 0.0;
#pragma unroll
        for (int i = 0; i < NPX; ++i) {
            if (ok[i]) {
                const double r = gp(Y.rb[0])[gi[i]];
                v[1] = fma(r, r, v[1]);
#pragma unroll
                for (int j = 0; j < QT; ++j)
                    if (j < q) v[4 + j] = fma(zl[i][j], r, v[4 + j]);
            }
        }
        if (has) {
            block_sum_to_slot<NVT>(v, s_red, gp(A.part[1]), PS, slot);
        }
    }
    int nbar = 0;
    if (!step_sync(flags + Y.tile_base, F, chunk, has, (unsigned long long)(++nbar), A.abort_flag, A.timeout_ticks))
        return;
    // optional phase timestamps of workgroup 0 (diagnostics): [it][k], k = 0..8
    auto stamp = [&](int it, int k) {
        if (A.stamps && blockIdx.x == 0 && threadIdx.x == 0 && it < DBG_ITERS)
            A.stamps[it * DBG_SLOTS + k] = __builtin_amdgcn_s_memrealtime();
    };

    EWts ew;   // the weights do not change during the launch
    tile_E_load(I, y0, x0, 0, Y.gamma, ew);

    for (int it = 0;; ++it) {
        stamp(it, 0);
        const int pj = it & 1, pk = (it + 1) & 1;      // buffers of step j and of step j - 1
        const double *pprev = (it & 1) ? A.part[0] : A.part[1];
        double *pcur = (it & 1) ? A.part[1] : A.part[0];
        // ---- the previous phase's partials: p.w, r.r, r.w, w.w and Z^T r, Z^T w
        // (issued first: loads complete in order, and these are needed first)
        double accz[QT > 0 ? 2 * QT : 1];
        const bool zok = threadIdx.x < F;
        if constexpr (QT > 0) {
            const int k = zok ? (int)threadIdx.x : 0;
            const double *pz = pprev + 4 * PS + Y.tile_base + k;
#pragma unroll
            for (int j = 0; j < 2 * QT; ++j) accz[j] = cld(pz + j * PS);
        }
        double fv[4];
        {
            const double *p = pprev + Y.tile_base + (zok ? (int)threadIdx.x : 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) fv[u] = cld(p + u * PS);
        }
        // the step j-1 vectors on the first window rows: they do not depend on
        // alpha and beta, so their loads overlap the reductions below (branch-free;
        // at j = 0 the w and p loads read r_0 and are discarded)
        const gdbl *__restrict__ rsrc = gp(it > 0 ? Y.rb[pk] : Y.rb[0]);
        const gdbl *__restrict__ wsrc = it > 0 ? gp(Y.wb[pk]) : rsrc;
        const gdbl *__restrict__ psrc = it > 0 ? gp(Y.pb[pk]) : rsrc;
        double rq[NBP], wq[NBP], pq[NBP];
#pragma unroll
        for (int u = 0; u < NBP; ++u) {
            rq[u] = cld(rsrc + wiP[u]);
            wq[u] = cld(wsrc + wiP[u]);
            pq[u] = cld(psrc + wiP[u]);
        }
        double *fl = tile;   // [4][F]
        if (zok) {
#pragma unroll
            for (int u = 0; u < 4; ++u) fl[u * F + threadIdx.x] = fv[u];
        }
        for (int f = threadIdx.x + NT; f < F; f += NT) {
            const double *p = pprev + Y.tile_base + f;
            const double v0 = cld(p), v1 = cld(p + PS), v2 = cld(p + 2 * PS), v3 = cld(p + 3 * PS);
            fl[f] = v0;
            fl[F + f] = v1;
            fl[2 * F + f] = v2;
            fl[3 * F + f] = v3;
        }
        __syncthreads();
        stamp(it, 1);
        // Z^T r, Z^T w as block_sum does it, whose second barrier is shared with
        // the decisions: wave 0 forms the flat sums (a wave reduction leaves
        // them in every lane) and decides from them without a round trip
        // through LDS.
        if constexpr (QT > 0) {
#pragma unroll
            for (int j = 0; j < 2 * QT; ++j) accz[j] = zok ? accz[j] : 0.0;
            wave_partials<2 * QT>(accz, 2 * QT, s_red + ((int)threadIdx.x >> 6) * NVP);
            __syncthreads();
            if (threadIdx.x < 2 * QT) {
                double sz = 0.0;
                for (int w = 0; w < NT / 64; ++w) sz += s_red[w * NVP + threadIdx.x];
                s_vals[threadIdx.x] = sz;
            }
        }
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = lane; k < F; k += 64)
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] += fl[u * F + k];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = wave_sum(v[u]);
            const double pw = v[0], rr = v[1], rw = v[2], ww = v[3];
            double rho, alpha = 0.0, beta = 0.0;
            int st = 0;
            if (it == 0) {
                rho = rr;
                if (!isfinite(rr)) st = -3;
            } else {
                // alpha_{j-1} from the exact rho_{j-1}; rho_j = ||r_{j-1} - alpha w_{j-1}||^2 expanded
                alpha = rr / pw;
                rho = fma(alpha, fma(alpha, ww, -2.0 * rw), rr);
                if (rho < 0.0) rho = 0.0;
                beta = rho / rr;
                if (!isfinite(pw) || !isfinite(rr) || !isfinite(rho)) st = -3;
                else if (!(pw > 0.0)) st = -4;
            }
            if (st == 0) {
                if (rho <= tol2) st = 1;
                else if (it >= A.maxit) st = 2;
            }
            if (lane == 0) {
                // Lanczos capture: alpha_{j-1}, beta_{j-1} and rho_j of a step j = it that runs
                if (LZ && st == 0 && Y.nlz > 0 && chunk == 0) {
                    if (it >= 1 && it <= Y.nlz) {
                        gp(Y.lzc)[it - 1] = alpha;
                        gp(Y.lzc)[Y.nlz + it - 1] = beta;
                    }
                    if (it < Y.nlz) gp(Y.lzc)[2 * Y.nlz + it] = rho;
                }
                s_dec[0] = alpha;
                s_dec[1] = beta;
                s_dec[2] = st;
                if (st != 0 && blockIdx.x == 0) {
                    A.out_status[0] = st;
                    A.out_iters[0] = it;
                    A.out_rho[0] = rho;
                    A.out_alpha[0] = st > 0 ? alpha : 0.0;   // x_j = x_{j-1} + alpha p_{j-1} is applied after the launch
                }
            }
        }
        __syncthreads();
        stamp(it, 2);
        const double alpha = s_dec[0], beta = s_dec[1];
        if (s_dec[2] != 0.0) {
            // x_{j-1} and p_{j-1} of the own pixels, for the step left to the host
#pragma unroll
            for (int i = 0; i < NPX; ++i)
                if (ok[i]) {
                    gp(Y.x)[gi[i]] = xr[i];
                    gp(Y.pa)[gi[i]] = pr[i];
                }
            return;
        }
        if constexpr (QT > 0) {
            // mu = Ginv (Z^T r_{j-1} - alpha Z^T w_{j-1}); c_j = beta c_{j-1} + mu
            if (threadIdx.x < q) s_z[threadIdx.x] = fma(-alpha, s_vals[QT + threadIdx.x], s_vals[threadIdx.x]);
            __syncthreads();
            if (threadIdx.x < q) {
                double m = 0.0;
                for (int j = 0; j < q; ++j) m += Y.Ginv[threadIdx.x * QMAX + j] * s_z[j];
                s_c[threadIdx.x] = fma(beta, s_c[threadIdx.x], m);
            }
            __syncthreads();
        }
        stamp(it, 3);

        if (has) {
            gdbl *__restrict__ rdst = gp(Y.rb[pj]);
            gdbl *__restrict__ wdst = gp(Y.wb[pj]);
            gdbl *__restrict__ pdst = gp(Y.pb[pj]);
            double *pbuf = tile + g.offP;
            double *rbuf = tile + g.offR;
                // stage ph_j = r_j + beta ph_{j-1} with r_j = r_{j-1} - alpha w_{j-1} on the
            // window (halo recomputed from the neighbours' step j-1 vectors)
#pragma unroll
            for (int u = 0; u < NBP; ++u) {
                const int li = lbase + u * wm.rs;
                const double wj = it > 0 ? wq[u] : 0.0, pj1 = it > 0 ? pq[u] : 0.0;
                const double rj = fma(-alpha, wj, rq[u]);
                const double ph = wokP[u] ? fma(beta, pj1, rj) : 0.0;
                double *d = (lj < g.W0 && li < g.H0) ? tile + li * g.P0 + lj : tile + g.offT + threadIdx.x;
                *d = ph;
                if (wokP[u] && ownP[u]) {
                    const int ii = (li - g.hy) * g.PE + (lj - g.hx);
                    pbuf[ii] = ph;
                    rbuf[ii] = rj;
                }
            }
            const int gx = gxw;
            for (int li0 = lbase + NBP * wm.rs; li0 < g.H0; li0 += wm.rs * NBW) {
                int wi[NBW];
                bool wok[NBW], own[NBW];
#pragma unroll
                for (int u = 0; u < NBW; ++u) {
                    const int li = li0 + u * wm.rs;
                    const int gy = y0 - g.hy + li;
                    wok[u] = colok && li < g.H0 && gy >= 0 && gy < I.ny;
                    own[u] = colown && li >= g.hy && li < g.hy + I.ty;
                    wi[u] = wok[u] ? gy * I.nx + gx : 0;
                }
                // every window cell with coherent loads (halo cells were written by
                // other workgroups), branch-free so that all loads are in flight together
                double rv[NBW], wv[NBW], pv[NBW];
#pragma unroll
                for (int u = 0; u < NBW; ++u) rv[u] = cld(rsrc + wi[u]);
                if (it > 0) {
#pragma unroll
                    for (int u = 0; u < NBW; ++u) {
                        wv[u] = cld(wsrc + wi[u]);
                        pv[u] = cld(psrc + wi[u]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < NBW; ++u) wv[u] = pv[u] = 0.0;
                }
#pragma unroll
                for (int u = 0; u < NBW; ++u) {
                    const int li = li0 + u * wm.rs;
                    const double rj = fma(-alpha, wv[u], rv[u]);
                    const double ph = wok[u] ? fma(beta, pv[u], rj) : 0.0;
                    double *d = (lj < g.W0 && li < g.H0) ? tile + li * g.P0 + lj : tile + g.offT + threadIdx.x;
                    *d = ph;
                    if (wok[u] && own[u]) {
                        const int ii = (li - g.hy) * g.PE + (lj - g.hx);
                        pbuf[ii] = ph;
                        rbuf[ii] = rj;
                    }
                }
            }
            __syncthreads();
            stamp(it, 4);
            tile_E(I, g, tile, y0, x0, Y.gamma, ew);
            tile_A(I, g, tile, taps, y0, x0, 1.0);
            stamp(it, 5);
            // interior: x_j = x_{j-1} + alpha p_{j-1}; p_j = ph_j - W c_j; w_j = B ph_j - Z c_j;
            // partials p.w, r.r, r.w, w.w, Z^T r, Z^T w
            const double *ebuf = tile + g.offE;
            double v[NVT];
#pragma unroll
            for (int j = 0; j < NVT; ++j) v[j] = 0.0;
#pragma unroll
            for (int i = 0; i < NPX; ++i) {
                const int k = i * NT + threadIdx.x;
                const int ii = ok[i] ? (k >> I.ltx) : 0, jj = ok[i] ? (k & (I.tx - 1)) : 0;
                double p = pbuf[ii * g.PE + jj];
                double w = ebuf[ii * g.PE + jj];
                const double rj = rbuf[ii * g.PE + jj];
#pragma unroll
                for (int j = 0; j < QT; ++j) {
                    p = fma(-s_c[j], wl[i][j], p);
                    w = fma(-s_c[j], zl[i][j], w);
                }
                if (ok[i]) {
                    if (it > 0) xr[i] = fma(alpha, pr[i], xr[i]);
                    pr[i] = p;
                    if (it > 0) wst(rdst + gi[i], rj);
                    if (LZ && it < Y.nlz) gp(Y.lz)[it * Y.ldw + gi[i]] = rj;   // Lanczos capture of r_j
                    wst(pdst + gi[i], pbuf[ii * g.PE + jj]);
                    wst(wdst + gi[i], w);
                    v[0] = fma(p, w, v[0]);
                    v[1] = fma(rj, rj, v[1]);
                    v[2] = fma(rj, w, v[2]);
                    v[3] = fma(w, w, v[3]);
#pragma unroll
                    for (int j = 0; j < QT; ++j) {
                        v[4 + j] = fma(zl[i][j], rj, v[4 + j]);
                        v[4 + QT + j] = fma(zl[i][j], w, v[4 + QT + j]);
                    }
                }
            }
            stamp(it, 6);
            block_sum_to_slot<NVT>(v, s_red, gp(pcur), PS, slot);
        }
        stamp(it, 7);
        if (!step_sync(flags + Y.tile_base, F, chunk, has, (unsigned long long)(++nbar), A.abort_flag,
                       A.timeout_ticks))
            return;
        stamp(it, 8);
    }
}

}  // namespace

const void *cg1_kernel(int qt, bool lz)
{
    if (lz) return qt == 0 ? (const void *)k_cg1<0, true> : (const void *)k_cg1<QMAX, true>;
    switch (qt) {
    case 0: return (const void *)k_cg1<0, false>;
    case 3: return (const void *)k_cg1<3, false>;
    case 5: return (const void *)k_cg1<5, false>;
    default: return (const void *)k_cg1<QMAX, false>;
    }
}

}  // namespace rsr
