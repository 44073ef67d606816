// Persistent multi-system deflated CG (gfx950, FP64).
//
// Every system (A + gamma E) x = b of a shift set advances in one cooperative
// launch.  Deflated CG with local space W (Z = B W, G = W^T Z) takes
//   p_{j+1} = r_{j+1} + beta_j p_j - W mu_{j+1},   mu = G^{-1} Z^T r.
// To keep W off the stencil halo the kernel recurs the undeflated part
//   ph_{j+1} = r_{j+1} + beta_j ph_j,   c_{j+1} = beta_j c_j + mu_{j+1},
// so that p = ph - W c and B p = B ph - Z c: the stencil runs on ph (two
// loads per halo pixel) and W, Z are read on the tile interior only.
//
// One iteration is one grid-wide phase between two grid barriers.  At the
// top every workgroup reduces the previous phase's partials p.w, r.r, r.w, w.w
// and takes alpha_{j-1} = rho_{j-1} / p.w and rho_j = ||r_{j-1} - alpha w||^2
// (expanded from the three reduced products); the phase then recomputes
// r_j = r_{j-1} - alpha w_{j-1} and ph_j = r_j + beta ph_{j-1} on each tile's
// window (halo included, ping-pong buffers), applies B to ph_j, forms
// w_j = B ph_j - Z c_j and p_j = ph_j - W c_j, advances x by the previous step
// and leaves the partials of the next top.  The last x update is applied after
// the launch.
// The active systems' tiles are concatenated and split into G contiguous
// chunks (one per workgroup, XCD-aware), each chunk's partials land in their
// own slots, and every workgroup reduces the slots it needs in a fixed order,
// so all workgroups take identical decisions and results are deterministic.
// A system leaves the launch once sqrt(r.r) <= tol ||b|| (or on maxit /
// breakdown); the remaining tiles are re-split, and the grid shrinks to the
// workgroups that still hold tiles.
#include "cgcore.hpp"

namespace rsr {

// Exclusive scan of n <= 2*NT ints in LDS (in place); returns the total.
__device__ int block_excl_scan(int *v, int n, int *tmp)
{
    const int t = threadIdx.x;
    const int i0 = 2 * t, i1 = 2 * t + 1;
    const int a0 = i0 < n ? v[i0] : 0, a1 = i1 < n ? v[i1] : 0;
    const int s = a0 + a1;
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

// Work assignment of one phase: the active systems (ascending ids), their
// tiles concatenated, split into G chunks of ipb items.
struct Assign {
    int *act;    // [MAXSYS] system ids, ascending
    int *tb;     // [MAXSYS] their first partial slots (a copy of tile_base: no global load at the loop top)
    int *pre;    // [MAXSYS+1] tile prefix
    int *foff;   // [MAXSYS+1] prefix of chunk counts (flat partial offsets)
};

__device__ __forceinline__ int nch_of(int pre_a, int nt, int ipb)
{
    return (pre_a + nt - 1) / ipb - pre_a / ipb + 1;
}

__device__ __forceinline__ int find_pos(const int *v, int n, int key)   // last i with v[i] <= key
{
    int l = 0, h = n - 1;
    while (l < h) {
        const int md = (l + h + 1) >> 1;
        if (v[md] <= key) l = md;
        else h = md - 1;
    }
    return l;
}

// With shrink set (and G a multiple of 8) the grid may also shrink once every
// workgroup holds at most one tile (T <= G): it drops to T rounded up to a
// multiple of 8.  The workgroups past it would only wait at the barriers and
// reduce partials.  While T > G the grid is kept whole, since the active set
// only shrinks and the workgroups that leave cannot come back.  The new grid
// size is left in *s_g.
// (It takes the descriptor array, not the argument block: a reference to the
// block would make the kernel keep a copy of it in scratch.)
__device__ void build_assign(const SysDev *sys, Assign &S, int m, int G, int *s_m, int *s_ipb, int *tmp, bool shrink,
                             int *s_g)
{
    for (int k = threadIdx.x; k < m; k += NT) {
        S.pre[k] = sys[S.act[k]].ntiles;
        S.tb[k] = sys[S.act[k]].tile_base;
    }
    __syncthreads();
    const int T = block_excl_scan(S.pre, m, tmp);
    if (threadIdx.x == 0) {
        S.pre[m] = T;
        *s_m = m;
        const int ipb = T > 0 ? (T + G - 1) / G : 1;
        *s_ipb = ipb;
        int gn = G;
        if (shrink && G % 8 == 0 && T > 0 && T <= G) {
            gn = (T + 7) & ~7;
            if (gn < 8) gn = 8;
        }
        *s_g = gn;
    }
    __syncthreads();
    const int ipb = *s_ipb;
    for (int k = threadIdx.x; k < m; k += NT) S.foff[k] = nch_of(S.pre[k], sys[S.act[k]].ntiles, ipb);
    __syncthreads();
    const int F = block_excl_scan(S.foff, m, tmp);
    if (threadIdx.x == 0) S.foff[m] = F;
    __syncthreads();
}

// QT: widest local space of the launch (the loops over basis columns are
// unrolled to QT).  LZ: the launch records CG-Lanczos data for the systems that
// ask for it (a separate instantiation, so launches without it carry no trace).  Chunk partial layout: p.w, r.r, r.w, w.w, Z^T r[QT],
// Z^T w[QT] in a slot of NVP values.
// At most 256 registers per lane keeps two waves per SIMD.
// FORM 0: fused iterations, other workgroups' cells read with coherent loads
// (the L2 keeps this workgroup's own data between iterations: small launches);
// FORM 1: fused iterations, an agent-scope acquire after every barrier and plain
// window loads (halo cells shared by neighbouring tiles hit the L2: large
// launches, whose data does not stay in the L2 anyway); FORM 2: two-pass
// iterations with the same acquire and plain loads.
template <int QT, bool LZ, int FORM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((FORM == 0 && QT > 0) ? 1 : 2))) void k_cg(CGArgs A)
{
    constexpr bool TWO = FORM == 2, ACQ = FORM != 0;
    // a window cell written by another workgroup in the previous phase
    auto wld = [](const gdbl *p) -> double {
        if constexpr (ACQ) return *p;
        else return cld(p);
    };
    constexpr int NVT = 4 + 2 * QT;   // used values per partial slot
    extern __shared__ double smem[];
    double *tile = smem;                          // stencil buffers / reduction scratch
    const int ms = A.msys;                        // per-system arrays sized by the launch
    double *taps = smem + A.tile_lds;             // bands and end corrections of the staged instance
    double *s_rho = taps + A.taps_lds;            // [ms] rho_j (one recurrence step from the exact rho_{j-1})
    double *s_alpha = s_rho + ms;                 // [ms] alpha_{j-1}
    double *s_beta = s_alpha + ms;                // [ms] beta_j
    double *s_tol = s_beta + ms;                  // [ms] squared absolute tolerances (tol ||b||)^2
    int *ib = (int *)(s_tol + ms);
    Assign S0, S1;   // two named assignments (a runtime-indexed array would live in scratch)
    S0.act = ib; ib += ms;
    S0.tb = ib; ib += ms;
    S0.pre = ib; ib += ms + 1;
    S0.foff = ib; ib += ms + 1;
    S1.act = ib; ib += ms;
    S1.tb = ib; ib += ms;
    S1.pre = ib; ib += ms + 1;
    S1.foff = ib; ib += ms + 1;
    const BarCtl bc = bar_ctl(A);
    __shared__ int s_m[2], s_ipb[2], s_tmp[NT / 64], s_flag;
    __shared__ int s_g;                           // current grid size (shrinks as systems leave)
    __shared__ unsigned long long s_arr;          // arrivals counted on this workgroup's group counter
    __shared__ double s_red[(NT / 64) * NVP];
    __shared__ double s_vals[NVP];
    __shared__ double s_acc[NVP];                 // partial sums of the current system over the chunk
    __shared__ double s_z[QMAX];
    __shared__ double s_c[QMAX];                  // c_j of the current system
    // LDS copies of the current system's descriptor and of its instance: a
    // workgroup keeps the same system from one iteration to the next while the
    // assignment is unchanged, so these are refetched only when it changes
    __shared__ SysDev s_sd;
    __shared__ InstDev s_id;
    __shared__ int s_sd_sys;
    __shared__ int s_taps_inst;                   // instance whose constants are in taps (or -1)

    const int PS = A.pstride;                     // slots per value plane of the partials
    int cur = 0;
    if (threadIdx.x == 0) {
        s_sd_sys = -1;
        s_taps_inst = -1;
        s_arr = 0;
    }

    for (int k = threadIdx.x; k < A.nsys; k += NT) {
        S0.act[k] = k;
        s_tol[k] = A.sys[k].tolabs * A.sys[k].tolabs;   // compared with rho = ||r||^2
    }
    __syncthreads();
    build_assign(A.sys, S0, A.nsys, A.G, &s_m[0], &s_ipb[0], s_tmp, false, &s_g);

    auto slot_of = [&](const Assign &As, int m, int ipb, int s, int chunk) {
        const int a = find_pos(As.act, m, s);
        return As.tb[a] + (chunk - As.pre[a] / ipb);
    };

    // ---- initial pass: r_0.r_0 and Z^T r_0 into the partial slots read by iteration 0
    {
        const Assign &As = S0;
        const int m = s_m[0], ipb = s_ipb[0];
        const int chunk = chunk_of_block(blockIdx.x, A.G);
        const int T = As.pre[m];
        const int lo = chunk * ipb;
        const int hi = lo + ipb < T ? lo + ipb : T;
        double *pout = A.part[1];
        int a = lo < hi ? find_pos(As.pre, m, lo) : 0;
        int cur_sys = -1, q = 0;
        for (int item = lo; item < hi; ++item) {
            while (item >= As.pre[a + 1]) ++a;
            const int s = uni(As.act[a]);
            if (s != cur_sys) {
                if (cur_sys >= 0 && threadIdx.x < NVP) gp(pout)[(int)threadIdx.x * PS + slot_of(As, m, ipb, cur_sys, chunk)] = s_acc[threadIdx.x];
                cur_sys = s;
                q = A.sys[s].q;
                if (threadIdx.x < NVP) s_acc[threadIdx.x] = 0.0;
                __syncthreads();
            }
            const SysDev &Y = A.sys[s];
            const InstDev I = A.inst[Y.inst];
            const gdbl *__restrict__ Yr = gp(Y.rb[0]);
            const gdbl *__restrict__ YZ = gp(Y.Z);
            const long ldw = Y.ldw;
            const int t = uni(item - As.pre[a]);
            const int y0 = (t / I.ntx) * I.ty, x0 = (t % I.ntx) * I.tx;
            const int ne = I.ty * I.tx;
            double v[NVT];
#pragma unroll
            for (int j = 0; j < NVT; ++j) v[j] = 0.0;
            for (int k = threadIdx.x; k < ne; k += NT) {
                const int gy = y0 + (k >> I.ltx), gx = x0 + (k & (I.tx - 1));
                if (gy < I.ny && gx < I.nx) {
                    const int gi = gy * I.nx + gx;
                    const double r = Yr[gi];
                    v[1] = fma(r, r, v[1]);
#pragma unroll
                    for (int j = 0; j < QT; ++j)
                        if (j < q) v[4 + j] = fma(YZ[j * ldw + gi], r, v[4 + j]);
                }
            }
            block_accumulate<NVT>(v, NVT, s_acc, s_red);
        }
        if (cur_sys >= 0 && threadIdx.x < NVP) gp(pout)[(int)threadIdx.x * PS + slot_of(As, m, ipb, cur_sys, chunk)] = s_acc[threadIdx.x];
    }
    int nbar = 0;
    if (!grid_barrier(bc, (unsigned long long)(++nbar), A.timeout_ticks, &s_flag, &s_arr, &s_g)) return;

    auto stamp = [&](int it, int k) {
        if (A.stamps && threadIdx.x == 0) {
            if (blockIdx.x == 0 && it < DBG_ITERS) A.stamps[it * DBG_SLOTS + k] = realtime();
            // every workgroup's phase times over a few iterations, with its hardware slot
            if (k < 4 && it >= DBG_WG_IT0 && it < DBG_WG_IT0 + DBG_WG_NIT && blockIdx.x < DBG_WG_MAX) {
                unsigned long long *w = A.stamps + DBG_ITERS * DBG_SLOTS + ((it - DBG_WG_IT0) * DBG_WG_MAX + blockIdx.x) * 8;
                w[k] = realtime();
                if (k == 0) {
                    w[4] = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID: wave, SIMD, CU, SH, SE
                    w[5] = __builtin_amdgcn_s_getreg((31 << 11) | 20);   // XCC_ID
                }
            }
        }
    };
    // (kept in LDS: registers are the binding resource across the stencil)
    __shared__ int s_clast;   // last system of the previous phase: s_c holds its c_{j-1}
    __shared__ int s_zsys;    // system whose c_j the loop top formed (or -1)
    if (threadIdx.x == 0) s_clast = -1;
    for (int it = 0;; ++it) {
        stamp(it, 0);
        // (selects, not A.part[i]: a runtime index into the argument block would copy it to scratch)
        const double *pprev = (it & 1) ? A.part[0] : A.part[1];   // written by the previous phase (or the initial pass)
        double *pcur = (it & 1) ? A.part[1] : A.part[0];
        // ---- p.w, r.r, r.w, w.w of every active system and the decisions
        Assign O = cur ? S1 : S0;
        const int mo = s_m[cur];
        const int ipbo = s_ipb[cur];
        const int F = O.foff[mo];
        // Steady state of a deflated system: when this workgroup's chunk lies in
        // one system, the one it finished the previous phase with, the system's
        // Z^T r / Z^T w partials are loaded here together with the flat
        // partials below, and c_j is formed from the c_{j-1} kept in s_c -- one
        // global round trip fewer than at a system switch inside the phase.
        int zsys = -1, zfirst = 0;
        bool zok = false;
        double accz[QT > 0 ? 2 * QT : 1];
        if (threadIdx.x == 0) s_zsys = -1;
        if constexpr (QT > 0) {
            const int c_last = s_clast;
            const int chunk = chunk_of_block(blockIdx.x, s_g);
            const int lo = chunk * ipbo;
            const int hi = lo + ipbo < O.pre[mo] ? lo + ipbo : O.pre[mo];
            if (lo < hi && c_last >= 0 && s_sd_sys == c_last && s_sd.q > 0) {
                const int a0 = find_pos(O.pre, mo, lo);
                const int nch = O.foff[a0 + 1] - O.foff[a0];
                if (O.act[a0] == c_last && hi <= O.pre[a0 + 1] && nch <= NT) {
                    zsys = c_last;
                    zfirst = chunk == O.pre[a0] / ipbo;
                    // one slot per thread, no accumulation here: the values are first
                    // used after the flat loads below are issued, so both are in flight
                    // together (the sums equal those of partial_load, as 0 + v = v)
                    zok = threadIdx.x < nch;
                    const int k = zok ? threadIdx.x : 0;
                    const double *pz = pprev + 4 * PS + s_sd.tile_base + k;
#pragma unroll
                    for (int j = 0; j < 2 * QT; ++j) accz[j] = cld(pz + j * PS);
                }
            }
        }
        double *fl = tile;   // [4][F] then [4][mo]
        for (int f = threadIdx.x; f < F; f += NT) {
            const int l = find_pos(O.foff, mo, f);
            const double *p = pprev + O.tb[l] + (f - O.foff[l]);
            const double v0 = cld(p), v1 = cld(p + PS), v2 = cld(p + 2 * PS), v3 = cld(p + 3 * PS);
            fl[f] = v0;
            fl[F + f] = v1;
            fl[2 * F + f] = v2;
            fl[3 * F + f] = v3;
        }
        __syncthreads();
        stamp(it, 8);
        if constexpr (QT > 0) {
            if (zsys >= 0) {   // Z^T r_{j-1}, Z^T w_{j-1}
#pragma unroll
                for (int j = 0; j < 2 * QT; ++j) accz[j] = zok ? accz[j] : 0.0;
                block_sum<2 * QT>(accz, 2 * QT, s_vals, s_red);
            }
        }
        double *sums = fl + 4 * F;   // [4][mo]
        if (mo <= 16) {
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
            for (int a = wid; a < mo; a += NT / 64) {
                double v[4] = {0.0, 0.0, 0.0, 0.0};
                for (int k = O.foff[a] + lane; k < O.foff[a + 1]; k += 64)
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] += fl[u * F + k];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double sv = wave_sum(v[u]);
                    if (lane == 0) sums[u * mo + a] = sv;
                }
            }
        } else {
            for (int a = threadIdx.x; a < mo; a += NT) {
                double v[4] = {0.0, 0.0, 0.0, 0.0};
                for (int k = O.foff[a]; k < O.foff[a + 1]; ++k)
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] += fl[u * F + k];
#pragma unroll
                for (int u = 0; u < 4; ++u) sums[u * mo + a] = v[u];
            }
        }
        __syncthreads();
        stamp(it, 9);
        Assign N = cur ? S0 : S1;
        int *keep = N.pre;       // scratch, rebuilt by build_assign
        int *newpos = N.foff;    // scratch
        for (int a = threadIdx.x; a < mo; a += NT) {
            const int s = O.act[a];
            const double pw = sums[a], rr = sums[mo + a], rw = sums[2 * mo + a], ww = sums[3 * mo + a];
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
                if (rho <= s_tol[s]) st = 1;
                else if (it >= A.maxit) st = 2;
            }
            s_rho[s] = rho;
            s_alpha[s] = alpha;
            s_beta[s] = beta;
            keep[a] = (st == 0);
            newpos[a] = (st == 0);
            if (st != 0 && blockIdx.x == 0) {
                A.out_status[s] = st;
                A.out_iters[s] = it;
                A.out_rho[s] = rho;
                A.out_alpha[s] = st > 0 ? alpha : 0.0;   // x_j = x_{j-1} + alpha p_{j-1} is applied after the launch
            }
        }
        __syncthreads();
        // compact the active list (keep ascending order)
        if (mo <= 64) {
            // one wave: ballot of the flags, position = flags set in lower lanes
            if (threadIdx.x < 64) {
                const bool k = (int)threadIdx.x < mo && keep[threadIdx.x];
                const unsigned long long msk = __ballot(k);
                const int pos = __popcll(msk & ((1ull << threadIdx.x) - 1ull));
                if (k) N.act[pos] = O.act[threadIdx.x];
                if (threadIdx.x == 0) s_m[cur ^ 1] = __popcll(msk);
            }
            __syncthreads();
        } else {
            int kk[2];
            for (int u = 0; u < 2; ++u) kk[u] = (2 * threadIdx.x + u < mo) ? keep[2 * threadIdx.x + u] : 0;
            __syncthreads();
            const int mn_ = block_excl_scan(newpos, mo, s_tmp);
            for (int u = 0; u < 2; ++u) {
                const int a = 2 * threadIdx.x + u;
                if (a < mo && kk[u]) N.act[newpos[a]] = O.act[a];
            }
            if (threadIdx.x == 0) s_m[cur ^ 1] = mn_;
            __syncthreads();
        }
        const int mn = s_m[cur ^ 1];
        stamp(it, 10);
        if (mn == 0) break;
        if (mn != mo) {
            // tiles move between workgroups when the active set shrinks: drop cached copies
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int gold = s_g;
            build_assign(A.sys, N, mn, gold, &s_m[cur ^ 1], &s_ipb[cur ^ 1], s_tmp, true, &s_g);
            // every workgroup takes the same decision; the ones past the new grid
            // have published all they wrote at the last barrier
            if ((int)blockIdx.x >= s_g) return;
        } else {
            N = O;   // unchanged: keep the assignment (and its buffers)
        }
        const bool flip = mn != mo;
        if (A.stamps && blockIdx.x == 0 && threadIdx.x == 0 && it < DBG_ITERS) {
            A.stamps[it * DBG_SLOTS + 4] = mn;
            A.stamps[it * DBG_SLOTS + 5] = s_g;
        }
        const int ipbn = flip ? s_ipb[cur ^ 1] : ipbo;
        stamp(it, 11);
        if constexpr (QT > 0) {
            if (zsys >= 0 && !flip) {
                // mu = Ginv (Z^T r_{j-1} - alpha Z^T w_{j-1}); c_j = beta c_{j-1} + mu
                const SysDev &Y = s_sd;
                const int q = Y.q;
                if (threadIdx.x == 0) s_zsys = zsys;   // read inside the phase, after the syncs below
                if (threadIdx.x < q)
                    s_z[threadIdx.x] = fma(-s_alpha[zsys], s_vals[QT + threadIdx.x], s_vals[threadIdx.x]);
                __syncthreads();
                if (threadIdx.x < q) {
                    double m = 0.0;
                    for (int j = 0; j < q; ++j) m += Y.Ginv[threadIdx.x * QMAX + j] * s_z[j];
                    const double cn = fma(s_beta[zsys], s_c[threadIdx.x], m);
                    s_c[threadIdx.x] = cn;
                    if (zfirst) gp(Y.cbuf)[(it & 1) * QMAX + threadIdx.x] = cn;
                }
                __syncthreads();
            }
        }
        stamp(it, 1);

        if constexpr (TWO) {
            // ---- two-pass iterations, first pass: r_j = r_{j-1} - alpha w_{j-1} and
            // ph_j = r_j + beta ph_{j-1} on the own cells of every item of this
            // workgroup (elementwise, several cells per thread in flight); the
            // stencil pass after the barrier then reads ph_j alone on its window.
            // The tiles are those of the stencil pass, so the own cells written here
            // are read back by the same workgroup; the halo cells come from others.
            const int T = N.pre[mn];
            const int chunk = chunk_of_block(blockIdx.x, s_g);
            const int lo = chunk * ipbn;
            const int hi = lo + ipbn < T ? lo + ipbn : T;
            int a = lo < hi ? find_pos(N.pre, mn, lo) : 0;
            const int pj = it & 1, pk = (it + 1) & 1;
            for (int item = lo; item < hi; ++item) {
                while (item >= N.pre[a + 1]) ++a;
                const int s = uni(N.act[a]);
                const SysDev &Y = A.sys[s];
                const InstDev &I = A.inst[Y.inst];
                const double alpha = s_alpha[s], beta = s_beta[s];
                const int t = uni(item - N.pre[a]);
                const int y0 = (t / I.ntx) * I.ty, x0 = (t % I.ntx) * I.tx;
                const gdbl *__restrict__ rsrc = gp(it > 0 ? Y.rb[pk] : Y.rb[0]);
                gdbl *__restrict__ rdst = gp(Y.rb[pj]);
                const gdbl *__restrict__ wsrc = gp(Y.wb[pk]);
                const gdbl *__restrict__ psrc = gp(Y.pb[pk]);
                gdbl *__restrict__ pdst = gp(Y.pb[pj]);
                const int ne = I.ty * I.tx;
                constexpr int NA = 4;
                for (int base = 0; base < ne; base += NT * NA) {
                    int gi[NA];
                    bool ok[NA];
#pragma unroll
                    for (int u = 0; u < NA; ++u) {
                        const int k = base + u * NT + threadIdx.x;
                        const int gy = y0 + (k >> I.ltx), gx = x0 + (k & (I.tx - 1));
                        ok[u] = k < ne && gy < I.ny && gx < I.nx;
                        gi[u] = ok[u] ? gy * I.nx + gx : 0;
                    }
                    double rv[NA], wv[NA], pv[NA];
#pragma unroll
                    for (int u = 0; u < NA; ++u) {
                        rv[u] = rsrc[gi[u]];
                        wv[u] = it > 0 ? wsrc[gi[u]] : 0.0;
                        pv[u] = it > 0 ? psrc[gi[u]] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < NA; ++u) {
                        const double rj = fma(-alpha, wv[u], rv[u]);
                        const double ph = fma(beta, pv[u], rj);
                        if (ok[u]) {
                            if (it > 0) rdst[gi[u]] = rj;
                            if (LZ && it < Y.nlz) gp(Y.lz)[it * Y.ldw + gi[u]] = rj;   // Lanczos capture of r_j
                            pdst[gi[u]] = ph;
                        }
                    }
                }
            }
            if (!grid_barrier<ACQ>(bc, (unsigned long long)(++nbar), A.timeout_ticks, &s_flag, &s_arr, &s_g)) return;
        }

        // ---- the iteration's stencil phase under N (its only phase in fused mode)
        {
            const int T = N.pre[mn];
            const int chunk = chunk_of_block(blockIdx.x, s_g);
            const int lo = chunk * ipbn;
            const int hi = lo + ipbn < T ? lo + ipbn : T;
            int a = lo < hi ? find_pos(N.pre, mn, lo) : 0;
            int cur_sys = -1;
            int q = 0;
            double alpha = 0.0, beta = 0.0;
            for (int item = lo; item < hi; ++item) {
                while (item >= N.pre[a + 1]) ++a;
                const int s = uni(N.act[a]);
                if (s != s_sd_sys) {
                    // descriptor words, then the instance's (two dependent loads, only
                    // when the workgroup moves to another system)
                    static_assert(sizeof(SysDev) % 8 == 0 && sizeof(InstDev) % 8 == 0, "descriptor size");
                    constexpr int NSD = (int)(sizeof(SysDev) / 8), NID = (int)(sizeof(InstDev) / 8);
                    const unsigned long long *src = (const unsigned long long *)(A.sys + s);
                    if (threadIdx.x < NSD) ((unsigned long long *)&s_sd)[threadIdx.x] = src[threadIdx.x];
                    const int ii = A.sys[s].inst;
                    const unsigned long long *isrc = (const unsigned long long *)(A.inst + ii);
                    if (threadIdx.x >= 128 && threadIdx.x - 128 < NID)
                        ((unsigned long long *)&s_id)[threadIdx.x - 128] = isrc[threadIdx.x - 128];
                    __syncthreads();
                    if (threadIdx.x == 0) s_sd_sys = s;
                    if (ii != s_taps_inst) {
                        // the instance's constants stay in LDS until another instance comes
                        stage_taps(s_id, taps);
                        __syncthreads();
                        if (threadIdx.x == 0) s_taps_inst = ii;
                    }
                }
                const SysDev &Y = s_sd;
                if (s != cur_sys) {
                    if (cur_sys >= 0 && threadIdx.x < NVP)
                        gp(pcur)[(int)threadIdx.x * PS + slot_of(N, mn, ipbn, cur_sys, chunk)] = s_acc[threadIdx.x];
                    cur_sys = s;
                    q = Y.q;
                    alpha = s_alpha[s];
                    beta = s_beta[s];
                    // Lanczos capture: alpha_{j-1}, beta_{j-1} and rho_j of step j = it
                    if (LZ && Y.nlz > 0 && threadIdx.x == 0 && chunk == N.pre[a] / ipbn) {
                        if (it >= 1 && it <= Y.nlz) {
                            gp(Y.lzc)[it - 1] = alpha;
                            gp(Y.lzc)[Y.nlz + it - 1] = beta;
                        }
                        if (it < Y.nlz) gp(Y.lzc)[2 * Y.nlz + it] = s_rho[s];
                    }
                    if (threadIdx.x < NVP) s_acc[threadIdx.x] = 0.0;
                    if (threadIdx.x >= q && threadIdx.x < QMAX) s_c[threadIdx.x] = 0.0;   // unused columns
                    if (q > 0 && s != s_zsys) {
                        // Z^T r_j = Z^T r_{j-1} - alpha Z^T w_{j-1}; mu = Ginv Z^T r_j; c_j = beta c_{j-1} + mu
                        // (c_{j-1} is fetched first so that it travels with the partial-sum loads)
                        const double cold =
                            (it > 0 && threadIdx.x < q) ? cld(Y.cbuf + ((it + 1) & 1) * QMAX + threadIdx.x) : 0.0;
                        const int po = find_pos(O.act, mo, s);
                        block_reduce_partials<(QT > 0 ? 2 * QT : 1)>(pprev, PS, Y.tile_base, O.foff[po + 1] - O.foff[po], 4,
                                                                   2 * QT, s_vals, s_red);
                        if (threadIdx.x < q)
                            s_z[threadIdx.x] = fma(-alpha, s_vals[QT + threadIdx.x], s_vals[threadIdx.x]);
                        __syncthreads();
                        if (threadIdx.x < q) {
                            double m = 0.0;
                            for (int j = 0; j < q; ++j) m += Y.Ginv[threadIdx.x * QMAX + j] * s_z[j];
                            const double cn = fma(beta, cold, m);
                            s_c[threadIdx.x] = cn;
                            // the workgroup holding the system's first chunk publishes c_j
                            if (chunk == N.pre[a] / ipbn) gp(Y.cbuf)[(it & 1) * QMAX + threadIdx.x] = cn;
                        }
                    }
                    __syncthreads();
                }
                if (item == lo) stamp(it, 12);
                const InstDev &I = s_id;
                const Geo g = make_geo(I.ty, I.tx, I.sy, I.sx, I.sep);
                const int t = uni(item - N.pre[a]);
                const int y0 = (t / I.ntx) * I.ty, x0 = (t % I.ntx) * I.tx;
                // local copies: no reloads after the global stores
                const int pj = it & 1, pk = (it + 1) & 1;      // buffers of step j and of step j - 1
                const gdbl *__restrict__ rsrc = gp(it > 0 ? Y.rb[pk] : Y.rb[0]);
                gdbl *__restrict__ rdst = gp(Y.rb[pj]);
                const gdbl *__restrict__ wsrc = gp(Y.wb[pk]);
                gdbl *__restrict__ wdst = gp(Y.wb[pj]);
                const gdbl *__restrict__ psrc = gp(Y.pb[pk]);
                gdbl *__restrict__ pdst = gp(Y.pb[pj]);
                const gdbl *__restrict__ YW = gp(Y.W);
                const gdbl *__restrict__ YZ = gp(Y.Z);
                gdbl *__restrict__ Ypa = gp(Y.pa);
                gdbl *__restrict__ Yx = gp(Y.x);
                const long ldw = Y.ldw;
                const double gam = Y.gamma;
                double *pbuf = tile + g.offP;
                double *rbuf = tile + g.offR;
                // stage ph_j = r_j + beta ph_{j-1} with r_j = r_{j-1} - alpha w_{j-1} on the
                // window (halo recomputed from the neighbours' step j-1 vectors); keep the
                // interior of ph_j and r_j in LDS
                EWts ew;
                tile_E_load(I, y0, x0, 0, gam, ew);   // in flight with the window loads
                const WinMap wm = win_map(g.W0);
                const int lj = threadIdx.x & ((1 << wm.lw_log) - 1);     // window column of this thread
                const int gx = x0 - g.hx + lj;
                const bool colok = lj < g.W0 && gx >= 0 && gx < I.nx;
                const bool colown = lj >= g.hx && lj < g.hx + I.tx;
                if constexpr (TWO) {
                    // ph_j on the window as the first pass left it, all rows of a thread in
                    // flight together (r_j of the own cells is read in the epilogue)
                    const gdbl *__restrict__ phs = gp(Y.pb[pj]);
                    for (int li0 = threadIdx.x >> wm.lw_log; li0 < g.H0; li0 += wm.rs * NBW2) {
                        int gi[NBW2];
                        bool ok[NBW2];
#pragma unroll
                        for (int u = 0; u < NBW2; ++u) {
                            const int li = li0 + u * wm.rs;
                            const int gy = y0 - g.hy + li;
                            ok[u] = colok && li < g.H0 && gy >= 0 && gy < I.ny;
                            gi[u] = ok[u] ? gy * I.nx + gx : 0;
                        }
                        double pv[NBW2];
#pragma unroll
                        for (int u = 0; u < NBW2; ++u) pv[u] = wld(phs + gi[u]);
#pragma unroll
                        for (int u = 0; u < NBW2; ++u) {
                            const int li = li0 + u * wm.rs;
                            const double ph = ok[u] ? pv[u] : 0.0;
                            double *d = (lj < g.W0 && li < g.H0) ? tile + li * g.P0 + lj : tile + g.offT + threadIdx.x;
                            *d = ph;
                            if (ok[u] && colown && li >= g.hy && li < g.hy + I.ty)
                                pbuf[(li - g.hy) * g.PE + (lj - g.hx)] = ph;
                        }
                    }
                } else
                for (int li0 = threadIdx.x >> wm.lw_log; li0 < g.H0; li0 += wm.rs * NBW) {
                    int gi[NBW];
                    bool ok[NBW], own[NBW];
#pragma unroll
                    for (int u = 0; u < NBW; ++u) {
                        const int li = li0 + u * wm.rs;
                        const int gy = y0 - g.hy + li;
                        ok[u] = colok && li < g.H0 && gy >= 0 && gy < I.ny;
                        own[u] = colown && li >= g.hy && li < g.hy + I.ty;
                        gi[u] = ok[u] ? gy * I.nx + gx : 0;
                    }
                    // every window cell with coherent loads (halo cells were written by
                    // other workgroups), branch-free so that all loads are in flight
                    // together; masked lanes load element 0 and discard it
                    double rv[NBW], wv[NBW], pv[NBW];
#pragma unroll
                    for (int u = 0; u < NBW; ++u) rv[u] = wld(rsrc + gi[u]);
                    if (it > 0) {
#pragma unroll
                        for (int u = 0; u < NBW; ++u) {
                            wv[u] = wld(wsrc + gi[u]);
                            pv[u] = wld(psrc + gi[u]);
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < NBW; ++u) wv[u] = pv[u] = 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < NBW; ++u) {
                        const int li = li0 + u * wm.rs;
                        const double rj = fma(-alpha, wv[u], rv[u]);
                        const double ph = ok[u] ? fma(beta, pv[u], rj) : 0.0;
                        double *d = (lj < g.W0 && li < g.H0) ? tile + li * g.P0 + lj : tile + g.offT + threadIdx.x;
                        *d = ph;
                        if (ok[u] && own[u]) {
                            if (it > 0) rdst[gi[u]] = rj;
                            if (LZ && it < Y.nlz) gp(Y.lz)[it * Y.ldw + gi[u]] = rj;   // Lanczos capture of r_j
                            pdst[gi[u]] = ph;
                            const int ii = (li - g.hy) * g.PE + (lj - g.hx);
                            pbuf[ii] = ph;
                            rbuf[ii] = rj;
                        }
                    }
                }
                __syncthreads();
                if (item == lo) stamp(it, 6);
                tile_E(I, g, tile, y0, x0, gam, ew);
                tile_A(I, g, tile, taps, y0, x0, 1.0);
                if (item == lo) stamp(it, 7);
                // interior: x_j = x_{j-1} + alpha p_{j-1}; p_j = ph_j - W c_j; w_j = B ph_j - Z c_j;
                // partials p.w, r.r, r.w, w.w, Z^T r, Z^T w (all 2q basis loads of a pixel batch together)
                const double *ebuf = tile + g.offE;
                const int ne = I.ty * I.tx;
                double v[NVT];
#pragma unroll
                for (int j = 0; j < NVT; ++j) v[j] = 0.0;
                for (int base = 0; base < ne; base += NT * NBE) {
                    int gi[NBE];
                    bool ok[NBE];
#pragma unroll
                    for (int u = 0; u < NBE; ++u) {
                        const int k = base + u * NT + threadIdx.x;
                        const int gy = y0 + (k >> I.ltx), gx = x0 + (k & (I.tx - 1));
                        ok[u] = k < ne && gy < I.ny && gx < I.nx;
                        gi[u] = ok[u] ? gy * I.nx + gx : 0;
                    }
                    double wl[NBE][QT > 0 ? QT : 1], zl[NBE][QT > 0 ? QT : 1], xo[NBE], po[NBE], ro[NBE];
#pragma unroll
                    for (int u = 0; u < NBE; ++u) {
#pragma unroll
                        for (int j = 0; j < QT; ++j) {
                            wl[u][j] = (j < q && ok[u]) ? YW[j * ldw + gi[u]] : 0.0;
                            zl[u][j] = (j < q && ok[u]) ? YZ[j * ldw + gi[u]] : 0.0;
                        }
                        xo[u] = Yx[gi[u]];
                        po[u] = Ypa[gi[u]];
                        if constexpr (TWO) ro[u] = gp(Y.rb[pj])[gi[u]];   // r_j of the own cell (first pass)
                    }
#pragma unroll
                    for (int u = 0; u < NBE; ++u) {
                        const int k = base + u * NT + threadIdx.x;
                        const int ii = ok[u] ? (k >> I.ltx) : 0, jj = ok[u] ? (k & (I.tx - 1)) : 0;
                        double p = pbuf[ii * g.PE + jj];
                        double w = ebuf[ii * g.PE + jj];
                        double rj;
                        if constexpr (TWO) rj = ro[u];
                        else rj = rbuf[ii * g.PE + jj];
#pragma unroll
                        for (int j = 0; j < QT; ++j) {
                            p = fma(-s_c[j], wl[u][j], p);
                            w = fma(-s_c[j], zl[u][j], w);
                        }
                        if (ok[u]) {
                            if (it > 0) Yx[gi[u]] = fma(alpha, po[u], xo[u]);
                            Ypa[gi[u]] = p;
                            wdst[gi[u]] = w;
                            v[0] = fma(p, w, v[0]);
                            v[1] = fma(rj, rj, v[1]);
                            v[2] = fma(rj, w, v[2]);
                            v[3] = fma(w, w, v[3]);
#pragma unroll
                            for (int j = 0; j < QT; ++j) {
                                v[4 + j] = fma(zl[u][j], rj, v[4 + j]);
                                v[4 + QT + j] = fma(zl[u][j], w, v[4 + QT + j]);
                            }
                        }
                    }
                }
                if (item == lo) stamp(it, 13);
                block_accumulate<NVT>(v, NVT, s_acc, s_red);
                if (item == lo) stamp(it, 14);
            }
            if (cur_sys >= 0 && threadIdx.x < NVP)
                gp(pcur)[(int)threadIdx.x * PS + slot_of(N, mn, ipbn, cur_sys, chunk)] = s_acc[threadIdx.x];
            if (threadIdx.x == 0) s_clast = cur_sys;   // read after the barrier
        }
        stamp(it, 2);
        if (!grid_barrier<ACQ>(bc, (unsigned long long)(++nbar), A.timeout_ticks, &s_flag, &s_arr, &s_g)) return;
        stamp(it, 3);
        if (flip) cur ^= 1;
    }
}

int cg_tile_lds(int tile_lds, int msys)
{
    // the tile region doubles as the scratch of the per-iteration reduction:
    // 4 values for each of at most G + 2 msys chunk partials (G <= 1024) and 4 sums per system
    const int need = 4 * (1024 + 2 * msys) + 4 * msys;
    return tile_lds > need ? tile_lds : need;
}

size_t cg_lds_bytes(int tile_lds, int taps_lds, int msys)
{
    const size_t d = (size_t)tile_lds + taps_lds + 4 * (size_t)msys;   // tile, constants, rho, alpha, beta, tol
    const size_t ints = 2 * (size_t)(2 * msys + 2 * (msys + 1)) + 2; // two assignments
    return d * sizeof(double) + ints * sizeof(int);
}

// Compiled widths of the local space; a launch uses the smallest one >= its widest q.
// The capturing variant exists for q = 0 (a first solve) and the widest space, in
// the fused form only (captures are single systems, where fused iterations win).
static const void *cg_kernel(int qt, bool lz, int form)
{
    if (form == 3) return cg1_kernel(qt, lz);
    if (lz) return qt == 0 ? (const void *)k_cg<0, true, 0> : (const void *)k_cg<QMAX, true, 0>;
#define RSR_CG_FORM(F)                                          \
    if (form == F) {                                           \
        switch (qt) {                                          \
        case 0: return (const void *)k_cg<0, false, F>;        \
        case 3: return (const void *)k_cg<3, false, F>;        \
        case 5: return (const void *)k_cg<5, false, F>;        \
        default: return (const void *)k_cg<QMAX, false, F>;    \
        }                                                      \
    }
    RSR_CG_FORM(1)
    RSR_CG_FORM(2)
#undef RSR_CG_FORM
    switch (qt) {
    case 0: return (const void *)k_cg<0, false, 0>;
    case 3: return (const void *)k_cg<3, false, 0>;
    case 5: return (const void *)k_cg<5, false, 0>;
    default: return (const void *)k_cg<QMAX, false, 0>;
    }
}

int cg_width(int qmax)
{
    return qmax <= 0 ? 0 : qmax <= 3 ? 3 : qmax <= 5 ? 5 : QMAX;
}

int cg_max_blocks_per_cu(size_t lds, int qt, bool lz, int form)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cg_kernel(qt, lz, form), NT, lds) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_cg(const CGArgs &a, int qt, bool lz, int G, size_t lds, hipStream_t s, const SysDev *sys1)
{
    if (a.form == 3) {
        if (!sys1 && !a.sys) return hipErrorInvalidValue;
        SysDev none{};   // unused when a.sys is given
        void *args[] = {(void *)&a, (void *)(sys1 ? sys1 : &none)};
        return hipLaunchCooperativeKernel(cg_kernel(qt, lz, a.form), dim3(G), dim3(NT), args, (unsigned)lds, s);
    }
    void *args[] = {(void *)&a};
    return hipLaunchCooperativeKernel(cg_kernel(qt, lz, a.form), dim3(G), dim3(NT), args, (unsigned)lds, s);
}

}  // namespace rsr
