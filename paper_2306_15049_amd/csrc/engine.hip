// Host engine and C ABI of the recycled shifted solver.
//
// Per outer step k the caller sets W_k (rsr_update_weights /
// rsr_weights_from_image), the principal recycle space U_k
// (rsr_set_recycle_space: Algorithm 1 plus the products A U, E U and their
// small Gram blocks, Sections 4.1 and 5.3), and solves the shift set
// (rsr_solve_shift_set).  A solve
//   1. takes an initial guess from U_k: x0 = U q with q minimising
//      ||b - (AU + gamma EU) q|| (Section 4.1, eq. orthupdate), all from the
//      cached Gram blocks -- no operator application per shift;
//   2. builds each system's local space W = [Ritz block, g^(k-1,l), g^(k,l-1)]
//      (Algorithms 2-4), Z = B W from the cached A U, E U plus one A and one E
//      application per correction column, and applies the Galerkin correction
//      x0 += W G^{-1} W^T r0 (G = W^T Z);
//   3. runs deflated CG for every system in one persistent launch;
//   4. accepts on the recomputed true residual, restarting if needed, and keeps
//      the correction g = x - x0 for the next shift / outer step.
#include "internal.hpp"
#include "outer.hpp"
#include "smalldense.hpp"
#include "../../include/rsr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <future>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

using namespace rsr;

namespace {

struct Err {
    rsr_status st;
    std::string msg;
};

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            throw Err{e_ == hipErrorOutOfMemory ? RSR_E_NOMEM : RSR_E_HIP,                         \
                      std::string(#expr) + ": " + hipGetErrorString(e_)};                         \
    } while (0)

void fail(rsr_status st, const std::string &m) { throw Err{st, m}; }

// Scratch of rsr_solve_shift_set_noalloc: one array per device, mapped when the
// code object loads (no allocation by the library).  In host code the name is a
// host-side stand-in; kernels get the device address from hipGetSymbolAddress,
// taken once per device in rsr_create and kept in g_scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

// Device and pinned allocations made by the library (all contexts), for checks
// that a call allocated nothing.
std::atomic<long long> g_alloc_calls{0};

// Grow-only device buffer.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void ensure(size_t b)
    {
        if (b <= bytes) return;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        size_t nb = std::max(b, (size_t)256);
        g_alloc_calls.fetch_add(1);
        HIPCHK(hipMalloc(&p, nb));
        bytes = nb;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return (T *)p; }
};

struct Instance {
    int ny = 0, nx = 0, sy = 1, sx = 1;
    long n = 0;
    std::vector<double> psf;
    int sep = 0;                       // stencil path: 1 banded separable (rank 1), 2 rank-R sum, 0 direct
    int sep_ok = 0;                    // the PSF is rank 1 (the banded factors exist)
    int rank = 0;                      // rank of the PSF when 2..RMAX (the rank-R factors exist), else 0
    std::vector<double> rk;            // rank-R factors, per term [fy reversed][fx reversed][fy][fx]
    int form = -1;                     // tuned persistent-CG iteration form (-1: by launch size)
    int ssq = 0;                       // separable path: zero-padded square size
    std::vector<double> fy, fx;
    std::vector<double> band;          // banded factors of K^T K (separable path), see band_tables
    DBuf d_fy, d_fx, d_psf, d_wh, d_wv, d_band, d_rk;
    int ty = 16, tx = 16;
    // tomography instance (rsr_set_ct_operators): projector geometry and scale
    bool ct = false;
    int na = 0, nd = 0;
    double spacing = 1.0, ct_scale = 1.0;
    DBuf d_cs;                         // [na][4] cos, sin, 1/(-sin), 1/cos
    // principal recycle space
    int p = 0;
    DBuf d_U, d_AE;   // U: p columns; AE: [AU | EU], 2p columns; stride n
    std::vector<double> Ahat, Ehat, Gaa, Gae, Gee;   // p x p row-major
    bool ae_valid = false;
    // latest correction g = x - x0 per shift slot: column gcol[slot] of gpool
    // (one allocation for all slots, grown geometrically when a slot is new)
    std::map<int, int> gcol;
    DBuf gpool;
    int gpool_cols = 0;
    double *gslot(int slot)
    {
        auto it = gcol.find(slot);
        return it == gcol.end() ? nullptr : gpool.as<double>() + (size_t)it->second * n;
    }
    // Ritz blocks [R | AR | ER] per shift group, valid for the current U (version)
    long u_version = 0;
    struct RitzBlock {
        long version = -1;
        double gamma = 0.0;
        int nr = 0;
        DBuf buf;
    } ritz[2];
    // eigenpairs of Ahat + gamma Ehat for the current U: the retained Ritz
    // vectors of the next principal space, computed on the host while a CG
    // launch runs (the first launch after U changes, at its smallest shift)
    struct EigPre {
        long version = -1;
        double gamma = 0.0;
        std::vector<double> w, V;
    } eig_pre;
};

inline int eff_sy(const Instance &I) { return I.sep == 1 ? I.ssq : I.sy; }
inline int eff_sx(const Instance &I) { return I.sep == 1 ? I.ssq : I.sx; }

}  // namespace

struct rsr_ctx {
    int dev = 0;
    int n_cu = 256;
    double wall_khz = 100000.0;
    std::string err;
    std::vector<std::unique_ptr<Instance>> inst;
    DBuf d_inst;                       // InstDev[n_inst]
    std::vector<InstDev> h_inst;
    // scratch
    DBuf d_jobs, d_gram_scratch, d_small, d_sys, d_partA, d_partB, d_ctl, d_out;
    DBuf d_ws;                         // per-system vectors of a solve
    DBuf d_dbg;                        // optional phase timestamps
    DBuf d_tmp;                        // grouped initial guesses x0, r0 before they are copied out
    DBuf d_rcC, d_rcQ, d_rcR, d_rcT;   // recycle-space candidates, their orthonormal basis, the projected
                                       // residual block and a staging block (kept: no
                                       // allocation, and no free that drains the device, per update)
    DBuf d_lz, d_lzc, d_lzr;           // CG-Lanczos capture (residuals, coefficients) and its Ritz vectors
    DBuf d_aux;                        // workgroup partials of the edge-weight and L-curve reductions
    DBuf d_corr;                       // right-hand side of the correction equation
    DBuf d_r0sq;                       // ||r0||^2 per system of a solve call, read back at its end
    DBuf d_grad;                       // gradient partials, shifts and scratch weight planes of rsr_adjoint
    // staging arena for launch descriptors and coefficients: pinned host and
    // device halves bump-allocated in step, reset whenever the stream is drained,
    // so that launches whose inputs come from the host need no synchronisation
    DBuf ar_dev;
    char *ar_host = nullptr;
    size_t ar_cap = 0, ar_used = 0;
    // pinned host buffer that every device-to-host read-back lands in (no copy
    // into pageable memory is left to the runtime's staging)
    char *rb_host = nullptr;
    size_t rb_cap = 0;
    // caller workspace of the current call (null base: the library's own grow-only
    // buffers).  Device scratch is carved from it with a stack discipline (see
    // WsMark); host data bound for the device is kept until the stream is drained,
    // and read-backs go to ordinary host memory, so a call on a workspace
    // allocates no device or pinned memory.
    char *wsa_base = nullptr;
    size_t wsa_cap = 0, wsa_used = 0, wsa_peak = 0;
    std::vector<std::vector<char>> wsa_hold;
    // per-call caches of right-hand-side quantities shared by the shifts of one
    // rsr_solve_shift_set (the same b for every shift): ||b|| and U^T b or
    // [AU EU]^T b, keyed by (b, instance, init); cleared at the start of each call
    std::map<std::pair<const double *, int>, double> bnorm_cache;
    std::map<std::tuple<const double *, int, int>, std::vector<double>> rhs_cache;
    // optional host-side stage timing of the solves (diagnostics, RSR_HOST_PROF)
    bool hprof = false;
    double hprof_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // counters and timing
    long mv_A = 0, mv_E = 0;
    int cg_gmax = 1024;                // cap on persistent-kernel workgroups (autotuned)
    double bar_timeout_s = 30.0;       // bound on one grid-barrier wait (RSR_BARRIER_TIMEOUT_US)
    int cg_mode = 0;                   // persistent-CG iteration form: 0 by launch size, else form + 1
    void *scratch_dev = nullptr;       // this device's address of the static no-allocation scratch
    double last_cg_ms = 0.0;
    int last_launches = 0;
    long last_items = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // tomography instances: every instance of the context is one (rsr_set_ct_operators)
    bool ct = false;
    DBuf d_ctinst;                     // CtDev[n_inst]
    std::vector<CtDev> h_ct;
    DBuf d_ct_sino;                    // sinogram scratch of K^T K applications
};

namespace {

hipStream_t S(void *s) { return (hipStream_t)s; }

void set_device(rsr_ctx *c) { HIPCHK(hipSetDevice(c->dev)); }

Instance &get_inst(rsr_ctx *c, int i)
{
    if (c->inst.empty()) fail(RSR_E_STATE, "operators not set");
    if (i < 0 || i >= (int)c->inst.size()) fail(RSR_E_ARG, "instance index out of range");
    return *c->inst[i];
}

void upload_inst(rsr_ctx *c)
{
    c->h_inst.resize(c->inst.size());
    for (size_t i = 0; i < c->inst.size(); ++i) {
        Instance &I = *c->inst[i];
        InstDev &d = c->h_inst[i];
        d.ny = I.ny;
        d.nx = I.nx;
        d.ty = I.ty;
        d.tx = I.tx;
        d.lty = __builtin_ctz((unsigned)I.ty);
        d.ltx = __builtin_ctz((unsigned)I.tx);
        d.nty = (I.ny + I.ty - 1) / I.ty;
        d.ntx = (I.nx + I.tx - 1) / I.tx;
        d.sep = I.sep;
        d.rank = I.sep == 2 ? I.rank : 0;
        d.rsv = 0;
        d.sy = eff_sy(I);
        d.sx = eff_sx(I);
        d.fy = I.d_fy.as<double>();
        d.fx = I.d_fx.as<double>();
        d.band = I.sep == 2 ? I.d_rk.as<double>() : I.d_band.as<double>();
        d.psf = I.d_psf.as<double>();
        d.wh = I.d_wh.as<double>();
        d.wv = I.d_wv.as<double>();
    }
    c->d_inst.ensure(sizeof(InstDev) * std::max<size_t>(1, c->h_inst.size()));
    HIPCHK(hipMemcpy(c->d_inst.p, c->h_inst.data(), sizeof(InstDev) * c->h_inst.size(), hipMemcpyHostToDevice));
    if (c->ct) {
        c->h_ct.resize(c->inst.size());
        for (size_t i = 0; i < c->inst.size(); ++i) {
            Instance &I = *c->inst[i];
            c->h_ct[i] = CtDev{I.ny, I.nx, I.na, I.nd, I.spacing, I.ct_scale, I.d_cs.as<double>(),
                               I.d_wh.as<double>(), I.d_wv.as<double>()};
        }
        c->d_ctinst.ensure(sizeof(CtDev) * c->h_ct.size());
        HIPCHK(hipMemcpy(c->d_ctinst.p, c->h_ct.data(), sizeof(CtDev) * c->h_ct.size(), hipMemcpyHostToDevice));
    }
}

// Upload a host array through the job buffer region starting at byte offset.
template <class T> T *upload(rsr_ctx *c, DBuf &buf, const std::vector<T> &v, hipStream_t s)
{
    buf.ensure(sizeof(T) * std::max<size_t>(1, v.size()));
    if (!v.empty()) HIPCHK(hipMemcpyAsync(buf.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return buf.as<T>();
}

// Drains the stream; the staging arena can then be reused from the start.
void sync(rsr_ctx *c, hipStream_t s)
{
    HIPCHK(hipStreamSynchronize(s));
    c->ar_used = 0;
    c->wsa_hold.clear();
}

// Device scratch of a call: from the caller's workspace when the call has one,
// else from the library-owned buffer `own` (grown as needed).
void *dscratch(rsr_ctx *c, DBuf &own, size_t bytes)
{
    if (!c->wsa_base) {
        own.ensure(bytes);
        return own.p;
    }
    const size_t off = (c->wsa_used + 255) & ~(size_t)255;
    if (off + bytes > c->wsa_cap)
        fail(RSR_E_ARG, "workspace of " + std::to_string(c->wsa_cap) + " bytes is too small (this call needs more than " +
                            std::to_string(off + bytes) + "); size it with rsr_workspace_size");
    c->wsa_used = off + bytes;
    c->wsa_peak = std::max(c->wsa_peak, c->wsa_used);
    return c->wsa_base + off;
}

// Scratch taken from the caller's workspace inside a scope is handed back when
// the scope ends.  Work already enqueued that reads it runs before any later
// work that reuses it (one stream), so only the host side is released early.
struct WsMark {
    rsr_ctx *c;
    size_t used;
    explicit WsMark(rsr_ctx *c_) : c(c_), used(c_->wsa_used) {}
    ~WsMark() { c->wsa_used = used; }
};

// Wall time of a solve stage, accumulated when stage timing is on (the stream
// is drained at both ends so that the device work of the stage is included).
struct StageTimer {
    rsr_ctx *c;
    hipStream_t s;
    int k;
    std::chrono::steady_clock::time_point t0;
    StageTimer(rsr_ctx *c_, hipStream_t s_, int k_) : c(c_), s(s_), k(k_)
    {
        if (c->hprof) {
            sync(c, s);
            t0 = std::chrono::steady_clock::now();
        }
    }
    ~StageTimer()
    {
        if (c->hprof) {
            (void)hipStreamSynchronize(s);
            c->hprof_ms[k] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    }
};

// Reserves nb bytes of the staging arena (pinned host half h, device half d),
// draining the stream first when the arena is full.
void arena_reserve(rsr_ctx *c, size_t nb, hipStream_t s, char *&h, char *&d)
{
    const size_t bytes = (std::max<size_t>(nb, 1) + 255) & ~(size_t)255;
    if (c->wsa_base) {
        // host half: ordinary memory kept until the stream is drained; device half
        // from the workspace
        c->wsa_hold.emplace_back(bytes);
        h = c->wsa_hold.back().data();
        d = (char *)dscratch(c, c->ar_dev, bytes);
        return;
    }
    if (c->ar_used + bytes > c->ar_cap) {
        sync(c, s);
        if (bytes > c->ar_cap) {
            const size_t cap = std::max<size_t>(bytes, (size_t)1 << 20);
            if (c->ar_host) (void)hipHostFree(c->ar_host);
            c->ar_host = nullptr;
            c->ar_cap = 0;
            g_alloc_calls.fetch_add(1);
            HIPCHK(hipHostMalloc((void **)&c->ar_host, cap, hipHostMallocDefault));
            c->ar_dev.ensure(cap);
            c->ar_cap = cap;
        }
    }
    h = c->ar_host + c->ar_used;
    d = c->ar_dev.as<char>() + c->ar_used;
    c->ar_used += bytes;
}

// Copies v into the staging arena (pinned host -> device, asynchronous) and
// returns its device address, valid until the next sync().
template <class T> T *stage(rsr_ctx *c, const std::vector<T> &v, hipStream_t s)
{
    const size_t nb = sizeof(T) * v.size();
    char *h, *d;
    arena_reserve(c, nb, s, h, d);
    if (nb) {
        memcpy(h, v.data(), nb);
        HIPCHK(hipMemcpyAsync(d, h, nb, hipMemcpyHostToDevice, s));
    }
    return (T *)d;
}

// Device-to-host read-backs: the listed copies land in the pinned read-back
// buffer, the stream is drained, and the bytes are copied out to dst.
struct ReadBack {
    void *dst;
    const void *src;
    size_t bytes;
};
void read_back(rsr_ctx *c, const std::vector<ReadBack> &v, hipStream_t s)
{
    if (c->wsa_base) {   // no pinned buffer is allocated for a call on a workspace
        for (const auto &r : v)
            if (r.bytes) HIPCHK(hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToHost, s));
        sync(c, s);
        return;
    }
    size_t tot = 0;
    for (const auto &r : v) tot += (r.bytes + 15) & ~(size_t)15;
    if (tot > c->rb_cap) {
        sync(c, s);
        if (c->rb_host) (void)hipHostFree(c->rb_host);
        c->rb_host = nullptr;
        c->rb_cap = 0;
        const size_t cap = std::max<size_t>(tot, (size_t)1 << 16);
        g_alloc_calls.fetch_add(1);
        HIPCHK(hipHostMalloc((void **)&c->rb_host, cap, hipHostMallocDefault));
        c->rb_cap = cap;
    }
    size_t o = 0;
    for (const auto &r : v) {
        if (r.bytes) HIPCHK(hipMemcpyAsync(c->rb_host + o, r.src, r.bytes, hipMemcpyDeviceToHost, s));
        o += (r.bytes + 15) & ~(size_t)15;
    }
    sync(c, s);
    o = 0;
    for (const auto &r : v) {
        if (r.bytes) memcpy(r.dst, c->rb_host + o, r.bytes);
        o += (r.bytes + 15) & ~(size_t)15;
    }
}

int max_tile_lds(rsr_ctx *c)
{
    int m = 2048;
    for (auto &p : c->inst) m = std::max(m, tile_lds_doubles(p->ty, p->tx, eff_sy(*p), eff_sx(*p), p->sep));
    return m;
}

int max_taps_lds(rsr_ctx *c)
{
    int m = 0;
    for (auto &p : c->inst) m = std::max(m, taps_lds_doubles(eff_sy(*p), p->sep));
    return m;
}

// LDS of the one-tile apply kernel: the tile buffers, then the instance's constants
size_t apply_lds_bytes(const Instance &I)
{
    return sizeof(double) * (tile_lds_doubles(I.ty, I.tx, eff_sy(I), eff_sx(I), I.sep) + taps_lds_doubles(eff_sy(I), I.sep));
}

// ----------------------------------------------------------- operators --
// Projector applications of tomography instances: one forward launch (the
// sinograms K v of the jobs that need them, into scratch or the output) and
// one backward launch (K^T of those sinograms, plus cE E v) for the batch.
void ct_apply_jobs(rsr_ctx *c, const std::vector<ApplyJob> &jobs, hipStream_t s)
{
    if (jobs.empty()) return;
    WsMark mark(c);
    size_t need = 0;
    for (const auto &j : jobs) {
        const Instance &I = *c->inst[j.inst];
        if (j.op == 0 && j.cA != 0.0) need += (size_t)I.na * I.nd;
    }
    double *sino = (double *)dscratch(c, c->d_ct_sino, sizeof(double) * std::max<size_t>(1, need));
    std::vector<CtJob> cj;
    size_t o = 0;
    int max_rays = 1;
    long max_px = 1;
    for (const auto &j : jobs) {
        const Instance &I = *c->inst[j.inst];
        CtJob t{j.inst, j.op, j.cA, j.cE, j.v, j.y, nullptr};
        if (j.op == 0 && j.cA != 0.0) {
            t.sino = sino + o;
            o += (size_t)I.na * I.nd;
        }
        cj.push_back(t);
        max_rays = std::max(max_rays, I.na * I.nd);
        max_px = std::max(max_px, I.n);
        if (j.op == 0 && j.cA != 0.0) c->mv_A++;
        if (j.op == 0 && j.cE != 0.0) c->mv_E++;
    }
    CtJob *dj = stage(c, cj, s);
    HIPCHK(launch_ct_fwd(c->d_ctinst.as<CtDev>(), dj, (int)cj.size(), max_rays, s));
    HIPCHK(launch_ct_back(c->d_ctinst.as<CtDev>(), dj, (int)cj.size(), max_px, s));
}

// y_j = cA A v_j + cE E v_j for nvec vectors of one instance.
void apply_op(rsr_ctx *c, int ii, double cA, double cE, const double *v, long ldv, double *y, long ldy,
              int nvec, hipStream_t s, DBuf *jobbuf = nullptr)
{
    if (nvec <= 0) return;
    Instance &I = get_inst(c, ii);
    std::vector<ApplyJob> jobs(nvec);
    for (int j = 0; j < nvec; ++j) jobs[j] = ApplyJob{ii, 0, cA, cE, v + j * ldv, y + j * ldy};
    if (I.ct) {
        ct_apply_jobs(c, jobs, s);
        return;
    }
    // up to KJ jobs travel in the kernel arguments
    ApplyJob *dj = nvec <= KJ ? nullptr : jobbuf ? upload(c, *jobbuf, jobs, s) : stage(c, jobs, s);
    const size_t lds = apply_lds_bytes(I);
    HIPCHK(launch_apply(c->d_inst.as<InstDev>(), c->h_inst[ii], dj, jobs.data(), nvec, lds, s));
    if (cA != 0.0) c->mv_A += nvec;
    if (cE != 0.0) c->mv_E += nvec;
}

void apply_jobs(rsr_ctx *c, std::vector<ApplyJob> &jobs, hipStream_t s)
{
    if (c->ct) {
        ct_apply_jobs(c, jobs, s);
        return;
    }
    WsMark mark(c);
    // group by instance (one launch per instance)
    std::map<int, std::vector<ApplyJob>> by;
    for (auto &j : jobs) by[j.inst].push_back(j);
    for (auto &kv : by) {
        Instance &I = get_inst(c, kv.first);
        const int nj = (int)kv.second.size();
        ApplyJob *dj = nj <= KJ ? nullptr : stage(c, kv.second, s);
        const size_t lds = apply_lds_bytes(I);
        HIPCHK(launch_apply(c->d_inst.as<InstDev>(), c->h_inst[kv.first], dj, kv.second.data(), nj, lds, s));
        for (auto &j : kv.second) {
            if (j.cA != 0.0) c->mv_A++;
            if (j.cE != 0.0) c->mv_E++;
        }
    }
}

// C_j = X_j^T Y_j for a list of jobs; results copied to host (row-major a x c each).
std::vector<std::vector<double>> gram(rsr_ctx *c, std::vector<GramJob> jobs, hipStream_t s)
{
    std::vector<std::vector<double>> out(jobs.size());
    if (jobs.empty()) return out;
    WsMark mark(c);
    size_t coff = 0;
    for (auto &j : jobs) coff += (size_t)j.a * j.c;
    double *small = (double *)dscratch(c, c->d_small, sizeof(double) * std::max<size_t>(1, coff));
    size_t o = 0, sc = 0;
    for (auto &j : jobs) {
        j.C = small + o;
        o += (size_t)j.a * j.c;
        j.sc_off = (long)sc;
        sc += gram_scratch_doubles(&j, 1);
    }
    double *gsc = (double *)dscratch(c, c->d_gram_scratch, sizeof(double) * std::max<size_t>(1, sc));
    GramJob *dj = jobs.size() <= (size_t)KJ ? nullptr : stage(c, jobs, s);
    HIPCHK(launch_gram(dj, jobs.data(), (int)jobs.size(), gsc, sc, s));
    std::vector<double> h(coff);
    read_back(c, {ReadBack{h.data(), small, sizeof(double) * coff}}, s);
    o = 0;
    for (size_t k = 0; k < jobs.size(); ++k) {
        out[k].assign(h.begin() + o, h.begin() + o + (size_t)jobs[k].a * jobs[k].c);
        o += (size_t)jobs[k].a * jobs[k].c;
    }
    return out;
}

// X^T Y products written to device memory (each job's C set by the caller),
// with no read-back: for results the host needs only at the end of a call.
void gram_to_device(rsr_ctx *c, std::vector<GramJob> jobs, hipStream_t s)
{
    if (jobs.empty()) return;
    WsMark mark(c);
    size_t sc = 0;
    for (auto &j : jobs) {
        j.sc_off = (long)sc;
        sc += gram_scratch_doubles(&j, 1);
    }
    double *gsc = (double *)dscratch(c, c->d_gram_scratch, sizeof(double) * std::max<size_t>(1, sc));
    GramJob *dj = jobs.size() <= (size_t)KJ ? nullptr : stage(c, jobs, s);
    HIPCHK(launch_gram(dj, jobs.data(), (int)jobs.size(), gsc, sc, s));
}

// Y_j = beta Y_j + X_j Q_j (Q from host, column-major a x c with ldq = a).
void combo(rsr_ctx *c, std::vector<ComboJob> jobs, const std::vector<std::vector<double>> &Qs, hipStream_t s)
{
    if (jobs.empty()) return;
    WsMark mark(c);
    size_t tot = 0;
    for (auto &q : Qs) tot += q.size();
    bool inl = jobs.size() <= (size_t)KJ && tot <= (size_t)KQ;
    for (size_t k = 0; inl && k < jobs.size(); ++k) {
        const size_t nq = (size_t)jobs[k].a * jobs[k].c;
        inl = Qs[k].size() == nq && (nq == 0 || jobs[k].ldq == jobs[k].a);
    }
    if (inl) {
        // descriptors and coefficients in the kernel arguments: no upload
        std::vector<const double *> qp(jobs.size());
        for (size_t k = 0; k < jobs.size(); ++k) qp[k] = Qs[k].data();
        HIPCHK(launch_combo(nullptr, jobs.data(), (int)jobs.size(), s, qp.data()));
        return;
    }
    // coefficients and descriptors in one upload: [Q_0 Q_1 ... | jobs]
    const size_t nq = sizeof(double) * tot;
    const size_t offj = (nq + 15) & ~(size_t)15;
    const size_t nj = sizeof(ComboJob) * jobs.size();
    char *h, *d;
    arena_reserve(c, offj + nj, s, h, d);
    size_t o = 0;
    for (size_t k = 0; k < jobs.size(); ++k) {
        if (!Qs[k].empty()) memcpy(h + sizeof(double) * o, Qs[k].data(), sizeof(double) * Qs[k].size());
        jobs[k].Q = (const double *)d + o;
        o += Qs[k].size();
    }
    memcpy(h + offj, jobs.data(), nj);
    HIPCHK(hipMemcpyAsync(d, h, offj + nj, hipMemcpyHostToDevice, s));
    HIPCHK(launch_combo((const ComboJob *)(d + offj), jobs.data(), (int)jobs.size(), s));
}

// Runs fn(i) for i in [0, n) on up to nt host threads, the calling thread
// included (the small dense solves of independent shifts and groups).  Each i
// is computed the same way whichever thread takes it.
template <class F> void parallel_for(int n, int nt, F fn)
{
    nt = std::max(1, std::min(nt, n));
    if (nt == 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::future<void>> fut;
    for (int t = 1; t < nt; ++t)
        fut.push_back(std::async(std::launch::async, [&fn, n, nt, t] {
            for (int i = t; i < n; i += nt) fn(i);
        }));
    std::exception_ptr err;
    try {
        for (int i = 0; i < n; i += nt) fn(i);
    } catch (...) {
        err = std::current_exception();
    }
    for (auto &f : fut) {
        try {
            f.get();
        } catch (...) {
            if (!err) err = std::current_exception();
        }
    }
    if (err) std::rethrow_exception(err);
}
constexpr int HOST_THREADS = 4;

// Eigenpairs (ascending) of Ahat + gamma Ehat for the instance's current U,
// from the cache when it holds this U version and shift.
void retained_eig(Instance &I, double gamma, std::vector<double> &w, std::vector<double> &V)
{
    auto &E = I.eig_pre;
    if (E.version == I.u_version && E.gamma == gamma && (int)E.w.size() == I.p) {
        w = E.w;
        V = E.V;
        return;
    }
    const int p = I.p;
    std::vector<double> H((size_t)p * p);
    for (size_t k = 0; k < H.size(); ++k) H[k] = I.Ahat[k] + gamma * I.Ehat[k];
    sym_eig(p, H.data(), w, V);
    E.version = I.u_version;
    E.gamma = gamma;
    E.w = w;
    E.V = V;
}

// dst_k = src_k for a list of vectors, in one launch (a combination with the
// single coefficient 1, which reproduces every finite value exactly)
struct CopyJob {
    const double *src;
    double *dst;
    long n;
};
void copy_many(rsr_ctx *c, const std::vector<CopyJob> &v, hipStream_t s)
{
    if (v.empty()) return;
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    for (const auto &j : v) {
        cj.push_back(ComboJob{j.src, j.n, 1, nullptr, 1, j.dst, j.n, 1, 0.0, nullptr, 0, j.n});
        qs.push_back(std::vector<double>{1.0});
    }
    combo(c, cj, qs, s);
}

std::vector<double> norms(rsr_ctx *c, const std::vector<const double *> &v, const std::vector<long> &n,
                          hipStream_t s)
{
    std::vector<GramJob> jobs;
    for (size_t i = 0; i < v.size(); ++i) jobs.push_back(GramJob{v[i], n[i], 1, v[i], n[i], 1, n[i], nullptr, 0});
    auto r = gram(c, jobs, s);
    std::vector<double> out(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        const double t = r[i][0];
        out[i] = std::isnan(t) ? t : std::sqrt(std::max(0.0, t));   // a NaN must not read as a zero norm
    }
    return out;
}

// ---------------------------------------------------------- PSF factors --
// Banded form of T^T T for the zero-boundary "same" 1-D convolution
// (T v)[k] = sum_c f[c] v[k + r - c] (S = 2r + 1 taps; row factor of K along x,
// column factor along y; K^T K = (Ty^T Ty) (x) (Tx^T Tx)).  Summing over every
// k gives the Toeplitz part c(s) = sum_m f[m] f[m + s]; restricting k to the
// line removes, for outputs and inputs both among the first r positions,
//   Lc[j][i] = sum_{u = max(i,j)}^{r-1} f[u - j] f[u - i]     (k < 0), and for
// the last r positions (j = n - r + p, i = n - r + q)
//   Rc[p][q] = sum_{u = 0}^{min(p,q)} f[u + 2r - p] f[u + 2r - q]   (k >= n).
// So (T^T T v)[j] = sum_{t=0}^{4r} c(2r - t) v[j - 2r + t] - [j < r] (Lc v)[j]
// - [j >= n - r] (Rc v)[j - n + r], with v = 0 outside the line.
// Layout of I.band: [band x: 4r+1][band y: 4r+1][Lx: r*r][Rx: r*r][Ly: r*r][Ry: r*r].
void band_tables(Instance &I)
{
    const int S = I.ssq, r = S / 2, nb = 4 * r + 1, rr = r * r;
    I.band.assign(2 * nb + 4 * rr, 0.0);
    const std::vector<double> *fs[2] = {&I.fx, &I.fy};
    for (int ax = 0; ax < 2; ++ax) {
        const std::vector<double> &f = *fs[ax];
        double *band = I.band.data() + ax * nb;
        double *Lc = I.band.data() + 2 * nb + (2 * ax) * rr;
        double *Rc = Lc + rr;
        for (int t = 0; t < nb; ++t) {
            const int sh = 2 * r - t;
            double c = 0.0;
            for (int m = 0; m < S; ++m)
                if (m + sh >= 0 && m + sh < S) c += f[m] * f[m + sh];
            band[t] = c;
        }
        for (int j = 0; j < r; ++j)
            for (int i = 0; i < r; ++i) {
                double l = 0.0, q = 0.0;
                for (int u = std::max(i, j); u < r; ++u) l += f[u - j] * f[u - i];
                for (int u = 0; u <= std::min(i, j); ++u) q += f[u + 2 * r - j] * f[u + 2 * r - i];
                Lc[j * r + i] = l;
                Rc[j * r + i] = q;
            }
    }
}

void factor_psf(Instance &I)
{
    // rank-1 test: h = fy fx^T iff h equals the outer product built from its
    // largest entry's row and column.
    const int sy = I.sy, sx = I.sx;
    int am = 0, cm = 0;
    double best = -1.0, nrm = 0.0;
    for (int a = 0; a < sy; ++a)
        for (int c2 = 0; c2 < sx; ++c2) {
            const double v = std::fabs(I.psf[a * sx + c2]);
            nrm += v * v;
            if (v > best) { best = v; am = a; cm = c2; }
        }
    I.sep = 0;
    I.sep_ok = 0;
    I.rank = 0;
    I.rk.clear();
    if (best <= 0.0 || sx > MAXS || sy > MAXS) return;
    const double piv = I.psf[am * sx + cm];
    std::vector<double> fy(sy), fx(sx);
    const double sc = std::sqrt(std::fabs(piv));
    for (int a = 0; a < sy; ++a) fy[a] = I.psf[a * sx + cm] / sc;
    for (int c2 = 0; c2 < sx; ++c2) fx[c2] = I.psf[am * sx + c2] / sc * (piv < 0 ? -1.0 : 1.0);
    double err = 0.0;
    for (int a = 0; a < sy; ++a)
        for (int c2 = 0; c2 < sx; ++c2) {
            const double d = I.psf[a * sx + c2] - fy[a] * fx[c2];
            err += d * d;
        }
    if (err > 1e-28 * nrm) {
        // a sum of R <= RMAX separable terms: h = sum_k s_k u_k v_k^T from the SVD of
        // the PSF (the singular values past the rank vanish to rounding); each term
        // is split as fy_k = sqrt(s_k) u_k, fx_k = sqrt(s_k) v_k
        std::vector<double> sv, Ul;
        left_svd_jacobi(sy, sx, I.psf.data(), sv, Ul);
        int R = 0;
        while (R < (int)sv.size() && sv[R] > 1e-13 * sv[0]) ++R;
        if (R >= 2 && R <= RMAX) {
            std::vector<double> f((size_t)R * 2 * (sy + sx));
            double e2 = 0.0;
            std::vector<double> rec((size_t)sy * sx, 0.0);
            for (int k = 0; k < R; ++k) {
                double *fyr = f.data() + (size_t)k * 2 * (sy + sx), *fxr = fyr + sy, *fyk = fxr + sx, *fxk = fyk + sy;
                const double sq = std::sqrt(sv[k]);
                for (int a = 0; a < sy; ++a) fyk[a] = Ul[(size_t)k * sy + a] * sq;
                for (int c2 = 0; c2 < sx; ++c2) {   // v_k = h^T u_k / s_k
                    double t = 0.0;
                    for (int a = 0; a < sy; ++a) t += I.psf[a * sx + c2] * Ul[(size_t)k * sy + a];
                    fxk[c2] = t / sq;
                }
                for (int a = 0; a < sy; ++a) fyr[a] = fyk[sy - 1 - a];
                for (int c2 = 0; c2 < sx; ++c2) fxr[c2] = fxk[sx - 1 - c2];
                for (int a = 0; a < sy; ++a)
                    for (int c2 = 0; c2 < sx; ++c2) rec[(size_t)a * sx + c2] += fyk[a] * fxk[c2];
            }
            for (size_t t = 0; t < rec.size(); ++t) e2 += (rec[t] - I.psf[t]) * (rec[t] - I.psf[t]);
            if (e2 <= 1e-28 * nrm) {
                I.rank = R;
                I.rk = f;
                I.sep = 2;
            }
        }
        return;
    }
    if (err <= 1e-28 * nrm) {
        // zero-pad both factors symmetrically to one odd square size: zero taps add
        // exact zeros, so the operator is unchanged and one compiled pass width serves
        // both directions
        const int S = std::max(sy, sx);
        I.sep = 1;
        I.sep_ok = 1;
        I.ssq = S;
        I.fy.assign(S, 0.0);
        I.fx.assign(S, 0.0);
        for (int a = 0; a < sy; ++a) I.fy[(S - sy) / 2 + a] = fy[a];
        for (int c2 = 0; c2 < sx; ++c2) I.fx[(S - sx) / 2 + c2] = fx[c2];
        band_tables(I);
    }
}

void default_tile(Instance &I)
{
    const long n = I.n;
    if (n <= 512L * 512L) { I.ty = 16; I.tx = 16; }
    else { I.ty = 32; I.tx = 32; }
}

// ------------------------------------------------------ persistent CG --
struct SysHost {
    int inst;
    int slot;
    int shift = 0;             // shift index l of the system (its group: l < split_I is the left group)
    int fwd_slot = -1;         // adjoint systems: the slot of the forward solve of the same shift
    double gamma;
    long n;
    const double *b;
    double *x;
    double *r, *r1, *p0, *p1, *w, *w1, *xinit, *rt, *pa;   // workspace vectors (r, w, p ping-pong in CG)
    double *cbuf;                             // [2][QMAX]
    double *W, *Z;                            // QMAX columns each
    int q = 0;
    std::vector<double> Ginv;                 // q x q
    double bnorm = 0.0;
    int iters = 0, restarts = 0, mvA = 0, mvE = 0, status = 0;
    double relres_init = 0.0, relres_true = 0.0;
    double *r0sq_dev = nullptr;   // when set, ||r0||^2 lands here and relres_init is filled in later
    bool done = false;
    // CG-Lanczos capture of the first launch (principal-space seeding)
    double *lz = nullptr, *lzc = nullptr;
    long nlz = 0;
    int lz_its = 0;            // iterations of the captured launch
};

struct Opts {
    double tol;
    int maxit;
    int init;
    int n_ritz;
    int use_prev_k;
    int use_prev_shift;
    int split_I;
    double gJL, gJR;
    int solver = RSR_SOLVER_CG;
};

// Launch shape of the persistent CG kernel for m systems of px pixels and
// `tiles` tiles in all, widest local space qmax.
struct CgLaunch {
    int qt, form, G, msys, tl, taps;
    size_t lds;
};
CgLaunch cg_config(rsr_ctx *c, int m, int qmax, bool lz, long px, long tiles, int tuned_form = -1, int tile_px = 0,
                   bool allow_one = true)
{
    CgLaunch L;
    L.msys = (m + 7) & ~7;
    L.tl = cg_tile_lds(max_tile_lds(c), L.msys);
    L.taps = max_taps_lds(c);
    L.lds = cg_lds_bytes(L.tl, L.taps, L.msys);
    L.qt = lz && qmax > 0 ? QMAX : cg_width(qmax);
    // Iteration forms.  Small launches keep their own data in the L2 from one
    // iteration to the next and read other workgroups' cells with coherent
    // loads (form 0).  In large launches the data streams through the L2 anyway;
    // there an agent-scope acquire per barrier lets the halo reads of
    // neighbouring tiles share L2 lines (form 1).  Two-pass iterations (an
    // elementwise pass, a barrier, a stencil pass that reads ph alone, form 2)
    // read a third of the halo for a second barrier.  A single system whose
    // tiles each get a workgroup runs the single-system kernel (form 3: tile
    // data in registers, no assignment).  Other launches that record CG-Lanczos
    // data use form 0.
    int mode = c->cg_mode;
    if (const char *e = getenv("RSR_CG_MODE")) mode = atoi(e);   // override for tuning sweeps
    const bool one = allow_one && m == 1 && tiles <= NT && tile_px > 0 && tile_px <= 4 * NT;
    const int by_size = px >= (2L << 20) ? 1 : 0;
    if (lz)
        L.form = one && mode != 1 ? 3 : 0;   // mode 1 forces form 0 (comparisons)
    else
        L.form = (mode >= 1 && mode <= 4) ? mode - 1 : tuned_form >= 0 ? tuned_form : one ? 3 : by_size;
    if (L.form == 3 && !one) L.form = lz ? 0 : by_size;
    for (;;) {
        const int bpc = cg_max_blocks_per_cu(L.lds, L.qt, lz, L.form);
        if (bpc < 1) fail(RSR_E_HIP, "persistent kernel does not fit on a CU");
        int G = std::min<long>((long)bpc * c->n_cu, std::min(1024, c->cg_gmax));
        if (const char *cap = getenv("RSR_CG_MAX_BLOCKS")) {   // launch-shape override for tuning sweeps
            const int v = atoi(cap);
            if (v >= 8) G = std::min(G, v);
        }
        // no more workgroups than tiles (rounded up to the 8 XCDs)
        G = (int)std::min<long>(G, (std::max<long>(8, tiles) + 7) & ~7L);
        if (G >= 8) G -= G % 8;
        L.G = G;
        if (L.form == 3 && G < tiles) {   // a workgroup per tile does not fit this grid
            L.form = lz ? 0 : by_size;
            continue;
        }
        return L;
    }
}

// Runs deflated CG from the current (x, r) of each listed system to the
// recursive-residual tolerance.  Returns per-system kernel status.
void run_cg(rsr_ctx *c, std::vector<SysHost *> &sy, const Opts &o, hipStream_t s)
{
    const int m = (int)sy.size();
    if (m == 0) return;
    if (m > MAXSYS) fail(RSR_E_ARG, "too many systems in one launch");
    std::vector<SysDev> hd(m);
    long tiles = 0;
    for (int i = 0; i < m; ++i) {
        SysHost &Y = *sy[i];
        const InstDev &I = c->h_inst[Y.inst];
        SysDev &d = hd[i];
        memset(&d, 0, sizeof(d));
        d.inst = Y.inst;
        d.q = Y.q;
        d.ntiles = I.nty * I.ntx;
        d.tile_base = (int)tiles;
        tiles += d.ntiles;
        d.gamma = Y.gamma;
        d.tolabs = o.tol * Y.bnorm;
        d.x = Y.x;
        d.rb[0] = Y.r;
        d.rb[1] = Y.r1;
        d.wb[0] = Y.w;
        d.wb[1] = Y.w1;
        d.pb[0] = Y.p0;
        d.pb[1] = Y.p1;
        d.pa = Y.pa;
        d.cbuf = Y.cbuf;
        d.W = Y.W;
        d.Z = Y.Z;
        d.ldw = Y.n;
        for (int a = 0; a < Y.q; ++a)
            for (int b2 = 0; b2 < Y.q; ++b2) d.Ginv[a * QMAX + b2] = Y.Ginv[a * Y.q + b2];
        d.lz = Y.lz;
        d.lzc = Y.lzc;
        d.nlz = Y.nlz;
    }
    WsMark mark(c);
    double *partA = (double *)dscratch(c, c->d_partA, sizeof(double) * tiles * NVP);
    double *partB = (double *)dscratch(c, c->d_partB, sizeof(double) * tiles * NVP);
    // the barrier block, the step flags and the outputs, zeroed by one fill
    const size_t out_bytes = (sizeof(int) * 2 + 2 * sizeof(double)) * m + 64;
    const size_t ctl_bytes = BAR_BYTES + FLAG_BYTES + out_bytes;
    char *ctl = (char *)dscratch(c, c->d_ctl, ctl_bytes);
    char *outb = ctl + BAR_BYTES + FLAG_BYTES;
    HIPCHK(launch_fill((double *)ctl, 0.0, (long)(ctl_bytes / sizeof(double)), s));
    int *out_iters = (int *)outb;
    int *out_status = out_iters + m;
    double *out_rho = (double *)(((uintptr_t)(out_status + m) + 15) & ~(uintptr_t)15);
    double *out_alpha = out_rho + m;

    int qmax = 0;
    bool lz = false;   // some system records CG-Lanczos data in this launch
    long px = 0;
    int tile_px = 0;
    for (auto *Y : sy) {
        qmax = std::max(qmax, Y->q);
        lz = lz || Y->nlz > 0;
        px += Y->n;
        tile_px = std::max(tile_px, c->h_inst[Y->inst].ty * c->h_inst[Y->inst].tx);
    }
    // the autotuned form, when every instance of the launch has the same one
    int tuned = -2;
    for (auto *Y : sy) {
        const int f = c->inst[Y->inst]->form;
        tuned = tuned == -2 ? f : (tuned == f ? f : -1);
    }
    const CgLaunch L = cg_config(c, m, qmax, lz, px, tiles, tuned < 0 ? -1 : tuned, tile_px);
    const int qt = L.qt, form = L.form, G = L.G, msys = L.msys, tl = L.tl, taps_lds = L.taps;
    const size_t lds = L.lds;

    CGArgs a;
    a.nsys = m;
    // the single-system kernel takes its descriptor in the kernel arguments
    a.sys = form == 3 ? nullptr : stage(c, hd, s);
    a.inst = c->d_inst.as<InstDev>();
    a.part[0] = partA;
    a.part[1] = partB;
    a.pstride = (int)tiles;
    a.bar = (unsigned long long *)ctl;
    a.abort_flag = (int *)(ctl + 256);
    a.out_iters = out_iters;
    a.out_status = out_status;
    a.out_rho = out_rho;
    a.out_alpha = out_alpha;
    a.maxit = o.maxit;
    a.form = form;
    a.G = G;
    a.timeout_ticks = (long long)(c->wall_khz * 1000.0 * c->bar_timeout_s);
    a.tile_lds = tl;
    a.taps_lds = taps_lds;
    a.msys = msys;
    a.stamps = nullptr;
    const bool dbg = getenv("RSR_CG_STAMPS") != nullptr && !c->wsa_base;   // phase timing of workgroup 0 (diagnostics)
    if (dbg) {
        c->d_dbg.ensure(sizeof(unsigned long long) * DBG_WORDS);
        HIPCHK(launch_fill((double *)c->d_dbg.p, 0.0, (long)DBG_WORDS, s));
        a.stamps = (unsigned long long *)c->d_dbg.p;
    }
    HIPCHK(hipEventRecord(c->ev0, s));
    {
        const hipError_t e = launch_cg(a, qt, lz, G, lds, s, form == 3 ? &hd[0] : nullptr);
        if (e != hipSuccess)
            fail(e == hipErrorOutOfMemory ? RSR_E_NOMEM : RSR_E_HIP,
                 std::string("persistent CG launch ") + std::to_string(c->last_launches + 1) + " of the call (" +
                     std::to_string(m) + " systems, " + std::to_string(G) + " workgroups): " + hipGetErrorString(e));
    }
    HIPCHK(hipEventRecord(c->ev1, s));
    // host work that does not depend on this launch, done while it runs
    for (auto *Y : sy) {
        Instance &I = *c->inst[Y->inst];
        if (I.p == 0 || !I.ae_valid || I.eig_pre.version == I.u_version) continue;
        double g = Y->gamma;
        for (auto *Z : sy)
            if (Z->inst == Y->inst) g = std::min(g, Z->gamma);
        std::vector<double> w, V;
        retained_eig(I, g, w, V);
    }
    std::vector<int> hi(2 * m + 8);
    std::vector<double> hr(2 * m);   // final r.r, then the pending step alpha
    int abort_h = 0;
    {
        // one copy from the abort flag to the end of the outputs
        const char *from = (const char *)a.abort_flag;
        std::vector<char> hb((size_t)(ctl + ctl_bytes - from));
        read_back(c, {ReadBack{hb.data(), from, hb.size()}}, s);
        memcpy(&abort_h, hb.data(), sizeof(int));
        memcpy(hi.data(), hb.data() + ((const char *)out_iters - from), sizeof(int) * 2 * m);
        memcpy(hr.data(), hb.data() + ((const char *)out_rho - from), sizeof(double) * 2 * m);
    }
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    if (dbg && form == 3) {
        // the single-system kernel's phases of workgroup 0: loads, sums and
        // decisions, deflation step, window, stencil, epilogue, partials, barrier
        std::vector<unsigned long long> st((size_t)DBG_ITERS * DBG_SLOTS);
        HIPCHK(hipMemcpy(st.data(), c->d_dbg.p, sizeof(unsigned long long) * st.size(), hipMemcpyDeviceToHost));
        const double tk = c->wall_khz / 1000.0;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int n = 0;
        for (int it = 1; it + 1 < DBG_ITERS; ++it) {
            const unsigned long long *e = st.data() + (size_t)it * DBG_SLOTS;
            if (!e[0] || !e[8] || !st[(size_t)(it + 1) * DBG_SLOTS]) break;
            for (int k = 0; k < 8; ++k) acc[k] += (double)(e[k + 1] - e[k]);
            ++n;
        }
        if (n > 0)
            fprintf(stderr, "[rsr cg1 stamps] G=%d iters=%d us: loads %.2f sums+decide %.2f local %.2f window %.2f "
                            "stencil %.2f epilogue %.2f partials %.2f barrier %.2f\n",
                    G, n, acc[0] / n / tk, acc[1] / n / tk, acc[2] / n / tk, acc[3] / n / tk, acc[4] / n / tk,
                    acc[5] / n / tk, acc[6] / n / tk, acc[7] / n / tk);
    } else if (dbg) {
        std::vector<unsigned long long> st(DBG_WORDS);
        HIPCHK(hipMemcpy(st.data(), c->d_dbg.p, sizeof(unsigned long long) * st.size(), hipMemcpyDeviceToHost));
        {
            // per-workgroup spread of a few iterations: the phase (assignment to
            // barrier arrival) of every workgroup, the slowest one and its CU, and
            // how many CUs hold more than one workgroup
            const double tk0 = c->wall_khz / 1000.0;
            for (int i = 0; i < DBG_WG_NIT; ++i) {
                const unsigned long long *w = st.data() + DBG_ITERS * DBG_SLOTS + (size_t)i * DBG_WG_MAX * 8;
                std::vector<std::pair<double, int>> ph;
                std::map<long, int> per_cu;
                double end_max = 0.0, top_max = 0.0, rel_max = 0.0;
                int b_end = -1, b_top = -1;
                unsigned long long t0 = ~0ull;
                for (int b = 0; b < std::min(G, DBG_WG_MAX); ++b)
                    if (w[b * 8] && w[b * 8 + 2]) t0 = std::min(t0, w[b * 8]);
                for (int b = 0; b < std::min(G, DBG_WG_MAX); ++b) {
                    const unsigned long long *e = w + b * 8;
                    if (!e[0] || !e[2]) continue;
                    ph.push_back({(double)(e[2] - e[1]) / tk0, b});
                    const double te = (double)(e[2] - t0) / tk0, tt = (double)(e[1] - e[0]) / tk0;
                    if (te > end_max) { end_max = te; b_end = b; }
                    if (tt > top_max) { top_max = tt; b_top = b; }
                    if (e[3]) rel_max = std::max(rel_max, (double)(e[3] - t0) / tk0);
                    const long hw = (long)(e[4] & 0xff00) | ((long)(e[5] & 0xf) << 16);   // CU, SH, SE, XCC
                    per_cu[hw]++;
                }
                if (ph.empty()) continue;
                std::sort(ph.begin(), ph.end());
                int shared = 0;
                for (auto &kv : per_cu) shared += kv.second > 1;
                const int bmax = ph.back().second;
                const unsigned long long *e = w + bmax * 8;
                fprintf(stderr,
                        "[rsr cg stamps] it %d: %zu wgs, phase us min %.2f med %.2f max %.2f (wg %d, hwid 0x%llx xcc %llu, "
                        "ends %.2f after the first top); last arrival %.2f (wg %d), longest top %.2f (wg %d), "
                        "last release seen %.2f; CUs with >1 wg: %d\n",
                        DBG_WG_IT0 + i, ph.size(), ph.front().first, ph[ph.size() / 2].first, ph.back().first, bmax,
                        e[4], e[5] & 0xf, (double)(e[2] - t0) / tk0, end_max, b_end, top_max, b_top, rel_max, shared);
            }
        }
        double acc[5] = {0, 0, 0, 0, 0}, top[5] = {0, 0, 0, 0, 0}, ph[5] = {0, 0, 0, 0, 0};
        int n = 0;
        for (int i = 1; i < DBG_ITERS && i + 1 < hi[0] && st[i * DBG_SLOTS + 3]; ++i, ++n) {
            for (int k = 0; k < 3; ++k) acc[k] += (double)(st[i * DBG_SLOTS + k + 1] - st[i * DBG_SLOTS + k]);
            if (st[i * DBG_SLOTS + 6] && st[i * DBG_SLOTS + 7]) {
                acc[3] += (double)(st[i * DBG_SLOTS + 6] - st[i * DBG_SLOTS + 1]);
                acc[4] += (double)(st[i * DBG_SLOTS + 7] - st[i * DBG_SLOTS + 6]);
            }
            // the loop top: flat loads, sums, decisions and compaction, assignment, local-space step
            const int kk[6] = {0, 8, 9, 10, 11, 1};
            for (int u = 0; u < 5; ++u)
                if (st[i * DBG_SLOTS + kk[u]] && st[i * DBG_SLOTS + kk[u + 1]])
                    top[u] += (double)(st[i * DBG_SLOTS + kk[u + 1]] - st[i * DBG_SLOTS + kk[u]]);
            // the first item: system switch, window staging, stencil, epilogue, partial sums
            const int kp[6] = {1, 12, 6, 7, 13, 14};
            for (int u = 0; u < 5; ++u)
                if (st[i * DBG_SLOTS + kp[u]] && st[i * DBG_SLOTS + kp[u + 1]])
                    ph[u] += (double)(st[i * DBG_SLOTS + kp[u + 1]] - st[i * DBG_SLOTS + kp[u]]);
        }
        const double tk = c->wall_khz / 1000.0;
        // iteration time by number of active systems (workgroup 0's loop-top stamps)
        // (key: active systems, grid size of that iteration)
        std::map<std::pair<int, int>, std::pair<double, int>> byact;
        for (int i = 0; i + 1 < DBG_ITERS && st[(i + 1) * DBG_SLOTS]; ++i) {
            auto &e = byact[{(int)st[i * DBG_SLOTS + 4], (int)st[i * DBG_SLOTS + 5]}];
            e.first += (double)(st[(i + 1) * DBG_SLOTS] - st[i * DBG_SLOTS]);
            e.second += 1;
        }
        if (!byact.empty()) {
            fprintf(stderr, "[rsr cg stamps] us/iteration by active systems:");
            for (auto &kv : byact)
                fprintf(stderr, " %d:%.1f(x%d,G%d)", kv.first.first, kv.second.first / kv.second.second / tk,
                        kv.second.second, kv.first.second);
            fprintf(stderr, "\n");
        }
        if (n > 0)
            fprintf(stderr, "[rsr cg stamps] G=%d iters=%d us: reduce+assign %.2f phase %.2f (first item: setup+load %.2f "
                            "stencil %.2f) barrier %.2f; top: loads %.2f sums %.2f decide %.2f assign %.2f local %.2f; "
                            "item: switch %.2f window %.2f stencil %.2f epilogue %.2f partials %.2f\n",
                    G, n, acc[0] / n / tk, acc[1] / n / tk, acc[3] / n / tk, acc[4] / n / tk, acc[2] / n / tk,
                    top[0] / n / tk, top[1] / n / tk, top[2] / n / tk, top[3] / n / tk, top[4] / n / tk, ph[0] / n / tk,
                    ph[1] / n / tk, ph[2] / n / tk, ph[3] / n / tk, ph[4] / n / tk);
    }
    c->last_cg_ms += ms;
    c->last_launches += 1;
    if (abort_h) fail(RSR_E_TIMEOUT, "persistent CG barrier timed out");
    for (int i = 0; i < m; ++i) {
        SysHost &Y = *sy[i];
        if (Y.nlz > 0) {   // only the first launch of a system is captured
            Y.lz_its = hi[i];
            Y.nlz = 0;
        }
        Y.iters += hi[i];
        Y.mvA += hi[i];
        Y.mvE += hi[i];
        c->mv_A += hi[i];
        c->mv_E += hi[i];
        Y.status = hi[m + i];
        c->last_items += (long)hi[i] * hd[i].ntiles;
    }
    // the kernel leaves the last step x += alpha p of each finished system to here
    std::vector<ComboJob> fj;
    std::vector<std::vector<double>> fq;
    for (int i = 0; i < m; ++i)
        if (hr[m + i] != 0.0) {
            SysHost &Y = *sy[i];
            fj.push_back(ComboJob{Y.pa, Y.n, 1, nullptr, 1, Y.x, Y.n, 1, 1.0, nullptr, 0, Y.n});
            fq.push_back(std::vector<double>{hr[m + i]});
        }
    if (!fj.empty()) combo(c, fj, fq, s);
}

// Galerkin correction with the local space: x += W y, r -= Z y, y = G^+ W^T r.
void local_correction(rsr_ctx *c, std::vector<SysHost *> &sy, hipStream_t s)
{
    std::vector<GramJob> gj;
    std::vector<SysHost *> act;
    for (auto *Y : sy)
        if (Y->q > 0) {
            gj.push_back(GramJob{Y->W, Y->n, Y->q, Y->r, Y->n, 1, Y->n, nullptr, 0});
            act.push_back(Y);
        }
    if (act.empty()) return;
    auto cs = gram(c, gj, s);
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    for (size_t k = 0; k < act.size(); ++k) {
        SysHost &Y = *act[k];
        std::vector<double> y(Y.q), ny(Y.q);
        matvec(Y.q, Y.q, Y.Ginv.data(), cs[k].data(), y.data());
        for (int i = 0; i < Y.q; ++i) ny[i] = -y[i];
        cj.push_back(ComboJob{Y.W, Y.n, Y.q, nullptr, Y.q, Y.x, Y.n, 1, 1.0, nullptr, 0, Y.n});
        qs.push_back(y);
        cj.push_back(ComboJob{Y.Z, Y.n, Y.q, nullptr, Y.q, Y.r, Y.n, 1, 1.0, nullptr, 0, Y.n});
        qs.push_back(ny);
    }
    combo(c, cj, qs, s);
}

// ------------------------------------------------------ recycled MINRES --
// The local recycle space of Sec. 4.2 (eq. localU): B Ut = K R with K^T K = I
// and U = Ut R^{-1}.  W holds Ut and Z = B Ut on entry; R comes from a Cholesky
// factorisation of Z^T Z on the host (a column whose pivot falls below 1e-12 of
// its diagonal is dropped), and K, U overwrite Z, W column by column
// (K_j = (Z_j - sum_{i<j} K_i R_ij) / R_jj, the same for U).
void minres_local_basis(rsr_ctx *c, std::vector<SysHost *> &sy, hipStream_t s)
{
    std::vector<GramJob> gj;
    std::vector<SysHost *> act;
    for (auto *Y : sy)
        if (Y->q > 0) {
            gj.push_back(GramJob{Y->Z, Y->n, Y->q, Y->Z, Y->n, Y->q, Y->n, nullptr, 0});
            act.push_back(Y);
        }
    if (act.empty()) return;
    auto G = gram(c, gj, s);
    std::vector<std::vector<double>> Rs(act.size());
    std::vector<std::vector<char>> keep(act.size());
    int qmax = 0;
    for (size_t k = 0; k < act.size(); ++k) {
        const int q = act[k]->q;
        qmax = std::max(qmax, q);
        std::vector<double> &R = Rs[k];   // row-major q x q, upper triangular, G = R^T R
        R.assign((size_t)q * q, 0.0);
        keep[k].assign(q, 1);
        const std::vector<double> &Gm = G[k];
        for (int j = 0; j < q; ++j) {
            double d = Gm[(size_t)j * q + j];
            for (int i = 0; i < j; ++i) d -= R[(size_t)i * q + j] * R[(size_t)i * q + j];
            if (!(d > 1e-12 * Gm[(size_t)j * q + j]) || !std::isfinite(d)) {
                keep[k][j] = 0;   // numerically inside the span of the earlier columns
                continue;
            }
            R[(size_t)j * q + j] = std::sqrt(d);
            for (int l = j + 1; l < q; ++l) {
                double t = Gm[(size_t)j * q + l];
                for (int i = 0; i < j; ++i) t -= R[(size_t)i * q + j] * R[(size_t)i * q + l];
                R[(size_t)j * q + l] = t / R[(size_t)j * q + j];
            }
        }
    }
    for (int j = 0; j < qmax; ++j) {
        std::vector<ComboJob> cj;
        std::vector<std::vector<double>> qs;
        for (size_t k = 0; k < act.size(); ++k) {
            SysHost &Y = *act[k];
            const int q = Y.q;
            if (j >= q) continue;
            const std::vector<double> &R = Rs[k];
            const long n = Y.n;
            const double rjj = keep[k][j] ? R[(size_t)j * q + j] : 0.0;
            const double sc = rjj > 0.0 ? 1.0 / rjj : 0.0;
            std::vector<double> co(std::max(j, 1), 0.0);
            for (int i = 0; i < j; ++i) co[i] = keep[k][i] ? -R[(size_t)i * q + j] * sc : 0.0;
            // Z_j <- (Z_j - K_{<j} R_{<j,j}) / R_jj and W_j likewise (in place)
            cj.push_back(ComboJob{Y.Z, n, j, nullptr, std::max(j, 1), Y.Z + (size_t)j * n, n, 1, sc, nullptr, 0, n});
            qs.push_back(co);
            cj.push_back(ComboJob{Y.W, n, j, nullptr, std::max(j, 1), Y.W + (size_t)j * n, n, 1, sc, nullptr, 0, n});
            qs.push_back(co);
        }
        combo(c, cj, qs, s);
    }
}

// Recycled MINRES (Sec. 2.3, Sec. 4.2) from the current (x, r = b - B x) of each
// listed system with its local space (K, U in Z, W): Lanczos with
// (I - K K^T) B from v_1 = (I - K K^T) r / xi; the tridiagonal's QR by Givens
// rotations gives the iterate y_m of min ||T_m y - xi e_1|| by short recurrences
// (direction vectors d_j); the residual norm |eta| of that problem is the true
// one of the augmented problem eq. minShift, whose U-part is solved exactly at
// the end: x = x + y_m + U K^T (r - B y_m) (eq. xFinal).  Every step is a
// batched launch over the active systems (operator applications, products,
// combinations); the scalar recurrences run on the host.
void run_minres(rsr_ctx *c, std::vector<SysHost *> &sy, const Opts &o, hipStream_t s)
{
    const int m = (int)sy.size();
    if (m == 0) return;
    struct St {
        double beta, eta, g_prev, g_cur, s_prev, s_cur;
        double *vp, *vc, *d2, *d1;   // v_{j-1}, v_j, d_{j-2}, d_{j-1}
        bool active;
        int its;
    };
    std::vector<St> st(m);
    // buffers: v in p0/p1 (adjacent), w in w, y_m in r1, directions in pa / w1, scratch rt
    {
        // r_p = (I - K K^T) r, then xi
        std::vector<GramJob> gj;
        for (auto *Y : sy)
            if (Y->q > 0) gj.push_back(GramJob{Y->Z, Y->n, Y->q, Y->r, Y->n, 1, Y->n, nullptr, 0});
        auto kr = gram(c, gj, s);
        std::vector<ComboJob> cj;
        std::vector<std::vector<double>> qs;
        size_t kk = 0;
        for (auto *Y : sy) {
            std::vector<double> co(std::max(Y->q, 1), 0.0);
            if (Y->q > 0) {
                for (int i = 0; i < Y->q; ++i) co[i] = -kr[kk][i];
                ++kk;
            }
            cj.push_back(ComboJob{Y->Z, Y->n, Y->q, nullptr, std::max(Y->q, 1), Y->p0, Y->n, 1, 0.0, Y->r, Y->n, Y->n});
            qs.push_back(co);
            // y_m = 0 and both directions 0 (combinations of no columns)
            cj.push_back(ComboJob{nullptr, Y->n, 0, nullptr, 0, Y->r1, Y->n, 1, 0.0, nullptr, 0, Y->n});
            qs.push_back({});
            cj.push_back(ComboJob{nullptr, Y->n, 0, nullptr, 0, Y->pa, Y->n, 1, 0.0, nullptr, 0, Y->n});
            qs.push_back({});
            cj.push_back(ComboJob{nullptr, Y->n, 0, nullptr, 0, Y->w1, Y->n, 1, 0.0, nullptr, 0, Y->n});
            qs.push_back({});
            cj.push_back(ComboJob{nullptr, Y->n, 0, nullptr, 0, Y->p1, Y->n, 1, 0.0, nullptr, 0, Y->n});
            qs.push_back({});
        }
        combo(c, cj, qs, s);
        std::vector<const double *> v;
        std::vector<long> n;
        for (auto *Y : sy) {
            v.push_back(Y->p0);
            n.push_back(Y->n);
        }
        auto xi = norms(c, v, n, s);
        cj.clear();
        qs.clear();
        for (int i = 0; i < m; ++i) {
            SysHost &Y = *sy[i];
            St &t = st[i];
            t = St{xi[i], xi[i], 1.0, 1.0, 0.0, 0.0, Y.p1, Y.p0, Y.w1, Y.pa, true, 0};
            if (!std::isfinite(xi[i])) fail(RSR_E_NONFINITE, "non-finite residual");
            if (!(xi[i] > o.tol * Y.bnorm)) {
                t.active = false;   // the local space alone meets the tolerance
                Y.status = 1;
                continue;
            }
            cj.push_back(ComboJob{nullptr, Y.n, 0, nullptr, 0, Y.p0, Y.n, 1, 1.0 / xi[i], nullptr, 0, Y.n});
            qs.push_back({});
        }
        combo(c, cj, qs, s);
    }
    for (int it = 0;; ++it) {
        std::vector<int> act;
        for (int i = 0; i < m; ++i)
            if (st[i].active) act.push_back(i);
        if (act.empty()) break;
        // w = B v_j
        std::vector<ApplyJob> aj;
        for (int i : act) {
            SysHost &Y = *sy[i];
            aj.push_back(ApplyJob{Y.inst, 0, 1.0, Y.gamma, st[i].vc, Y.w});
            Y.mvA++;
            Y.mvE++;
        }
        apply_jobs(c, aj, s);
        // K^T w and alpha = v_j^T w
        std::vector<GramJob> gj;
        for (int i : act) {
            SysHost &Y = *sy[i];
            gj.push_back(GramJob{st[i].vc, Y.n, 1, Y.w, Y.n, 1, Y.n, nullptr, 0});
            if (Y.q > 0) gj.push_back(GramJob{Y.Z, Y.n, Y.q, Y.w, Y.n, 1, Y.n, nullptr, 0});
        }
        auto h = gram(c, gj, s);
        std::vector<double> alpha(m, 0.0);
        {
            // w <- w - K c, then w <- w - alpha v_j - beta v_{j-1} (v_{j-1}, v_j are p0, p1)
            std::vector<ComboJob> c1, c2;
            std::vector<std::vector<double>> q1, q2;
            size_t k = 0;
            for (int i : act) {
                SysHost &Y = *sy[i];
                alpha[i] = h[k++][0];
                if (Y.q > 0) {
                    std::vector<double> co(Y.q);
                    for (int j = 0; j < Y.q; ++j) co[j] = -h[k][j];
                    ++k;
                    c1.push_back(ComboJob{Y.Z, Y.n, Y.q, nullptr, Y.q, Y.w, Y.n, 1, 1.0, nullptr, 0, Y.n});
                    q1.push_back(co);
                }
                const bool cur_is_p1 = st[i].vc == Y.p1;
                std::vector<double> co{cur_is_p1 ? -st[i].beta : -alpha[i], cur_is_p1 ? -alpha[i] : -st[i].beta};
                if (it == 0) co[cur_is_p1 ? 0 : 1] = 0.0;   // v_0 = 0
                c2.push_back(ComboJob{Y.p0, Y.n, 2, nullptr, 2, Y.w, Y.n, 1, 1.0, nullptr, 0, Y.n});
                q2.push_back(co);
            }
            combo(c, c1, q1, s);
            combo(c, c2, q2, s);
        }
        std::vector<const double *> v;
        std::vector<long> nn;
        for (int i : act) {
            v.push_back(sy[i]->w);
            nn.push_back(sy[i]->n);
        }
        auto bnew = norms(c, v, nn, s);
        // Givens on the new column of the tridiagonal; direction and iterate updates
        std::vector<ComboJob> ca, cb, cc;
        std::vector<std::vector<double>> qa, qb, qc;
        for (size_t a = 0; a < act.size(); ++a) {
            const int i = act[a];
            SysHost &Y = *sy[i];
            St &t = st[i];
            const double al = alpha[i], bn = bnew[a];
            const double delta = t.g_cur * al - t.g_prev * t.s_cur * t.beta;
            const double rho1 = std::hypot(delta, bn);
            const double rho2 = t.s_cur * al + t.g_prev * t.g_cur * t.beta;
            const double rho3 = t.s_prev * t.beta;
            if (!std::isfinite(rho1) || !std::isfinite(al)) fail(RSR_E_NONFINITE, "non-finite value in MINRES");
            if (!(rho1 > 0.0)) {   // exact breakdown: the current iterate solves the problem
                t.active = false;
                Y.status = 1;
                continue;
            }
            const double gn = delta / rho1, sn = bn / rho1;
            // d_j = (v_j - rho3 d_{j-2} - rho2 d_{j-1}) / rho1 into d_{j-2}'s buffer;
            // v_{j+1} = w / beta_{j+1} into v_{j-1}'s buffer
            ca.push_back(ComboJob{t.vc, Y.n, 1, nullptr, 1, t.d2, Y.n, 1, -rho3 / rho1, nullptr, 0, Y.n});
            qa.push_back({1.0 / rho1});
            if (bn > 0.0) {
                ca.push_back(ComboJob{Y.w, Y.n, 1, nullptr, 1, t.vp, Y.n, 1, 0.0, nullptr, 0, Y.n});
                qa.push_back({1.0 / bn});
            }
            cb.push_back(ComboJob{t.d1, Y.n, 1, nullptr, 1, t.d2, Y.n, 1, 1.0, nullptr, 0, Y.n});
            qb.push_back({-rho2 / rho1});
            cc.push_back(ComboJob{t.d2, Y.n, 1, nullptr, 1, Y.r1, Y.n, 1, 1.0, nullptr, 0, Y.n});
            qc.push_back({gn * t.eta});
            t.eta = -sn * t.eta;
            t.its++;
            std::swap(t.d2, t.d1);   // d_j becomes d_{j-1}
            std::swap(t.vp, t.vc);   // v_{j+1} becomes v_j
            t.g_prev = t.g_cur;
            t.g_cur = gn;
            t.s_prev = t.s_cur;
            t.s_cur = sn;
            t.beta = bn;
            if (std::fabs(t.eta) <= o.tol * Y.bnorm || bn == 0.0) {
                t.active = false;
                Y.status = 1;
            } else if (t.its >= o.maxit) {
                t.active = false;
                Y.status = 2;
            }
        }
        combo(c, ca, qa, s);
        combo(c, cb, qb, s);
        combo(c, cc, qc, s);
    }
    // x += y_m + U K^T (r - B y_m)
    std::vector<ApplyJob> aj;
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    for (int i = 0; i < m; ++i) {
        SysHost &Y = *sy[i];
        Y.iters += st[i].its;
        if (Y.q > 0) {
            aj.push_back(ApplyJob{Y.inst, 0, 1.0, Y.gamma, Y.r1, Y.rt});
            Y.mvA++;
            Y.mvE++;
        }
        cj.push_back(ComboJob{Y.r1, Y.n, 1, nullptr, 1, Y.x, Y.n, 1, 1.0, nullptr, 0, Y.n});
        qs.push_back({1.0});
    }
    apply_jobs(c, aj, s);
    combo(c, cj, qs, s);
    cj.clear();
    qs.clear();
    std::vector<GramJob> gj;
    std::vector<SysHost *> kq;
    for (int i = 0; i < m; ++i) {
        SysHost &Y = *sy[i];
        if (Y.q == 0) continue;
        cj.push_back(ComboJob{Y.rt, Y.n, 1, nullptr, 1, Y.rt, Y.n, 1, 0.0, Y.r, Y.n, Y.n});
        qs.push_back({-1.0});
        gj.push_back(GramJob{Y.Z, Y.n, Y.q, Y.rt, Y.n, 1, Y.n, nullptr, 0});
        kq.push_back(&Y);
    }
    combo(c, cj, qs, s);
    auto kz = gram(c, gj, s);
    cj.clear();
    qs.clear();
    for (size_t k = 0; k < kq.size(); ++k) {
        SysHost &Y = *kq[k];
        cj.push_back(ComboJob{Y.W, Y.n, Y.q, nullptr, Y.q, Y.x, Y.n, 1, 1.0, nullptr, 0, Y.n});
        qs.push_back(kz[k]);
    }
    combo(c, cj, qs, s);
}

// ------------------------------------------------- host-driven deflated CG --
// Deflated CG (Algorithm 4 in CG form) for systems whose operator has no
// persistent kernel (tomography instances): every step is one batched launch
// over the active systems (operator application, products, combinations) with
// the scalars formed on the host.  From x, r with W^T r = 0 (the Galerkin
// correction), p_0 = r_0 - W mu_0 and per step
//   w = B p, alpha = r.r / p.w, x += alpha p, r -= alpha w,
//   beta = r'.r' / r.r, mu = G^+ Z^T r', p = r' + beta p - W mu,
// with mu = G^+ Z^T r (G = W^T Z, Z = B W).
void run_cg_host(rsr_ctx *c, std::vector<SysHost *> &sy, const Opts &o, hipStream_t s)
{
    const int m = (int)sy.size();
    if (m == 0) return;
    struct St {
        double rr;
        bool active;
        int its;
    };
    std::vector<St> st(m);
    // r.r and Z^T r of the current residuals: the columns of one product
    auto rz = [&](const std::vector<int> &idx) {
        std::vector<GramJob> gj;
        for (int i : idx) {
            SysHost &Y = *sy[i];
            gj.push_back(GramJob{Y.r, Y.n, 1, Y.r, Y.n, 1, Y.n, nullptr, 0});
            if (Y.q > 0) gj.push_back(GramJob{Y.Z, Y.n, Y.q, Y.r, Y.n, 1, Y.n, nullptr, 0});
        }
        return gram(c, gj, s);
    };
    // p = beta p + r, then p -= W mu
    auto new_dir = [&](const std::vector<int> &idx, const std::vector<double> &beta,
                       const std::vector<std::vector<double>> &zr) {
        std::vector<ComboJob> c1, c2;
        std::vector<std::vector<double>> q1, q2;
        for (size_t a = 0; a < idx.size(); ++a) {
            SysHost &Y = *sy[idx[a]];
            c1.push_back(ComboJob{Y.r, Y.n, 1, nullptr, 1, Y.pa, Y.n, 1, beta[a], nullptr, 0, Y.n});
            q1.push_back({1.0});
            if (Y.q > 0) {
                std::vector<double> mu(Y.q);
                matvec(Y.q, Y.q, Y.Ginv.data(), zr[a].data(), mu.data());
                for (double &v : mu) v = -v;
                c2.push_back(ComboJob{Y.W, Y.n, Y.q, nullptr, Y.q, Y.pa, Y.n, 1, 1.0, nullptr, 0, Y.n});
                q2.push_back(mu);
            }
        }
        combo(c, c1, q1, s);
        combo(c, c2, q2, s);
    };
    {
        std::vector<int> all(m);
        for (int i = 0; i < m; ++i) all[i] = i;
        auto h = rz(all);
        std::vector<int> go;
        std::vector<double> beta;
        std::vector<std::vector<double>> zr;
        size_t k = 0;
        for (int i = 0; i < m; ++i) {
            SysHost &Y = *sy[i];
            const double rr = h[k++][0];
            std::vector<double> z;
            if (Y.q > 0) z = h[k++];
            if (!std::isfinite(rr)) fail(RSR_E_NONFINITE, "non-finite residual");
            st[i] = St{rr, true, 0};
            if (!(std::sqrt(rr) > o.tol * Y.bnorm)) {
                st[i].active = false;
                Y.status = 1;
                continue;
            }
            go.push_back(i);
            beta.push_back(0.0);
            zr.push_back(z);
        }
        new_dir(go, beta, zr);
    }
    for (;;) {
        std::vector<int> act;
        for (int i = 0; i < m; ++i)
            if (st[i].active) act.push_back(i);
        if (act.empty()) break;
        std::vector<ApplyJob> aj;
        std::vector<GramJob> gj;
        for (int i : act) {
            SysHost &Y = *sy[i];
            aj.push_back(ApplyJob{Y.inst, 0, 1.0, Y.gamma, Y.pa, Y.w});
            Y.mvA++;
            Y.mvE++;
            gj.push_back(GramJob{Y.pa, Y.n, 1, Y.w, Y.n, 1, Y.n, nullptr, 0});
        }
        apply_jobs(c, aj, s);
        auto pw = gram(c, gj, s);
        std::vector<ComboJob> cj;
        std::vector<std::vector<double>> qs;
        for (size_t a = 0; a < act.size(); ++a) {
            SysHost &Y = *sy[act[a]];
            const double d = pw[a][0];
            if (!std::isfinite(d)) fail(RSR_E_NONFINITE, "non-finite value in CG");
            if (!(d > 0.0)) fail(RSR_E_NOT_SPD, "shifted matrix not SPD (p^T B p <= 0)");
            const double alpha = st[act[a]].rr / d;
            cj.push_back(ComboJob{Y.pa, Y.n, 1, nullptr, 1, Y.x, Y.n, 1, 1.0, nullptr, 0, Y.n});
            qs.push_back({alpha});
            cj.push_back(ComboJob{Y.w, Y.n, 1, nullptr, 1, Y.r, Y.n, 1, 1.0, nullptr, 0, Y.n});
            qs.push_back({-alpha});
        }
        combo(c, cj, qs, s);
        auto h = rz(act);
        std::vector<int> go;
        std::vector<double> beta;
        std::vector<std::vector<double>> zr;
        size_t k = 0;
        for (int i : act) {
            SysHost &Y = *sy[i];
            St &t = st[i];
            const double rr = h[k++][0];
            std::vector<double> z;
            if (Y.q > 0) z = h[k++];
            if (!std::isfinite(rr)) fail(RSR_E_NONFINITE, "non-finite value in CG");
            t.its++;
            if (std::sqrt(rr) <= o.tol * Y.bnorm) {
                t.active = false;
                Y.status = 1;
            } else if (t.its >= o.maxit) {
                t.active = false;
                Y.status = 2;
            } else {
                go.push_back(i);
                beta.push_back(rr / t.rr);
                zr.push_back(z);
            }
            t.rr = rr;
        }
        new_dir(go, beta, zr);
    }
    for (int i = 0; i < m; ++i) sy[i]->iters += st[i].its;
}

// Builds W, Z, G^+ for each system (Algorithms 2-4 in CG form).
void build_local(rsr_ctx *c, std::vector<SysHost *> &sy, const Opts &o, const double *g_prev_shift,
                 hipStream_t s)
{
    // Ritz blocks per (instance, group): Algorithm 2 on A_hat + gamma_J E_hat, then
    // R = U W~, AR = AU W~, ER = EU W~; cached until U or gamma_J changes
    struct Grp {
        int inst;
        double gJ;
        int nr;
        double *R;   // [nr][n], AR, ER follow
    };
    std::map<std::pair<int, int>, Grp> groups;
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    // the groups whose Ritz block is stale: their eigenproblems run concurrently
    struct EigJob {
        Instance *I;
        double gJ;
        std::vector<double> w, V;
    };
    std::vector<EigJob> ej;
    {
        std::set<std::pair<int, int>> seen;
        for (auto *Y : sy) {
            Instance &I = *c->inst[Y->inst];
            if (o.n_ritz <= 0 || I.p == 0 || !I.ae_valid) continue;
            const int side = Y->shift < o.split_I ? 0 : 1;
            if (!seen.insert(std::make_pair(Y->inst, side)).second) continue;
            const double gJ = side == 0 ? o.gJL : o.gJR;
            const int nr = std::min(o.n_ritz, I.p);
            const Instance::RitzBlock &rb = I.ritz[side];
            if (rb.version != I.u_version || rb.gamma != gJ || rb.nr != nr) ej.push_back(EigJob{&I, gJ, {}, {}});
        }
        parallel_for((int)ej.size(), HOST_THREADS, [&](int k) {
            EigJob &e = ej[k];
            const int p = e.I->p;
            std::vector<double> H((size_t)p * p);
            for (size_t t = 0; t < H.size(); ++t) H[t] = e.I->Ahat[t] + e.gJ * e.I->Ehat[t];
            sym_eig(p, H.data(), e.w, e.V);
        });
    }
    size_t ejk = 0;
    for (auto *Y : sy) {
        Instance &I = *c->inst[Y->inst];
        if (o.n_ritz <= 0 || I.p == 0 || !I.ae_valid) continue;
        const int side = Y->shift < o.split_I ? 0 : 1;
        auto key = std::make_pair(Y->inst, side);
        if (groups.count(key)) continue;
        const double gJ = side == 0 ? o.gJL : o.gJR;
        const int nr = std::min(o.n_ritz, I.p);
        Instance::RitzBlock &rb = I.ritz[side];
        if (rb.version != I.u_version || rb.gamma != gJ || rb.nr != nr) {
            const int p = I.p;
            if (c->wsa_base && rb.buf.bytes < sizeof(double) * (size_t)3 * nr * I.n)
                fail(RSR_E_STATE, "Ritz block storage not reserved for this call: call rsr_workspace_size with its descriptor first");
            rb.buf.ensure(sizeof(double) * (size_t)3 * nr * I.n);
            const std::vector<double> &V = ej[ejk++].V;   // same order as the collection above
            std::vector<double> Wt((size_t)p * nr);   // column-major p x nr
            for (int j = 0; j < nr; ++j)
                for (int i = 0; i < p; ++i) Wt[(size_t)j * p + i] = V[(size_t)i * p + j];
            double *R = rb.buf.as<double>();
            cj.push_back(ComboJob{I.d_U.as<double>(), I.n, p, nullptr, p, R, I.n, nr, 0.0, nullptr, 0, I.n});
            qs.push_back(Wt);
            cj.push_back(ComboJob{I.d_AE.as<double>(), I.n, p, nullptr, p, R + (size_t)nr * I.n, I.n, nr, 0.0,
                                  nullptr, 0, I.n});
            qs.push_back(Wt);
            cj.push_back(ComboJob{I.d_AE.as<double>() + (size_t)p * I.n, I.n, p, nullptr, p,
                                  R + (size_t)2 * nr * I.n, I.n, nr, 0.0, nullptr, 0, I.n});
            qs.push_back(Wt);
            rb.version = I.u_version;
            rb.gamma = gJ;
            rb.nr = nr;
        }
        groups[key] = Grp{Y->inst, gJ, nr, rb.buf.as<double>()};
    }
    combo(c, cj, qs, s);
    // assemble W, Z per system
    std::vector<ApplyJob> aj;
    cj.clear();
    qs.clear();
    for (auto *Yp : sy) {
        SysHost &Y = *Yp;
        Instance &I = *c->inst[Y.inst];
        int q = 0;
        const int side = Y.shift < o.split_I ? 0 : 1;
        auto it = groups.find(std::make_pair(Y.inst, side));
        if (it != groups.end()) {
            Grp &g = it->second;
            const int nr = std::min(g.nr, QMAX);
            // W[:, 0:nr] = R ; Z[:, 0:nr] = AR + gamma ER
            std::vector<double> id((size_t)nr * nr, 0.0), gid((size_t)2 * nr * nr, 0.0);
            for (int j = 0; j < nr; ++j) id[(size_t)j * nr + j] = 1.0;
            cj.push_back(ComboJob{g.R, I.n, nr, nullptr, nr, Y.W, Y.n, nr, 0.0, nullptr, 0, Y.n});
            qs.push_back(id);
            // [AR ER] (2nr columns, contiguous) times [I; gamma I]
            for (int j = 0; j < nr; ++j) {
                gid[(size_t)j * 2 * nr + j] = 1.0;
                gid[(size_t)j * 2 * nr + nr + j] = Y.gamma;
            }
            cj.push_back(ComboJob{g.R + (size_t)g.nr * I.n, I.n, 2 * nr, nullptr, 2 * nr, Y.Z, Y.n, nr, 0.0, nullptr,
                                  0, Y.n});
            qs.push_back(gid);
            q = nr;
        }
        // previous corrections
        std::vector<const double *> gcols;
        if (o.use_prev_k) {
            if (double *gv = I.gslot(Y.slot)) gcols.push_back(gv);
            // an adjoint system also takes the forward solve's correction of its
            // shift: the same matrix, and the directions its CG had to resolve
            if (Y.fwd_slot >= 0)
                if (double *gv = I.gslot(Y.fwd_slot)) gcols.push_back(gv);
        }
        if (o.use_prev_shift && g_prev_shift) gcols.push_back(g_prev_shift);
        for (const double *gv : gcols) {
            if (q >= QMAX) break;
            // W[:, q] = g, a copy folded into the same combination launch
            cj.push_back(ComboJob{gv, Y.n, 1, nullptr, 1, Y.W + (size_t)q * Y.n, Y.n, 1, 0.0, nullptr, 0, Y.n});
            qs.push_back(std::vector<double>{1.0});
            aj.push_back(ApplyJob{Y.inst, 0, 1.0, Y.gamma, Y.W + (size_t)q * Y.n, Y.Z + (size_t)q * Y.n});
            Y.mvA += 1;
            Y.mvE += 1;
            ++q;
        }
        Y.q = q;
    }
    combo(c, cj, qs, s);
    apply_jobs(c, aj, s);
    // angle check between the two correction columns and G = W^T Z
    std::vector<GramJob> gj;
    std::vector<SysHost *> act;
    for (auto *Y : sy)
        if (Y->q > 0) {
            gj.push_back(GramJob{Y->W, Y->n, Y->q, Y->Z, Y->n, Y->q, Y->n, nullptr, 0});
            gj.push_back(GramJob{Y->W, Y->n, Y->q, Y->W, Y->n, Y->q, Y->n, nullptr, 0});
            act.push_back(Y);
        }
    auto G = gram(c, gj, s);
    for (size_t k = 0; k < act.size(); ++k) {
        SysHost &Y = *act[k];
        std::vector<double> Gm = G[2 * k], WW = G[2 * k + 1];
        const int q = Y.q;
        // symmetrise W^T Z (B symmetric)
        for (int i = 0; i < q; ++i)
            for (int j = i + 1; j < q; ++j) {
                const double v = 0.5 * (Gm[i * q + j] + Gm[j * q + i]);
                Gm[i * q + j] = Gm[j * q + i] = v;
            }
        // drop the later of two nearly parallel columns (|cos| > 0.99), footnote of Sec. 5.3
        std::vector<int> keep(q, 1);
        for (int i = 0; i < q; ++i)
            for (int j = i + 1; j < q; ++j) {
                const double den = std::sqrt(WW[i * q + i] * WW[j * q + j]);
                if (keep[i] && keep[j] && den > 0 && std::fabs(WW[i * q + j]) > 0.99 * den) keep[j] = 0;
            }
        for (int i = 0; i < q; ++i)
            if (!keep[i])
                for (int j = 0; j < q; ++j) Gm[i * q + j] = Gm[j * q + i] = 0.0;
        spd_pinv(q, Gm.data(), 1e-12, Y.Ginv);
    }
}

// ------------------------------------------------------------- solving --
void solve_group(rsr_ctx *c, std::vector<SysHost *> &sy, const Opts &o, const double *g_prev_shift,
                 hipStream_t s)
{
    // b norms (once per distinct right-hand side of the call)
    std::unique_ptr<StageTimer> tm(new StageTimer(c, s, 0));
    {
        std::vector<const double *> v;
        std::vector<long> n;
        std::vector<SysHost *> need;
        std::set<std::pair<const double *, int>> queued;
        for (auto *Y : sy) {
            const auto key = std::make_pair((const double *)Y->b, Y->inst);
            if (c->bnorm_cache.count(key) || queued.count(key)) continue;   // once per right-hand side
            queued.insert(key);
            v.push_back(Y->b);
            n.push_back(Y->n);
            need.push_back(Y);
        }
        if (!need.empty()) {
            auto bn = norms(c, v, n, s);
            for (size_t i = 0; i < need.size(); ++i) c->bnorm_cache[{need[i]->b, need[i]->inst}] = bn[i];
        }
        for (auto *Y : sy) {
            Y->bnorm = c->bnorm_cache[{Y->b, Y->inst}];
            if (!std::isfinite(Y->bnorm)) fail(RSR_E_NONFINITE, "non-finite right-hand side");
        }
    }
    // initial guess
    tm.reset(new StageTimer(c, s, 1));
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    std::vector<ApplyJob> aj;
    std::vector<SysHost *> need_r;   // r = b - B x
    for (auto *Yp : sy) {
        SysHost &Y = *Yp;
        Instance &I = *c->inst[Y.inst];
        int init = o.init;
        if ((init == RSR_INIT_MR || init == RSR_INIT_GALERKIN || init == RSR_INIT_OBLIQUE) && (I.p == 0 || !I.ae_valid))
            init = RSR_INIT_ZERO;
        if (init == RSR_INIT_ZERO) {
            // x = 0 (a combination of no columns) and r = b, in the launch shared by all systems
            cj.push_back(ComboJob{nullptr, Y.n, 0, nullptr, 0, Y.x, Y.n, 1, 0.0, nullptr, 0, Y.n});
            qs.push_back(std::vector<double>{});
            cj.push_back(ComboJob{Y.b, Y.n, 1, nullptr, 1, Y.r, Y.n, 1, 0.0, nullptr, 0, Y.n});
            qs.push_back(std::vector<double>{1.0});
        } else if (init == RSR_INIT_GIVEN) {
            aj.push_back(ApplyJob{Y.inst, 0, 1.0, Y.gamma, Y.x, Y.r});
            Y.mvA++;
            Y.mvE++;
            need_r.push_back(&Y);
        }
    }
    apply_jobs(c, aj, s);
    for (auto *Y : need_r) {
        std::vector<double> one{-1.0};
        cj.push_back(ComboJob{Y->r, Y->n, 1, nullptr, 1, Y->r, Y->n, 1, 0.0, Y->b, Y->n, Y->n});
        qs.push_back(one);
    }
    combo(c, cj, qs, s);
    cj.clear();
    qs.clear();
    // principal-space guesses (one small solve per shift, Section 4.1)
    std::vector<GramJob> gj;
    std::vector<SysHost *> prin, fresh;
    std::set<std::tuple<const double *, int, int>> queued;
    for (auto *Yp : sy) {
        SysHost &Y = *Yp;
        Instance &I = *c->inst[Y.inst];
        if (!((o.init == RSR_INIT_MR || o.init == RSR_INIT_GALERKIN || o.init == RSR_INIT_OBLIQUE) && I.p > 0 &&
              I.ae_valid))
            continue;
        prin.push_back(&Y);
        const auto key = std::make_tuple((const double *)Y.b, Y.inst, o.init);
        if (c->rhs_cache.count(key) || queued.count(key)) continue;   // once per right-hand side
        queued.insert(key);
        fresh.push_back(&Y);
        if (o.init == RSR_INIT_MR || o.init == RSR_INIT_OBLIQUE)
            gj.push_back(GramJob{I.d_AE.as<double>(), I.n, 2 * I.p, Y.b, Y.n, 1, Y.n, nullptr, 0});
        else
            gj.push_back(GramJob{I.d_U.as<double>(), I.n, I.p, Y.b, Y.n, 1, Y.n, nullptr, 0});
    }
    if (!prin.empty()) {
        // [AU EU]^T b (or U^T b) once per right-hand side of the call
        if (!fresh.empty()) {
            auto got = gram(c, gj, s);
            for (size_t k = 0; k < fresh.size(); ++k)
                c->rhs_cache[{fresh[k]->b, fresh[k]->inst, o.init}] = got[k];
        }
        std::vector<std::vector<double>> rhs;
        for (auto *Y : prin) rhs.push_back(c->rhs_cache[{Y->b, Y->inst, o.init}]);
        // systems that share an instance and a right-hand side form one
        // combination each for x0 and r0 (the panels U, [AU EU] are read once
        // per group); the columns land in scratch and are copied out together
        struct InitGrp {
            int inst;
            const double *b;
            std::vector<SysHost *> sys;
            std::vector<double> Qx, Qr;
        };
        std::vector<InitGrp> grp;
        grp.reserve(prin.size());
        // one small solve per shift, on several host threads
        std::vector<std::vector<double>> qv(prin.size());
        parallel_for((int)prin.size(), HOST_THREADS, [&](int k) {
            SysHost &Y = *prin[k];
            Instance &I = *c->inst[Y.inst];
            const int p = I.p;
            const double g = Y.gamma;
            std::vector<double> H((size_t)p * p), f(p), P;
            std::vector<double> &q = qv[k];
            q.assign(p, 0.0);
            bool solved = false;
            if (o.init == RSR_INIT_OBLIQUE) {
                // K = AU + gs EU with the group's reference shift gs; the oblique
                // condition K^T r0 = 0 gives K^T (AU + g EU) q = K^T b (eq. obliqueupdate)
                const double gs = Y.shift < o.split_I ? o.gJL : o.gJR;
                for (int i = 0; i < p; ++i)
                    for (int j = 0; j < p; ++j)
                        H[(size_t)i * p + j] = I.Gaa[(size_t)i * p + j] + g * I.Gae[(size_t)i * p + j] +
                                               gs * I.Gae[(size_t)j * p + i] + gs * g * I.Gee[(size_t)i * p + j];
                for (int i = 0; i < p; ++i) f[i] = rhs[k][i] + gs * rhs[k][p + i];
                solved = lu_solve(p, H.data(), f.data(), q.data());
            }
            if (!solved) {
                if (o.init == RSR_INIT_MR || o.init == RSR_INIT_OBLIQUE) {
                    // (AU + g EU)^T (AU + g EU) q = (AU + g EU)^T b
                    for (int i = 0; i < p; ++i)
                        for (int j = 0; j < p; ++j)
                            H[(size_t)i * p + j] = I.Gaa[(size_t)i * p + j] +
                                                   g * (I.Gae[(size_t)i * p + j] + I.Gae[(size_t)j * p + i]) +
                                                   g * g * I.Gee[(size_t)i * p + j];
                    for (int i = 0; i < p; ++i) f[i] = rhs[k][i] + g * rhs[k][p + i];
                } else {
                    for (size_t t = 0; t < H.size(); ++t) H[t] = I.Ahat[t] + g * I.Ehat[t];
                    for (int i = 0; i < p; ++i) f[i] = rhs[k][i];
                }
                // Cholesky of the scaled p x p system; eigen pseudo-inverse when it is
                // numerically singular (rank guard)
                if (!spd_solve(p, H.data(), f.data(), q.data())) {
                    spd_pinv(p, H.data(), 1e-15, P);
                    matvec(p, p, P.data(), f.data(), q.data());
                }
            }
        });
        for (size_t k = 0; k < prin.size(); ++k) {
            SysHost &Y = *prin[k];
            const int p = c->inst[Y.inst]->p;
            const double g = Y.gamma;
            const std::vector<double> &q = qv[k];
            // x = U q ; r = b - [AU EU] [q; g q]
            InitGrp *G = nullptr;
            for (auto &e : grp)
                if (e.inst == Y.inst && e.b == Y.b) G = &e;
            if (!G) {
                grp.push_back(InitGrp{Y.inst, Y.b, {}, {}, {}});
                G = &grp.back();
            }
            G->sys.push_back(&Y);
            G->Qx.insert(G->Qx.end(), q.begin(), q.end());
            for (int i = 0; i < p; ++i) G->Qr.push_back(-q[i]);
            for (int i = 0; i < p; ++i) G->Qr.push_back(-g * q[i]);
        }
        size_t tot = 0;
        for (auto &e : grp) tot += 2 * e.sys.size() * (size_t)c->inst[e.inst]->n;
        WsMark mark(c);
        double *T = (double *)dscratch(c, c->d_tmp, sizeof(double) * tot);
        std::vector<CopyJob> out;
        for (auto &e : grp) {
            Instance &I = *c->inst[e.inst];
            const int p = I.p, m = (int)e.sys.size();
            const long n = I.n;
            double *Tx = T, *Tr = T + (size_t)m * n;
            T += (size_t)2 * m * n;
            cj.push_back(ComboJob{I.d_U.as<double>(), n, p, nullptr, p, Tx, n, m, 0.0, nullptr, 0, n});
            qs.push_back(e.Qx);
            cj.push_back(ComboJob{I.d_AE.as<double>(), n, 2 * p, nullptr, 2 * p, Tr, n, m, 0.0, e.b, 0, n});
            qs.push_back(e.Qr);
            for (int j = 0; j < m; ++j) {
                out.push_back(CopyJob{Tx + (size_t)j * n, e.sys[j]->x, n});
                out.push_back(CopyJob{Tr + (size_t)j * n, e.sys[j]->r, n});
            }
        }
        combo(c, cj, qs, s);
        copy_many(c, out, s);
    }
    // keep x_init for the correction g = x - x_init
    tm.reset(new StageTimer(c, s, 2));
    {
        std::vector<CopyJob> xc;
        for (auto *Y : sy) xc.push_back(CopyJob{Y->x, Y->xinit, Y->n});
        copy_many(c, xc, s);
    }
    {
        // ||r0|| only feeds the statistics: systems with a device slot defer the read-back
        std::vector<const double *> v;
        std::vector<long> n;
        std::vector<SysHost *> now;
        std::vector<GramJob> later;
        for (auto *Y : sy) {
            if (Y->r0sq_dev) {
                later.push_back(GramJob{Y->r, Y->n, 1, Y->r, Y->n, 1, Y->n, Y->r0sq_dev, 0});
            } else {
                v.push_back(Y->r);
                n.push_back(Y->n);
                now.push_back(Y);
            }
        }
        gram_to_device(c, later, s);
        if (!now.empty()) {
            auto rn = norms(c, v, n, s);
            for (size_t i = 0; i < now.size(); ++i) now[i]->relres_init = now[i]->bnorm > 0 ? rn[i] / now[i]->bnorm : 0.0;
        }
    }
    // local spaces and Galerkin correction
    tm.reset(new StageTimer(c, s, 3));
    build_local(c, sy, o, g_prev_shift, s);
    tm.reset(new StageTimer(c, s, 4));
    if (o.solver == RSR_SOLVER_MINRES) minres_local_basis(c, sy, s);
    else local_correction(c, sy, s);
    tm.reset();

    // CG with true-residual acceptance
    std::vector<SysHost *> todo;
    for (auto *Y : sy) {
        if (Y->bnorm == 0.0) {
            HIPCHK(launch_fill(Y->x, 0.0, Y->n, s));
            Y->done = true;
            Y->status = 1;
            Y->relres_true = 0.0;
        } else {
            todo.push_back(Y);
        }
    }
    for (int attempt = 0; attempt <= 3 && !todo.empty(); ++attempt) {
        Opts oo = o;
        tm.reset(new StageTimer(c, s, 5));
        if (o.solver == RSR_SOLVER_MINRES) run_minres(c, todo, oo, s);
        else if (c->ct) run_cg_host(c, todo, oo, s);
        else run_cg(c, todo, oo, s);
        tm.reset(new StageTimer(c, s, 6));
        // true residual rt = b - B x
        std::vector<ApplyJob> tj;
        for (auto *Y : todo) {
            tj.push_back(ApplyJob{Y->inst, 0, 1.0, Y->gamma, Y->x, Y->rt});
            Y->mvA++;
            Y->mvE++;
        }
        apply_jobs(c, tj, s);
        std::vector<ComboJob> rj;
        std::vector<std::vector<double>> rq;
        for (auto *Y : todo) {
            rj.push_back(ComboJob{Y->rt, Y->n, 1, nullptr, 1, Y->rt, Y->n, 1, 0.0, Y->b, Y->n, Y->n});
            rq.push_back(std::vector<double>{-1.0});
        }
        combo(c, rj, rq, s);
        std::vector<const double *> v;
        std::vector<long> n;
        for (auto *Y : todo) { v.push_back(Y->rt); n.push_back(Y->n); }
        auto rn = norms(c, v, n, s);
        std::vector<SysHost *> again;
        for (size_t i = 0; i < todo.size(); ++i) {
            SysHost &Y = *todo[i];
            Y.relres_true = rn[i] / Y.bnorm;
            if (Y.status < 0) fail((rsr_status)Y.status, Y.status == -4 ? "shifted matrix not SPD (p^T B p <= 0)"
                                                                         : "non-finite value in CG");
            if (Y.relres_true <= o.tol || Y.status == 2 || attempt == 3 || !std::isfinite(Y.relres_true)) {
                Y.done = true;
                if (!std::isfinite(Y.relres_true)) fail(RSR_E_NONFINITE, "non-finite residual");
            } else {
                // restart from the true residual
                HIPCHK(hipMemcpyAsync(Y.r, Y.rt, sizeof(double) * Y.n, hipMemcpyDeviceToDevice, s));
                Y.restarts++;
                again.push_back(&Y);
            }
        }
        if (!again.empty() && o.solver != RSR_SOLVER_MINRES) local_correction(c, again, s);
        todo.swap(again);
    }
}

void store_corrections(rsr_ctx *c, std::vector<SysHost *> &sy, hipStream_t s)
{
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    // columns for slots seen for the first time
    for (auto *Y : sy) {
        Instance &I = *c->inst[Y->inst];
        if (I.gcol.count(Y->slot)) continue;
        const int col = (int)I.gcol.size();
        if (c->wsa_base && col >= I.gpool_cols) continue;   // not reserved: not kept (no allocation)
        I.gcol[Y->slot] = col;
        if (col < I.gpool_cols) continue;
        const int cap = std::max({col + 1, 2 * I.gpool_cols, 8});
        DBuf nb;
        nb.ensure(sizeof(double) * (size_t)cap * I.n);
        if (I.gpool_cols > 0)
            HIPCHK(hipMemcpyAsync(nb.p, I.gpool.p, sizeof(double) * (size_t)I.gpool_cols * I.n,
                                  hipMemcpyDeviceToDevice, s));
        std::swap(nb.p, I.gpool.p);
        std::swap(nb.bytes, I.gpool.bytes);
        nb.release();   // drains the device, so the copy above has landed
        I.gpool_cols = cap;
    }
    for (auto *Y : sy) {
        Instance &I = *c->inst[Y->inst];
        if (!I.gslot(Y->slot)) continue;
        // g = x - xinit
        cj.push_back(ComboJob{Y->xinit, Y->n, 1, nullptr, 1, I.gslot(Y->slot), Y->n, 1, 0.0, Y->x, Y->n, Y->n});
        qs.push_back(std::vector<double>{-1.0});
    }
    combo(c, cj, qs, s);
}

void alloc_ws(rsr_ctx *c, std::vector<SysHost> &sys)
{
    // per system: r r1 w1 p0 p1 w xinit rt pa + W, Z (QMAX each)
    size_t tot = 0;
    for (auto &Y : sys) tot += (size_t)Y.n * (9 + 2 * QMAX) + 2 * QMAX + 64;
    double *p = (double *)dscratch(c, c->d_ws, sizeof(double) * tot);
    for (auto &Y : sys) {
        const long n = Y.n;
        Y.r = p; p += n;
        Y.r1 = p; p += n;
        Y.w1 = p; p += n;
        Y.p0 = p; p += n;
        Y.p1 = p; p += n;
        Y.w = p; p += n;
        Y.xinit = p; p += n;
        Y.rt = p; p += n;
        Y.pa = p; p += n;
        Y.cbuf = p; p += 2 * QMAX;
        Y.W = p; p += n * QMAX;
        Y.Z = p; p += n * QMAX;
        p += 32 - ((uintptr_t)p / 8) % 32;   // keep 256-byte alignment
    }
}

}  // namespace

// ================================================================ C ABI ==
namespace {
rsr_status guard(rsr_ctx *c, const std::function<void()> &f)
{
    if (!c) return RSR_E_ARG;
    try {
        c->err.clear();
        f();
        return RSR_OK;
    } catch (const Err &e) {
        c->err = e.msg;
        return e.st;
    } catch (const std::exception &e) {
        c->err = e.what();
        return RSR_E_ARG;
    }
}
}  // namespace

extern "C" {

const char *rsr_version(void) { return "rsr 0.1 gfx950 fp64"; }

rsr_status rsr_create(rsr_ctx **out, int dev)
{
    if (!out) return RSR_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return RSR_E_HIP;
    if (dev < 0 || dev >= ndev) return RSR_E_ARG;
    rsr_ctx *c = new rsr_ctx();
    c->dev = dev;
    c->hprof = getenv("RSR_HOST_PROF") != nullptr;
    if (const char *t = getenv("RSR_BARRIER_TIMEOUT_US")) {   // bound on a grid-barrier wait (default 30 s)
        const double us = atof(t);
        if (us >= 0.0 && us < 3.6e9) c->bar_timeout_s = us * 1e-6;
    }
    rsr_status st = guard(c, [&] {
        set_device(c);
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        c->n_cu = prop.multiProcessorCount;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            c->wall_khz = khz;
        HIPCHK(hipEventCreate(&c->ev0));
        HIPCHK(hipEventCreate(&c->ev1));
        // the static scratch's address on this device, once per device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch_ptr.find(dev);
        if (it == g_scratch_ptr.end()) {
            void *ptr = nullptr;
            HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) fail(RSR_E_HIP, "no device address for the static scratch");
            it = g_scratch_ptr.emplace(dev, ptr).first;
        }
        c->scratch_dev = it->second;
    });
    if (st != RSR_OK) {
        delete c;
        return st;
    }
    *out = c;
    return RSR_OK;
}

void rsr_destroy(rsr_ctx *c)
{
    if (!c) return;
    if (c->hprof)
        fprintf(stderr, "[rsr host stages] ms: bnorm %.1f init %.1f r0 %.1f local %.1f correct %.1f cg %.1f "
                        "true-res %.1f store %.1f\n", c->hprof_ms[0], c->hprof_ms[1], c->hprof_ms[2], c->hprof_ms[3],
                c->hprof_ms[4], c->hprof_ms[5], c->hprof_ms[6], c->hprof_ms[7]);
    (void)hipSetDevice(c->dev);
    (void)hipDeviceSynchronize();
    for (auto &p : c->inst) {
        Instance &I = *p;
        I.d_fy.release(); I.d_fx.release(); I.d_psf.release(); I.d_wh.release(); I.d_wv.release(); I.d_band.release();
        I.d_rk.release();
        I.d_U.release(); I.d_AE.release();
        I.ritz[0].buf.release(); I.ritz[1].buf.release();
        I.gpool.release();
    }
    for (DBuf *b : {&c->d_inst, &c->d_jobs, &c->d_gram_scratch, &c->d_small, &c->d_sys, &c->d_partA, &c->d_partB,
                    &c->d_ctl, &c->d_out, &c->d_ws, &c->d_tmp, &c->d_dbg, &c->ar_dev, &c->d_rcC, &c->d_rcQ, &c->d_rcR, &c->d_rcT,
                    &c->d_lz, &c->d_lzc, &c->d_lzr, &c->d_aux, &c->d_corr, &c->d_r0sq, &c->d_grad})
        b->release();
    if (c->ar_host) (void)hipHostFree(c->ar_host);
    if (c->rb_host) (void)hipHostFree(c->rb_host);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

const char *rsr_last_error(const rsr_ctx *c) { return c ? c->err.c_str() : "null context"; }

rsr_status rsr_set_operators(rsr_ctx *c, int n_inst, const rsr_instance *in, void *stream)
{
    return guard(c, [&] {
        if (n_inst <= 0 || !in) fail(RSR_E_ARG, "n_inst must be positive");
        for (int i = 0; i < n_inst; ++i) {
            const rsr_instance &r = in[i];
            if (r.ny <= 0 || r.nx <= 0 || r.sy <= 0 || r.sx <= 0 || !(r.sy & 1) || !(r.sx & 1) || !r.psf_host)
                fail(RSR_E_ARG, "instance " + std::to_string(i) + ": sizes must be positive and the PSF odd");
            if (r.sy > 63 || r.sx > 63) fail(RSR_E_ARG, "PSF larger than 63 x 63");
            if ((long)r.ny * r.nx >= (1L << 31)) fail(RSR_E_ARG, "image of 2^31 pixels or more");
            for (int k = 0; k < r.sy * r.sx; ++k)
                if (!std::isfinite(r.psf_host[k])) fail(RSR_E_NONFINITE, "non-finite PSF entry");
        }
        set_device(c);
        hipStream_t s = S(stream);
        sync(c, s);
        for (auto &p : c->inst) {
            p->d_fy.release(); p->d_fx.release(); p->d_psf.release(); p->d_wh.release(); p->d_wv.release();
            p->d_band.release();
            p->d_rk.release();
            p->d_U.release(); p->d_AE.release();
            p->ritz[0].buf.release(); p->ritz[1].buf.release();
            p->gpool.release();
            p->d_cs.release();
        }
        c->inst.clear();
        c->ct = false;
        for (int i = 0; i < n_inst; ++i) {
            std::unique_ptr<Instance> I(new Instance());
            const rsr_instance &r = in[i];
            I->ny = r.ny; I->nx = r.nx; I->sy = r.sy; I->sx = r.sx;
            I->n = (long)r.ny * r.nx;
            I->psf.assign(r.psf_host, r.psf_host + r.sy * r.sx);
            factor_psf(*I);
            default_tile(*I);
            I->d_psf.ensure(sizeof(double) * I->psf.size());
            HIPCHK(hipMemcpy(I->d_psf.p, I->psf.data(), sizeof(double) * I->psf.size(), hipMemcpyHostToDevice));
            if (I->rank) {
                I->d_rk.ensure(sizeof(double) * I->rk.size());
                HIPCHK(hipMemcpy(I->d_rk.p, I->rk.data(), sizeof(double) * I->rk.size(), hipMemcpyHostToDevice));
            }
            if (I->sep == 1) {
                I->d_fy.ensure(sizeof(double) * I->ssq);
                I->d_fx.ensure(sizeof(double) * I->ssq);
                HIPCHK(hipMemcpy(I->d_fy.p, I->fy.data(), sizeof(double) * I->ssq, hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(I->d_fx.p, I->fx.data(), sizeof(double) * I->ssq, hipMemcpyHostToDevice));
                I->d_band.ensure(sizeof(double) * I->band.size());
                HIPCHK(hipMemcpy(I->d_band.p, I->band.data(), sizeof(double) * I->band.size(), hipMemcpyHostToDevice));
            }
            I->d_wh.ensure(sizeof(double) * I->n);
            I->d_wv.ensure(sizeof(double) * I->n);
            HIPCHK(launch_copy_weights(nullptr, nullptr, I->d_wh.as<double>(), I->d_wv.as<double>(), I->ny, I->nx, s));
            c->inst.push_back(std::move(I));
        }
        upload_inst(c);
        sync(c, s);
    });
}

rsr_status rsr_set_ct_operators(rsr_ctx *c, int n_inst, const rsr_ct_instance *in, void *stream)
{
    return guard(c, [&] {
        if (n_inst <= 0 || !in) fail(RSR_E_ARG, "n_inst must be positive");
        for (int i = 0; i < n_inst; ++i) {
            const rsr_ct_instance &r = in[i];
            const std::string who = "tomography instance " + std::to_string(i);
            if (r.ny <= 0 || r.nx <= 0 || r.n_angles <= 0 || r.n_det <= 0 || !r.angles_host)
                fail(RSR_E_ARG, who + ": sizes must be positive and the angles given");
            if (!(r.spacing > 0.0) || !std::isfinite(r.spacing)) fail(RSR_E_ARG, who + ": spacing must be positive");
            if ((long)r.ny * r.nx >= (1L << 31) || (long)r.n_angles * r.n_det >= (1L << 31))
                fail(RSR_E_ARG, who + ": image or sinogram of 2^31 values or more");
            for (int a = 0; a < r.n_angles; ++a)
                if (!std::isfinite(r.angles_host[a])) fail(RSR_E_ARG, who + ": angles must be finite");
        }
        set_device(c);
        hipStream_t s = S(stream);
        sync(c, s);
        for (auto &p : c->inst) {
            p->d_fy.release(); p->d_fx.release(); p->d_psf.release(); p->d_wh.release(); p->d_wv.release();
            p->d_band.release();
            p->d_rk.release();
            p->d_U.release(); p->d_AE.release();
            p->ritz[0].buf.release(); p->ritz[1].buf.release();
            p->gpool.release();
            p->d_cs.release();
        }
        c->inst.clear();
        c->ct = true;
        for (int i = 0; i < n_inst; ++i) {
            std::unique_ptr<Instance> I(new Instance());
            const rsr_ct_instance &r = in[i];
            I->ny = r.ny; I->nx = r.nx;
            I->n = (long)r.ny * r.nx;
            I->ct = true;
            I->na = r.n_angles;
            I->nd = r.n_det;
            I->spacing = r.spacing;
            // a 1 x 1 PSF keeps the stencil descriptor well formed; no stencil
            // kernel runs on a tomography instance
            I->psf.assign(1, 1.0);
            I->sy = I->sx = 1;
            default_tile(*I);
            I->d_psf.ensure(sizeof(double));
            HIPCHK(hipMemcpy(I->d_psf.p, I->psf.data(), sizeof(double), hipMemcpyHostToDevice));
            // per angle: cos, sin and the reciprocals of the ray direction (-sin, cos), 0 for a 0 component
            std::vector<double> cs(4 * (size_t)r.n_angles);
            for (int a = 0; a < r.n_angles; ++a) {
                const double co = std::cos(r.angles_host[a]), si = std::sin(r.angles_host[a]);
                cs[4 * a] = co;
                cs[4 * a + 1] = si;
                cs[4 * a + 2] = si != 0.0 ? 1.0 / -si : 0.0;
                cs[4 * a + 3] = co != 0.0 ? 1.0 / co : 0.0;
            }
            I->d_cs.ensure(sizeof(double) * cs.size());
            HIPCHK(hipMemcpy(I->d_cs.p, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice));
            I->d_wh.ensure(sizeof(double) * I->n);
            I->d_wv.ensure(sizeof(double) * I->n);
            HIPCHK(launch_copy_weights(nullptr, nullptr, I->d_wh.as<double>(), I->d_wv.as<double>(), I->ny, I->nx, s));
            c->inst.push_back(std::move(I));
        }
        upload_inst(c);
        // ||C||_F: per-ray sums of squared intersection lengths, summed on the host in ray order
        size_t rays = 0;
        for (auto &p : c->inst) rays = std::max(rays, (size_t)p->na * p->nd);
        DBuf sq;
        sq.ensure(sizeof(double) * rays);
        std::vector<double> h(rays);
        for (int i = 0; i < n_inst; ++i) {
            Instance &I = *c->inst[i];
            std::vector<CtJob> one{CtJob{i, 5, 0.0, 0.0, nullptr, nullptr, sq.as<double>()}};
            CtJob *dj = upload(c, c->d_jobs, one, s);
            HIPCHK(launch_ct_fwd(c->d_ctinst.as<CtDev>(), dj, 1, I.na * I.nd, s));
            read_back(c, {ReadBack{h.data(), sq.p, sizeof(double) * I.na * I.nd}}, s);
            double f = 0.0;
            for (long k = 0; k < (long)I.na * I.nd; ++k) f += h[k];
            if (!(f > 0.0)) {
                sq.release();
                fail(RSR_E_ARG, "tomography instance " + std::to_string(i) + ": no ray meets the image");
            }
            I.ct_scale = 1.0 / std::sqrt(f);
        }
        sq.release();
        upload_inst(c);
        sync(c, s);
    });
}

rsr_status rsr_update_weights(rsr_ctx *c, int ii, const double *wh, const double *wv, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (!wh || !wv) fail(RSR_E_ARG, "null weights");
        set_device(c);
        HIPCHK(launch_copy_weights(wh, wv, I.d_wh.as<double>(), I.d_wv.as<double>(), I.ny, I.nx, S(stream)));
        I.ae_valid = false;
    });
}

rsr_status rsr_weights_from_image(rsr_ctx *c, int ii, const double *x, double beta, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (!x) fail(RSR_E_ARG, "null image");
        if (!(beta > 0.0) || !std::isfinite(beta)) fail(RSR_E_ARG, "beta must be positive");
        set_device(c);
        HIPCHK(launch_weights(x, beta, I.d_wh.as<double>(), I.d_wv.as<double>(), I.ny, I.nx, S(stream)));
        I.ae_valid = false;
    });
}

rsr_status rsr_weights_edge_rule(rsr_ctx *c, int ii, const double *x, double p, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (!x) fail(RSR_E_ARG, "null image");
        if (!(p > 0.0) || !std::isfinite(p)) fail(RSR_E_ARG, "exponent p must be positive");
        set_device(c);
        c->d_aux.ensure(sizeof(double) * edge_rule_parts());
        HIPCHK(launch_edge_rule(x, I.d_wh.as<double>(), I.d_wv.as<double>(), I.ny, I.nx, p, c->d_aux.as<double>(),
                                S(stream)));
        I.ae_valid = false;
    });
}

// Corner of the discrete L-curve (Sec. 2.1): the interior point of largest
// signed curvature of (u, v) = (log rho, log eta) as functions of
// t = log lambda = (log gamma) / 2.  First and second derivatives are the
// three-point finite differences on the (possibly uneven) t grid; the curvature
// is (u' v'' - u'' v') / (u'^2 + v'^2)^(3/2), positive where the curve turns
// from falling steeply (small lambda) to running flat (large lambda).
// Returns -1 when fewer than three points or no finite curvature exist.
static int lcurve_corner(int m, const double *gam, const double *rho, const double *eta, double *kappa)
{
    int best = -1;
    double kb = -INFINITY;
    for (int i = 0; i < m; ++i) {
        if (kappa) kappa[i] = NAN;
        if (i == 0 || i == m - 1) continue;
        const double t0 = 0.5 * std::log(gam[i - 1]), t1 = 0.5 * std::log(gam[i]), t2 = 0.5 * std::log(gam[i + 1]);
        const double hm = t1 - t0, hp = t2 - t1, den = hm * hp * (hm + hp);
        const double u0 = std::log(rho[i - 1]), u1 = std::log(rho[i]), u2 = std::log(rho[i + 1]);
        const double v0 = std::log(eta[i - 1]), v1 = std::log(eta[i]), v2 = std::log(eta[i + 1]);
        const double du = (hm * hm * u2 - hp * hp * u0 - (hm * hm - hp * hp) * u1) / den;
        const double dv = (hm * hm * v2 - hp * hp * v0 - (hm * hm - hp * hp) * v1) / den;
        const double ddu = 2.0 * (hm * u2 - (hm + hp) * u1 + hp * u0) / den;
        const double ddv = 2.0 * (hm * v2 - (hm + hp) * v1 + hp * v0) / den;
        const double k = (du * ddv - ddu * dv) / std::pow(du * du + dv * dv, 1.5);
        if (kappa) kappa[i] = k;
        if (std::isfinite(k) && k > kb) {
            kb = k;
            best = i;
        }
    }
    return best;
}

rsr_status rsr_lcurve(rsr_ctx *c, int ii, int m, const double *gammas, const double *X, long ld_x, const double *d,
                      double *rho, double *eta, double *kappa, int *corner, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (I.ct) fail(RSR_E_ARG, "the L-curve kernel is for deblurring instances");
        if (m <= 0 || !gammas || !X || !d || !rho || !eta || !corner) fail(RSR_E_ARG, "null argument or m <= 0");
        if (m > 1 && ld_x < I.n) fail(RSR_E_ARG, "ld_x smaller than ny*nx");
        for (int i = 0; i < m; ++i) {
            if (!(gammas[i] > 0.0) || !std::isfinite(gammas[i])) fail(RSR_E_ARG, "gamma must be positive");
            if (i > 0 && !(gammas[i] > gammas[i - 1])) fail(RSR_E_ARG, "gammas must increase");
        }
        set_device(c);
        hipStream_t s = S(stream);
        const int nb = lcurve_parts(I.n);
        c->d_aux.ensure(sizeof(double) * 2 * (size_t)m * nb);
        HIPCHK(launch_lcurve(c->d_inst.as<InstDev>(), ii, I.n, m, X, m > 1 ? ld_x : I.n, d, c->d_aux.as<double>(), s));
        std::vector<double> h((size_t)2 * m * nb);
        read_back(c, {ReadBack{h.data(), c->d_aux.p, sizeof(double) * h.size()}}, s);
        for (int i = 0; i < m; ++i) {
            double sr = 0.0, se = 0.0;
            for (int k = 0; k < nb; ++k) {
                sr += h[2 * ((size_t)i * nb + k)];
                se += h[2 * ((size_t)i * nb + k) + 1];
            }
            rho[i] = std::sqrt(sr);
            eta[i] = std::sqrt(se);
        }
        *corner = lcurve_corner(m, gammas, rho, eta, kappa);
    });
}

rsr_status rsr_get_weights(rsr_ctx *c, int ii, double *wh, double *wv, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        set_device(c);
        if (wh) HIPCHK(hipMemcpyAsync(wh, I.d_wh.p, sizeof(double) * I.n, hipMemcpyDeviceToDevice, S(stream)));
        if (wv) HIPCHK(hipMemcpyAsync(wv, I.d_wv.p, sizeof(double) * I.n, hipMemcpyDeviceToDevice, S(stream)));
    });
}

rsr_status rsr_apply(rsr_ctx *c, int ii, int op, double gamma, const double *v, double *y, int n_vec, long ld,
                     void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (!v || !y || n_vec <= 0) fail(RSR_E_ARG, "null vectors or n_vec <= 0");
        if (!std::isfinite(gamma)) fail(RSR_E_ARG, "gamma not finite");
        if (I.ct) {
            // K and K^T read or write sinograms: their columns hold the larger of the two sizes
            const long big = (op == RSR_OP_K || op == RSR_OP_KT) ? std::max(I.n, (long)I.na * I.nd) : I.n;
            if (n_vec > 1 && ld < big) fail(RSR_E_ARG, "ld smaller than the image (or, for K and K^T, sinogram) size");
            if (ld <= 0) ld = big;
            if (op != RSR_OP_B && op != RSR_OP_A && op != RSR_OP_E && op != RSR_OP_K && op != RSR_OP_KT)
                fail(RSR_E_ARG, "unknown operator");
            set_device(c);
            hipStream_t s = S(stream);
            std::vector<ApplyJob> jobs(n_vec);
            const double cA = op == RSR_OP_E ? 0.0 : 1.0;
            const double cE = op == RSR_OP_B ? gamma : op == RSR_OP_E ? 1.0 : 0.0;
            const int jop = op == RSR_OP_K ? 3 : op == RSR_OP_KT ? 4 : 0;
            for (int j = 0; j < n_vec; ++j) jobs[j] = ApplyJob{ii, jop, cA, cE, v + j * ld, y + j * ld};
            ct_apply_jobs(c, jobs, s);
            sync(c, s);
            return;
        }
        if (n_vec > 1 && ld < I.n) fail(RSR_E_ARG, "ld smaller than ny*nx");
        if (ld <= 0) ld = I.n;
        set_device(c);
        hipStream_t s = S(stream);
        if (op == RSR_OP_K || op == RSR_OP_KT) {
            std::vector<ApplyJob> jobs(n_vec);
            for (int j = 0; j < n_vec; ++j) jobs[j] = ApplyJob{ii, op, 0.0, 0.0, v + j * ld, y + j * ld};
            ApplyJob *dj = upload(c, c->d_jobs, jobs, s);
            HIPCHK(launch_blur(c->d_inst.as<InstDev>(), c->h_inst[ii], dj, n_vec, s));
            sync(c, s);
            return;
        }
        double cA = 0.0, cE = 0.0;
        if (op == RSR_OP_B) { cA = 1.0; cE = gamma; }
        else if (op == RSR_OP_A) cA = 1.0;
        else if (op == RSR_OP_E) cE = 1.0;
        else fail(RSR_E_ARG, "unknown operator");
        apply_op(c, ii, cA, cE, v, ld, y, ld, n_vec, s);
    });
}

// Principal recycle space (Alg. 1, Sec. 5.2): see rsr_set_recycle_space.  Returns
// the dimension kept.
int set_recycle_space_impl(rsr_ctx *c, int ii, const double *U_raw, long ld, int ncols, int n_retain,
                           double gamma_retain, int p_max, double cond_max, hipStream_t s)
{
    Instance &I = get_inst(c, ii);
    if (ncols < 0 || n_retain < 0 || p_max < 0) fail(RSR_E_ARG, "negative sizes");
    if (ncols > 0 && (!U_raw || ld < I.n)) fail(RSR_E_ARG, "U_raw null or ld < ny*nx");
    if (!(cond_max > 1.0)) fail(RSR_E_ARG, "cond_max must exceed 1");
    set_device(c);
    const long n = I.n;
    const int nr = std::min(n_retain, I.p);
    const int m = nr + ncols;
    if (m == 0 || p_max == 0) {
        I.p = 0;
        I.ae_valid = false;
        return 0;
    }
    // Buffers are sized for the largest space this call allows (p_max kept
    // columns, p_max + ncols candidates), so that a space that grows over the
    // outer steps does not reallocate (a free drains the device).  U and
    // [AU EU] are resized only where they are rewritten: the candidates read U.
    const size_t pcap = (size_t)std::max(p_max, 1);
    // candidate block C = [U W~(:, 1:nr), U_raw]
    DBuf &Cb = c->d_rcC;
    Cb.ensure(sizeof(double) * std::max((size_t)m, pcap + ncols) * n);
    double *C = Cb.as<double>();
    if (nr > 0) {
        const int p = I.p;
        std::vector<double> w, V;
        retained_eig(I, gamma_retain, w, V);
        std::vector<double> Wt((size_t)p * nr);
        for (int j = 0; j < nr; ++j)
            for (int i = 0; i < p; ++i) Wt[(size_t)j * p + i] = V[(size_t)i * p + j];
        combo(c, {ComboJob{I.d_U.as<double>(), n, p, nullptr, p, C, n, nr, 0.0, nullptr, 0, n}}, {Wt}, s);
    }
    if (ncols > 0 && ld == n) {
        HIPCHK(hipMemcpyAsync(C + (size_t)nr * n, U_raw, sizeof(double) * ncols * n, hipMemcpyDeviceToDevice, s));
    } else {
        std::vector<CopyJob> uc;
        for (int j = 0; j < ncols; ++j) uc.push_back(CopyJob{U_raw + (size_t)j * ld, C + (size_t)(nr + j) * n, n});
        copy_many(c, uc, s);
    }
    // Algorithm 1 (Sec. 5.1): the left singular vectors of C with
    // sigma_1 / sigma_i < cond_max, at most p_max of them (largest first).  The
    // skinny SVD is taken as C = Q R followed by an SVD of the small R on the
    // host: with R = Ur diag(sigma) Vr^T, C = (Q Ur) diag(sigma) Vr^T.  Q is
    // built in levels.  Each level takes the eigenvectors of the Gram matrix of
    // the current residual block Z (Z = C at the first level) whose eigenvalues
    // lie within 1e12 of the level's largest, scales them to orthonormal
    // columns, orthogonalises those against the earlier levels and by Cholesky
    // QR, appends them to Q, and replaces Z by C projected twice onto the
    // complement of Range(Q).  A level resolves singular values down to about
    // 1e-6 of its own largest, so two levels reach 1e-12 sigma_1; the loop ends
    // once Z holds nothing above a tenth of sigma_1 / cond_max.  R = Q^T C is
    // then accurate to rounding of sigma_1, and its one-sided Jacobi SVD applies
    // the threshold.
    DBuf &Qb = c->d_rcQ, &Zb = c->d_rcR, &Tb = c->d_rcT;
    const size_t ccap = std::max((size_t)m, pcap + ncols) * n;
    Qb.ensure(sizeof(double) * ccap);
    Zb.ensure(sizeof(double) * ccap);
    Tb.ensure(sizeof(double) * ccap);
    double *Q = Qb.as<double>(), *Zr = Zb.as<double>(), *Tm = Tb.as<double>();
    // C_X^T C_Y (row-major a x b) and Y = beta Y (or Y0) + X Qc (Qc column-major a x b)
    auto gram1 = [&](const double *X, int a, const double *Y, int b) {
        return gram(c, {GramJob{X, n, a, Y, n, b, n, nullptr, 0}}, s)[0];
    };
    auto comb1 = [&](const double *X, int a, const std::vector<double> &Qc, double *Y, int b, double beta,
                     const double *Y0) {
        combo(c, {ComboJob{X, n, a, nullptr, a, Y, n, b, beta, Y0, n, n}}, {Qc}, s);
    };
    int r = 0;
    double lam1 = 0.0;
    const double *Z = C;
    for (int level = 0; level < 4 && r < m; ++level) {
        std::vector<double> Gm = gram1(Z, m, Z, m), w, V;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) Gm[(size_t)j * m + i] = Gm[(size_t)i * m + j];
        sym_eig(m, Gm.data(), w, V);
        const double lmax = w.empty() ? 0.0 : w.back();
        if (level == 0) {
            if (!std::isfinite(lmax)) fail(RSR_E_NONFINITE, "non-finite recycle candidates");
            if (!(lmax > 0.0)) fail(RSR_E_RANK, "recycle candidates are all zero");
            lam1 = lmax;
        } else if (!(lmax > 1e-2 * lam1 / (cond_max * cond_max)) || !(lmax > 1e-32 * lam1)) {
            break;   // nothing left above the threshold
        }
        std::vector<int> idx;
        for (int k = m - 1; k >= 0 && r + (int)idx.size() < m; --k)
            if (w[k] > 1e-12 * lmax && w[k] > 1e-32 * lam1) idx.push_back(k);
        const int kk = (int)idx.size();
        if (kk == 0) break;
        std::vector<double> T((size_t)m * kk);   // column-major m x kk
        for (int j = 0; j < kk; ++j) {
            const double sc = 1.0 / std::sqrt(w[idx[j]]);
            for (int i = 0; i < m; ++i) T[(size_t)j * m + i] = V[(size_t)i * m + idx[j]] * sc;
        }
        comb1(Z, m, T, Tm, kk, 0.0, nullptr);
        if (r > 0) {   // Tm -= Q (Q^T Tm)
            const std::vector<double> Sq = gram1(Q, r, Tm, kk);
            std::vector<double> Sc((size_t)r * kk);
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < kk; ++j) Sc[(size_t)j * r + i] = -Sq[(size_t)i * kk + j];
            comb1(Q, r, Sc, Tm, kk, 1.0, nullptr);
        }
        // Cholesky QR of the nearly orthonormal block (same span); the Gram
        // route again should the factorisation be refused
        std::vector<double> G2 = gram1(Tm, kk, Tm, kk), T2;
        int kq = kk;
        if (!chol_qr_factor(kk, G2.data(), T2)) {
            std::vector<double> w2, V2;
            sym_eig(kk, G2.data(), w2, V2);
            std::vector<int> id2;
            for (int k = kk - 1; k >= 0; --k)
                if (w2[k] > 1e-8 * w2.back()) id2.push_back(k);
            kq = (int)id2.size();
            T2.assign((size_t)kk * kq, 0.0);
            for (int j = 0; j < kq; ++j)
                for (int i = 0; i < kk; ++i) T2[(size_t)j * kk + i] = V2[(size_t)i * kk + id2[j]] / std::sqrt(w2[id2[j]]);
        }
        if (kq == 0) break;
        comb1(Tm, kk, T2, Q + (size_t)r * n, kq, 0.0, nullptr);
        r += kq;
        // Z = C - Q (Q^T C), then once more against Q
        for (int pass = 0; pass < 2; ++pass) {
            const double *X = pass == 0 ? C : Zr;
            const std::vector<double> Sq = gram1(Q, r, X, m);
            std::vector<double> Sc((size_t)r * m);
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < m; ++j) Sc[(size_t)j * r + i] = -Sq[(size_t)i * m + j];
            if (pass == 0) comb1(Q, r, Sc, Zr, m, 0.0, C);
            else comb1(Q, r, Sc, Zr, m, 1.0, nullptr);
        }
        Z = Zr;
    }
    // R = Q^T C, its SVD on the host, and U = Q Ur(:, kept)
    const std::vector<double> Rm = gram1(Q, r, C, m);
    std::vector<double> sig, Ur;
    left_svd_jacobi(r, m, Rm.data(), sig, Ur);
    int keep = 0;
    while (keep < r && keep < p_max && sig[keep] > 0.0 && sig[0] / sig[keep] < cond_max) ++keep;
    if (keep == 0) fail(RSR_E_RANK, "recycle space empty after stabilisation");
    I.d_U.ensure(sizeof(double) * std::max((size_t)keep, pcap) * n);
    comb1(Q, r, std::vector<double>(Ur.begin(), Ur.begin() + (size_t)r * keep), I.d_U.as<double>(), keep, 0.0,
          nullptr);
    const int p = keep;
    I.p = p;
    // A U and E U (p applications each), then the small blocks
    I.d_AE.ensure(sizeof(double) * (size_t)2 * std::max((size_t)p, pcap) * n);
    double *AU = I.d_AE.as<double>(), *EU = AU + (size_t)p * n;
    apply_op(c, ii, 1.0, 0.0, I.d_U.as<double>(), n, AU, n, p, s);
    apply_op(c, ii, 0.0, 1.0, I.d_U.as<double>(), n, EU, n, p, s);
    auto blocks = gram(c,
                       {GramJob{I.d_U.as<double>(), n, p, AU, n, p, n, nullptr, 0},
                        GramJob{I.d_U.as<double>(), n, p, EU, n, p, n, nullptr, 0},
                        GramJob{AU, n, p, AU, n, p, n, nullptr, 0}, GramJob{AU, n, p, EU, n, p, n, nullptr, 0},
                        GramJob{EU, n, p, EU, n, p, n, nullptr, 0}},
                       s);
    auto sym = [p](std::vector<double> M) {
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) {
                const double v = 0.5 * (M[(size_t)i * p + j] + M[(size_t)j * p + i]);
                M[(size_t)i * p + j] = M[(size_t)j * p + i] = v;
            }
        return M;
    };
    I.u_version += 1;
    I.Ahat = sym(blocks[0]);
    I.Ehat = sym(blocks[1]);
    I.Gaa = sym(blocks[2]);
    I.Gae = blocks[3];
    I.Gee = sym(blocks[4]);
    I.ae_valid = true;
    return p;
}

rsr_status rsr_set_recycle_space(rsr_ctx *c, int ii, const double *U_raw, long ld, int ncols, int n_retain,
                                 double gamma_retain, int p_max, double cond_max, int *p_kept, void *stream)
{
    return guard(c, [&] {
        if (p_kept) *p_kept = 0;
        const int p = set_recycle_space_impl(c, ii, U_raw, ld, ncols, n_retain, gamma_retain, p_max, cond_max,
                                             S(stream));
        if (p_kept) *p_kept = p;
    });
}

// Principal space from the CG-Lanczos data of one or two solves (Sec. 5.1: the
// representative systems' solutions and the Ritz vectors of their Krylov
// spaces seed U, eq. widetildeU).  With CG coefficients alpha_j and
// beta_j = rho_{j+1}/rho_j, the residuals v_j = r_j / ||r_j|| satisfy
// B V = V T + (residual) e_m^T, with T tridiagonal:
//   T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},   T_j,j+1 = -sqrt(beta_j)/alpha_j.
// For each captured system the k eigenvectors of T with the smallest Ritz values
// give the Ritz vectors V s; the candidates [x_1, .., x_s, V_1, .., V_s] go
// through Algorithm 1 (at most seed_p columns) to U (with AU, EU, the blocks).
// Returns the principal dimension (0 if no system recorded two steps).
int seed_from_lanczos(rsr_ctx *c, const std::vector<const SysHost *> &ys, long nlz, int seed_p, hipStream_t s)
{
    const int ns = (int)ys.size();
    if (ns == 0 || seed_p <= 0) return 0;
    const long n = ys[0]->n;
    // Ritz vectors per system: the seed_p - ns columns left beside the solutions, shared out
    const int kall = std::max(0, seed_p - ns);
    std::vector<std::vector<double>> Qs(ns);
    std::vector<int> ms(ns, 0), ks(ns, 0);
    int tot = ns;
    for (int i = 0; i < ns; ++i) {
        const SysHost &Y = *ys[i];
        const int m = (int)std::min<long>(nlz, (long)Y.lz_its - 1);   // steps with alpha and beta recorded
        if (m < 2) continue;
        std::vector<double> co((size_t)3 * nlz);
        read_back(c, {ReadBack{co.data(), Y.lzc, sizeof(double) * co.size()}}, s);
        const double *al = co.data(), *be = co.data() + nlz, *rho = co.data() + 2 * nlz;
        bool good = true;
        std::vector<double> T((size_t)m * m, 0.0);
        for (int j = 0; j < m && good; ++j) {
            if (!(al[j] > 0.0) || !(rho[j] > 0.0)) good = false;
            T[(size_t)j * m + j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
            if (j + 1 < m) T[(size_t)j * m + j + 1] = T[(size_t)(j + 1) * m + j] = -std::sqrt(be[j]) / al[j];
        }
        if (!good) continue;
        std::vector<double> w, V;
        sym_eig(m, T.data(), w, V);
        const int k = std::min(kall / ns + (i < kall % ns ? 1 : 0), m);
        std::vector<double> Q((size_t)m * k);   // column-major m x k: Ritz coefficients over the raw residuals
        for (int q = 0; q < k; ++q)
            for (int j = 0; j < m; ++j) Q[(size_t)q * m + j] = V[(size_t)j * m + q] / std::sqrt(rho[j]);
        Qs[i] = Q;
        ms[i] = m;
        ks[i] = k;
        tot += k;
    }
    bool any = false;
    for (int i = 0; i < ns; ++i) any = any || ms[i] > 0;
    if (!any) return 0;
    // candidates [x_1 .. x_ns, Ritz vectors of system 1, of system 2, ...]
    c->d_lzr.ensure(sizeof(double) * (size_t)tot * n);
    double *cand = c->d_lzr.as<double>();
    std::vector<CopyJob> cp;
    for (int i = 0; i < ns; ++i) cp.push_back(CopyJob{ys[i]->x, cand + (size_t)i * n, n});
    copy_many(c, cp, s);
    std::vector<ComboJob> cj;
    std::vector<std::vector<double>> qs;
    size_t col = ns;
    for (int i = 0; i < ns; ++i) {
        if (ks[i] == 0) continue;
        cj.push_back(ComboJob{ys[i]->lz, n, ms[i], nullptr, ms[i], cand + col * n, n, ks[i], 0.0, nullptr, 0, n});
        qs.push_back(Qs[i]);
        col += ks[i];
    }
    combo(c, cj, qs, s);
    return set_recycle_space_impl(c, ys[0]->inst, cand, n, tot, 0, 0.0, seed_p, 1e10, s);
}

// Correction space of the principal-space update (Sec. 5.2, eq. delta times
// gamma): at most max_steps CG steps on (A + gamma E_k) dx = gamma (E_k - E_{k-1}) x_prev
// from dx = 0, recording the first n_kry residuals; V = [dx, r_j / ||r_j||].
rsr_status rsr_correction_space(rsr_ctx *c, int ii, const double *x_prev, const double *wh_prev,
                                const double *wv_prev, double gamma, int max_steps, int n_kry, double *V, long ld,
                                int *n_out, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (!x_prev || !wh_prev || !wv_prev || !V || !n_out) fail(RSR_E_ARG, "null argument");
        *n_out = 0;
        if (I.ct) fail(RSR_E_ARG, "the correction space runs the persistent CG kernel (deblurring instances)");
        if (!(gamma > 0.0) || !std::isfinite(gamma)) fail(RSR_E_ARG, "gamma must be positive");
        if (max_steps < 1 || n_kry < 0 || n_kry > max_steps) fail(RSR_E_ARG, "need 1 <= max_steps, 0 <= n_kry <= max_steps");
        if (n_kry > 0 && ld < I.n) fail(RSR_E_ARG, "ld smaller than ny*nx");
        set_device(c);
        hipStream_t s = S(stream);
        const long n = I.n;
        c->d_corr.ensure(sizeof(double) * n);
        HIPCHK(launch_weight_delta(x_prev, I.d_wh.as<double>(), I.d_wv.as<double>(), wh_prev, wv_prev, gamma, I.ny,
                                   I.nx, c->d_corr.as<double>(), s));
        std::vector<SysHost> sys(1);
        SysHost &Y = sys[0];
        Y.inst = ii;
        Y.slot = -1;
        Y.gamma = gamma;
        Y.n = n;
        Y.b = c->d_corr.as<double>();
        Y.x = V;
        alloc_ws(c, sys);
        c->bnorm_cache.clear();
        c->rhs_cache.clear();
        if (n_kry > 0) {
            c->d_lz.ensure(sizeof(double) * (size_t)n_kry * n);
            c->d_lzc.ensure(sizeof(double) * (size_t)3 * n_kry);
            HIPCHK(launch_fill(c->d_lzc.as<double>(), 0.0, 3 * (long)n_kry, s));
            Y.lz = c->d_lz.as<double>();
            Y.lzc = c->d_lzc.as<double>();
            Y.nlz = n_kry;
        }
        c->last_cg_ms = 0.0;
        c->last_launches = 0;
        c->last_items = 0;
        // plain CG from zero for at most max_steps steps (no local space)
        Opts o{1e-15, max_steps, RSR_INIT_ZERO, 0, 0, 0, 1 << 30, gamma, gamma};
        std::vector<SysHost *> one{&Y};
        solve_group(c, one, o, nullptr, s);
        int got = 0;
        if (n_kry > 0 && Y.lz_its > 0) {
            std::vector<double> co((size_t)3 * n_kry);
            read_back(c, {ReadBack{co.data(), c->d_lzc.p, sizeof(double) * co.size()}}, s);
            const double *rho = co.data() + 2 * n_kry;
            const int m = std::min(n_kry, Y.lz_its);
            std::vector<ComboJob> cj;
            std::vector<std::vector<double>> qs;
            for (int j = 0; j < m && rho[j] > 0.0; ++j, ++got) {
                cj.push_back(ComboJob{c->d_lz.as<double>() + (size_t)j * n, n, 1, nullptr, 1, V + (size_t)(1 + j) * ld, n,
                                      1, 0.0, nullptr, 0, n});
                qs.push_back(std::vector<double>{1.0 / std::sqrt(rho[j])});
            }
            combo(c, cj, qs, s);
        }
        sync(c, s);
        *n_out = 1 + got;
    });
}

}  // extern "C"

namespace {
// The solve of a shift set.  slot_off > 0 marks the adjoint solves: system i
// keeps its correction in slot slot[i] + slot_off, so the forward corrections
// in slot[i] survive, and its local space may take the forward correction of
// its shift as well.  Returns true when every system reached tol.
bool solve_set(rsr_ctx *c, const rsr_solve_desc *d, const double *b, double *X, rsr_shift_stats *stats,
               hipStream_t s, int slot_off)
{
    if (!d || !b || !X) fail(RSR_E_ARG, "null descriptor, b or X");
    if (c->inst.empty()) fail(RSR_E_STATE, "operators not set");
    const int m = d->n_sys;
    if (m <= 0 || !d->inst || !d->gammas) fail(RSR_E_ARG, "n_sys must be positive with inst and gammas");
    if (!(d->tol > 0.0)) fail(RSR_E_ARG, "tol must be positive");
    if (d->init < 0 || d->init > 4) fail(RSR_E_ARG, "unknown init");
    if (d->n_ritz < 0 || d->n_ritz > QMAX) fail(RSR_E_ARG, "n_ritz out of range");
    if (d->seed_lanczos < 0 || d->seed_p < 0 || d->seed_n_ritz < 0 || d->seed_n_ritz > QMAX)
        fail(RSR_E_ARG, "seed sizes out of range");
    if (d->seed_lanczos > 0 && d->mode != RSR_SEQUENTIAL) fail(RSR_E_ARG, "seeding needs sequential mode");
    if (d->seed_lanczos > 0 && c->wsa_base) fail(RSR_E_ARG, "seeding keeps library-owned memory: not with a caller workspace");
    if (d->mode != RSR_BATCHED && d->mode != RSR_SEQUENTIAL) fail(RSR_E_ARG, "unknown mode");
    std::vector<SysHost> sys(m);
    for (int i = 0; i < m; ++i) {
        Instance &I = get_inst(c, d->inst[i]);
        if (!std::isfinite(d->gammas[i])) fail(RSR_E_ARG, "gamma must be finite");
        if (m > 1 && d->ld_x < I.n) fail(RSR_E_ARG, "ld_x smaller than ny*nx");
        if (d->ld_b != 0 && d->ld_b < I.n) fail(RSR_E_ARG, "ld_b smaller than ny*nx");
        SysHost &Y = sys[i];
        Y.inst = d->inst[i];
        Y.shift = d->slot ? d->slot[i] : i;
        if (Y.shift < 0 || Y.shift >= (1 << 20)) fail(RSR_E_ARG, "slots must lie in [0, 2^20)");
        Y.slot = Y.shift + slot_off;
        Y.fwd_slot = slot_off > 0 ? Y.shift : -1;
        Y.gamma = d->gammas[i];
        Y.n = I.n;
        Y.b = b + (size_t)i * d->ld_b;
        Y.x = X + (size_t)i * d->ld_x;
    }
    set_device(c);
    alloc_ws(c, sys);
    c->bnorm_cache.clear();
    c->rhs_cache.clear();
    double *r0sq_dev = (double *)dscratch(c, c->d_r0sq, sizeof(double) * (size_t)m);
    HIPCHK(launch_fill(r0sq_dev, 0.0, m, s));
    for (int i = 0; i < m; ++i) sys[i].r0sq_dev = r0sq_dev + i;
    Opts o{d->tol, d->maxit, d->init, d->n_ritz, d->use_prev_k, d->use_prev_shift, d->split_I, d->gamma_JL,
           d->gamma_JR, d->solver};
    if (d->solver != RSR_SOLVER_CG && d->solver != RSR_SOLVER_MINRES) fail(RSR_E_ARG, "unknown solver");
    if (d->solver == RSR_SOLVER_MINRES && d->seed_lanczos > 0) fail(RSR_E_ARG, "seeding records CG-Lanczos data");
    if (c->ct && d->seed_lanczos > 0) fail(RSR_E_ARG, "seeding records CG-Lanczos data of the persistent kernel");
    c->last_cg_ms = 0.0;
    c->last_launches = 0;
    c->last_items = 0;
    long maxn = 0;
    for (auto &Y : sys) maxn = std::max(maxn, Y.n);
    if (o.maxit <= 0) o.maxit = (int)std::min<long>(10 * maxn, 1 << 30);
    if (d->mode == RSR_BATCHED) {
        for (int i0 = 0; i0 < m; i0 += MAXSYS) {
            std::vector<SysHost *> grp;
            for (int i = i0; i < std::min(m, i0 + MAXSYS); ++i) grp.push_back(&sys[i]);
            solve_group(c, grp, o, nullptr, s);
            StageTimer tsc(c, s, 7);
            store_corrections(c, grp, s);
        }
    } else {
        const double *gp = nullptr;
        // principal-space seeding from the CG-Lanczos data of the first system and,
        // when asked, of a second representative system solved right after it
        const bool seed = d->seed_lanczos > 0 && c->inst[sys[0].inst]->p == 0;
        const int second = (seed && d->seed_second > 0 && d->seed_second < m &&
                            sys[d->seed_second].inst == sys[0].inst) ? d->seed_second : -1;
        std::vector<int> order;
        order.push_back(0);
        if (second > 0) order.push_back(second);
        for (int i = 1; i < m; ++i)
            if (i != second) order.push_back(i);
        if (seed) {
            const long nlz = d->seed_lanczos;
            const int ncap = second > 0 ? 2 : 1;
            c->d_lz.ensure(sizeof(double) * (size_t)ncap * nlz * sys[0].n);
            c->d_lzc.ensure(sizeof(double) * (size_t)ncap * 3 * nlz);
            HIPCHK(launch_fill(c->d_lzc.as<double>(), 0.0, ncap * 3 * nlz, s));
            for (int t = 0; t < ncap; ++t) {
                SysHost &Y = sys[t == 0 ? 0 : second];
                Y.lz = c->d_lz.as<double>() + (size_t)t * nlz * Y.n;
                Y.lzc = c->d_lzc.as<double>() + (size_t)t * 3 * nlz;
                Y.nlz = nlz;
            }
        }
        std::vector<char> solved(m, 0);
        for (int oi = 0; oi < m; ++oi) {
            const int i = order[oi];
            std::vector<SysHost *> one{&sys[i]};
            // g^(k,l-1): the correction of the previous system in list order, read in
            // place from its slot (not written again, nor the slot pool moved, before
            // this solve ends)
            gp = (i > 0 && solved[i - 1] && sys[i - 1].inst == sys[i].inst) ? c->inst[sys[i].inst]->gslot(sys[i - 1].slot)
                                                                             : nullptr;
            solve_group(c, one, o, o.use_prev_shift ? gp : nullptr, s);
            solved[i] = 1;
            {
                StageTimer tsc(c, s, 7);
                store_corrections(c, one, s);
            }
            const int last_seed = second > 0 ? 1 : 0;
            if (seed && oi == last_seed) {
                std::vector<const SysHost *> ys{&sys[0]};
                if (second > 0) ys.push_back(&sys[second]);
                if (seed_from_lanczos(c, ys, d->seed_lanczos, d->seed_p, s) > 0) {
                    // the remaining systems start from the seeded principal space
                    o.init = RSR_INIT_MR;
                    o.n_ritz = std::min(d->seed_n_ritz, QMAX);
                }
            }
        }
        sync(c, s);

    }
    {
        std::vector<double> r0sq(m);
        read_back(c, {ReadBack{r0sq.data(), r0sq_dev, sizeof(double) * m}}, s);
        for (int i = 0; i < m; ++i)
            sys[i].relres_init = sys[i].bnorm > 0 ? std::sqrt(std::max(0.0, r0sq[i])) / sys[i].bnorm : 0.0;
    }
    bool all = true;
    for (int i = 0; i < m; ++i) {
        SysHost &Y = sys[i];
        const bool conv = Y.relres_true <= d->tol;
        all = all && conv;
        if (stats) {
            rsr_shift_stats &t = stats[i];
            t.iters = Y.iters;
            t.matvec_A = Y.mvA;
            t.matvec_E = Y.mvE;
            t.converged = conv ? 1 : 0;
            t.restarts = Y.restarts;
            t.local_dim = Y.q;
            t.relres_init = Y.relres_init;
            t.relres_true = Y.relres_true;
        }
    }
    sync(c, s);
    return all;
}
// Bytes of caller workspace a solve (or, with adjoint set, an adjoint) of the
// described shift set uses: the per-system vectors and initial residual norms
// for the whole call, plus the largest of the transient needs (one persistent-CG
// launch with its partials, barrier block and outputs; the grouped initial
// guesses; the largest product batch), with room for the staged descriptors and
// the 256-byte alignment of every piece.
size_t solve_ws_bytes(rsr_ctx *c, const rsr_solve_desc *d, bool adjoint)
{
    auto al = [](size_t b) { return (b + 511) & ~(size_t)255; };
    const int m = d->n_sys;
    size_t per_sys = 0, sum_n = 0, max_tiles = 0, max_n = 0;
    int max_p = 0;
    std::vector<long> tiles(m);
    for (int i = 0; i < m; ++i) {
        Instance &I = get_inst(c, d->inst[i]);
        const InstDev &D = c->h_inst[d->inst[i]];
        per_sys += al(sizeof(double) * ((size_t)I.n * (9 + 2 * QMAX) + 2 * QMAX + 64));
        sum_n += (size_t)I.n;
        max_n = std::max(max_n, (size_t)I.n);
        tiles[i] = (long)D.nty * D.ntx;
        max_p = std::max(max_p, I.p);
    }
    // the largest launch: up to MAXSYS systems in batched mode, one in sequential
    const int ml = d->mode == RSR_BATCHED ? std::min(m, MAXSYS) : 1;
    if (d->mode == RSR_BATCHED) {
        for (int i0 = 0; i0 < m; i0 += MAXSYS) {
            size_t t = 0;
            for (int i = i0; i < std::min(m, i0 + MAXSYS); ++i) t += (size_t)tiles[i];
            max_tiles = std::max(max_tiles, t);
        }
    } else {
        for (int i = 0; i < m; ++i) max_tiles = std::max(max_tiles, (size_t)tiles[i]);
    }
    const size_t launch = al(sizeof(SysDev) * ml) + 2 * al(sizeof(double) * max_tiles * NVP) + al(BAR_BYTES + FLAG_BYTES) +
                          al((sizeof(int) * 2 + 2 * sizeof(double)) * ml + 64) +
                          al((sizeof(ComboJob) + sizeof(double)) * ml + 16);
    const size_t guesses = al(sizeof(double) * 2 * (d->mode == RSR_BATCHED ? sum_n : max_n)) +
                           al((sizeof(ComboJob) + sizeof(double)) * (2 + 2 * (size_t)m) +
                              sizeof(double) * 3 * (size_t)max_p * m + 16);
    // products: W^T Z and W^T W of every system, [AU EU]^T b and norms
    std::vector<GramJob> gj;
    for (int i = 0; i < m; ++i) {
        const long n = c->inst[d->inst[i]]->n;
        gj.push_back(GramJob{nullptr, n, QMAX, nullptr, n, QMAX, n, nullptr, 0});
        gj.push_back(GramJob{nullptr, n, QMAX, nullptr, n, QMAX, n, nullptr, 0});
        gj.push_back(GramJob{nullptr, n, 2 * std::max(max_p, 1), nullptr, n, 1, n, nullptr, 0});
    }
    const size_t grams = al(sizeof(double) * gram_scratch_doubles(gj.data(), (int)gj.size())) +
                         al(sizeof(double) * (2 * QMAX * QMAX + 2 * (size_t)std::max(max_p, 1)) * m) +
                         al(sizeof(GramJob) * gj.size());
    size_t need = per_sys + al(sizeof(double) * m) + std::max({launch, guesses, grams}) + 65536 + 4096 * (size_t)m;
    if (c->ct) {   // sinograms of the K^T K applications: up to two per system at once
        size_t rays = 0;
        for (int i = 0; i < m; ++i) rays = std::max(rays, (size_t)c->inst[d->inst[i]]->na * c->inst[d->inst[i]]->nd);
        need += al(sizeof(double) * rays * 2 * (size_t)m) + al(sizeof(CtJob) * 2 * (size_t)m);
    }
    if (adjoint) need += al(sizeof(double) * (512 * (size_t)m + 2 * max_n));
    return need;
}

// Workspace layout of rsr_solve_shift_set_async (byte offsets); checks the
// descriptor against what the device-only path supports.
struct AsyncLayout {
    size_t vec, cbuf, sys, jobs, bn2, part, ctl, out, part_a, part_b, bytes;
    long vstride;
    int nb;
};
AsyncLayout async_layout(rsr_ctx *c, const rsr_solve_desc *d)
{
    const int m = d->n_sys;
    if (m <= 0 || m > ASYNC_MAXSYS || !d->inst || !d->gammas)
        fail(RSR_E_ARG, "the device-only solve takes 1.." + std::to_string(ASYNC_MAXSYS) + " systems");
    if (!(d->tol > 0.0)) fail(RSR_E_ARG, "tol must be positive");
    if ((d->init != RSR_INIT_ZERO && d->init != RSR_INIT_GIVEN) || d->n_ritz != 0 || d->use_prev_k ||
        d->use_prev_shift || d->seed_lanczos || d->solver != RSR_SOLVER_CG)
        fail(RSR_E_ARG, "the device-only solve is plain CG (init ZERO or GIVEN, no local spaces, no seeding)");
    const int ii = d->inst[0];
    Instance &I = get_inst(c, ii);
    if (I.ct) fail(RSR_E_ARG, "the device-only solve runs the persistent CG kernel (deblurring instances)");
    for (int i = 0; i < m; ++i) {
        if (d->inst[i] != ii) fail(RSR_E_ARG, "the device-only solve takes one instance");
        if (!std::isfinite(d->gammas[i])) fail(RSR_E_ARG, "gamma must be finite");
    }
    if (m > 1 && d->ld_x < I.n) fail(RSR_E_ARG, "ld_x smaller than ny*nx");
    if (d->ld_b != 0 && d->ld_b < I.n) fail(RSR_E_ARG, "ld_b smaller than ny*nx");
    const InstDev &D = c->h_inst[ii];
    const long tiles = (long)m * D.nty * D.ntx;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    AsyncLayout L;
    L.nb = (int)std::max<long>(1, std::min<long>(64, (I.n + 4 * NT - 1) / (4 * NT)));
    L.vstride = (long)(al(sizeof(double) * 9 * (size_t)I.n) / sizeof(double));
    size_t o = 0;
    L.vec = o; o += al(sizeof(double) * L.vstride * m);
    L.cbuf = o; o += al(sizeof(double) * 2 * QMAX * m);
    L.sys = o; o += al(sizeof(SysDev) * m);
    L.jobs = o; o += al(sizeof(ApplyJob) * 2 * m);
    L.bn2 = o; o += al(sizeof(double) * m);
    L.part = o; o += al(sizeof(double) * (size_t)m * L.nb);
    L.ctl = o; o += al(BAR_BYTES);
    L.out = o; o += al((sizeof(int) * 2 + 2 * sizeof(double)) * m + 64);
    L.part_a = o; o += al(sizeof(double) * tiles * NVP);
    L.part_b = o; o += al(sizeof(double) * tiles * NVP);
    L.bytes = o;
    return L;
}

// Persistent storage a workspace call may not allocate: a correction column for
// every slot of the descriptor (and the adjoint slots) and the Ritz blocks of its
// groups.
void reserve_persistent(rsr_ctx *c, const rsr_solve_desc *d, bool adjoint, hipStream_t s)
{
    std::map<int, std::set<int>> need;
    for (int i = 0; i < d->n_sys; ++i) {
        const int sl = d->slot ? d->slot[i] : i;
        if (sl < 0 || sl >= (1 << 20)) fail(RSR_E_ARG, "slots must lie in [0, 2^20)");
        need[d->inst[i]].insert(sl);
        if (adjoint) need[d->inst[i]].insert(sl + (1 << 20));
    }
    for (auto &kv : need) {
        Instance &I = get_inst(c, kv.first);
        int add = 0;
        for (int sl : kv.second) add += I.gcol.count(sl) ? 0 : 1;
        const int want = (int)I.gcol.size() + add;
        if (want > I.gpool_cols) {
            DBuf nb;
            nb.ensure(sizeof(double) * (size_t)want * I.n);
            if (I.gpool_cols > 0)
                HIPCHK(hipMemcpyAsync(nb.p, I.gpool.p, sizeof(double) * (size_t)I.gpool_cols * I.n,
                                      hipMemcpyDeviceToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            std::swap(nb.p, I.gpool.p);
            std::swap(nb.bytes, I.gpool.bytes);
            nb.release();
            I.gpool_cols = want;
        }
        if (d->n_ritz > 0)
            for (auto &rb : I.ritz) rb.buf.ensure(sizeof(double) * (size_t)3 * std::min(d->n_ritz, QMAX) * I.n);
    }
}

// The caller's workspace for the duration of one call.
struct WsScope {
    rsr_ctx *c;
    hipStream_t s;
    WsScope(rsr_ctx *c_, void *ws, size_t bytes, hipStream_t s_) : c(c_), s(s_)
    {
        c->wsa_base = (char *)ws;
        c->wsa_cap = ws ? bytes : 0;
        c->wsa_used = 0;
        c->wsa_peak = 0;
    }
    ~WsScope()
    {
        // an error may leave copies from held host data in flight
        if (!c->wsa_hold.empty()) (void)hipStreamSynchronize(s);
        c->wsa_hold.clear();
        c->wsa_base = nullptr;
        c->wsa_cap = 0;
        c->wsa_used = 0;
    }
};
}  // namespace

extern "C" {

rsr_status rsr_solve_shift_set(rsr_ctx *c, const rsr_solve_desc *d, const double *b, double *X, void *ws,
                               size_t ws_bytes, rsr_shift_stats *stats, void *stream)
{
    return guard(c, [&] {
        if (ws && ((uintptr_t)ws & 255)) fail(RSR_E_ARG, "workspace must be 256-byte aligned");
        WsScope scope(c, ws, ws_bytes, S(stream));
        if (!solve_set(c, d, b, X, stats, S(stream), 0))
            throw Err{RSR_NOT_CONVERGED, "some systems did not reach tol"};
    });
}

rsr_status rsr_solve_shift_set_noalloc(rsr_ctx *c, const rsr_solve_desc *d, const double *b, double *X,
                                       rsr_shift_stats *stats, void *stream)
{
    return guard(c, [&] {
        if (!d || !b || !X) fail(RSR_E_ARG, "null descriptor, b or X");
        if (c->inst.empty()) fail(RSR_E_STATE, "operators not set");
        if (d->n_sys <= 0 || !d->inst) fail(RSR_E_ARG, "n_sys must be positive with inst");
        set_device(c);
        if (!c->scratch_dev) fail(RSR_E_STATE, "static scratch not mapped on this device");
        const size_t need = solve_ws_bytes(c, d, false);
        if (need > NOALLOC_SCRATCH_BYTES)
            fail(RSR_E_ARG, "this shift set needs up to " + std::to_string(need) + " bytes of scratch; the static "
                            "scratch holds " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                            " (use rsr_solve_shift_set with a caller workspace)");
        WsScope scope(c, c->scratch_dev, NOALLOC_SCRATCH_BYTES, S(stream));
        if (!solve_set(c, d, b, X, stats, S(stream), 0))
            throw Err{RSR_NOT_CONVERGED, "some systems did not reach tol"};
    });
}

rsr_status rsr_solve_shift_set_async(rsr_ctx *c, const rsr_solve_desc *d, const double *b, double *X, void *ws,
                                     size_t ws_bytes, double *stats_dev, void *stream)
{
    return guard(c, [&] {
        if (!d || !b || !X || !ws || !stats_dev) fail(RSR_E_ARG, "null descriptor, b, X, workspace or stats");
        if ((uintptr_t)ws & 255) fail(RSR_E_ARG, "workspace must be 256-byte aligned");
        if (c->inst.empty()) fail(RSR_E_STATE, "operators not set");
        AsyncLayout Lo = async_layout(c, d);
        if (ws_bytes < Lo.bytes)
            fail(RSR_E_ARG, "workspace of " + std::to_string(ws_bytes) + " bytes is too small (needs " +
                                std::to_string(Lo.bytes) + ")");
        set_device(c);
        hipStream_t s = S(stream);
        const int m = d->n_sys;
        const int ii = d->inst[0];
        Instance &I = *c->inst[ii];
        const InstDev &D = c->h_inst[ii];
        char *w = (char *)ws;
        AsyncArgs a;
        memset(&a, 0, sizeof(a));
        a.m = m;
        a.init = d->init == RSR_INIT_GIVEN ? 1 : 0;
        a.n = I.n;
        a.inst = ii;
        a.ntiles = D.nty * D.ntx;
        a.nb = Lo.nb;
        a.tol = d->tol;
        a.b = b;
        a.ld_b = d->ld_b;
        a.X = X;
        a.ld_x = d->ld_x;
        a.vec = (double *)(w + Lo.vec);
        a.vstride = Lo.vstride;
        a.cbuf = (double *)(w + Lo.cbuf);
        a.sys = (SysDev *)(w + Lo.sys);
        a.jobs = (ApplyJob *)(w + Lo.jobs);
        a.bn2 = (double *)(w + Lo.bn2);
        a.part = (double *)(w + Lo.part);
        char *ctl = w + Lo.ctl;
        char *outb = w + Lo.out;
        a.clear = (double *)ctl;
        a.clear_n = (int)((Lo.part_a - Lo.ctl) / sizeof(double));   // barrier block and outputs (contiguous)
        int *out_iters = (int *)outb;
        int *out_status = out_iters + m;
        double *out_rho = (double *)(((uintptr_t)(out_status + m) + 15) & ~(uintptr_t)15);
        double *out_alpha = out_rho + m;
        a.out_iters = out_iters;
        a.out_status = out_status;
        a.out_alpha = out_alpha;
        for (int i = 0; i < m; ++i) a.gam[i] = d->gammas[i];
        // x0, r0 and ||b||; descriptors and cleared control blocks; r0 = b - B x0
        HIPCHK(launch_async_elem(a, 0, s));
        HIPCHK(launch_async_setup(a, s));
        const size_t alds = apply_lds_bytes(I);
        if (a.init == 1) {
            HIPCHK(launch_apply(c->d_inst.as<InstDev>(), D, a.jobs, nullptr, m, alds, s));
            HIPCHK(launch_async_elem(a, 1, s));
        }
        // the persistent CG launch
        const long tiles = (long)m * a.ntiles;
        const CgLaunch L = cg_config(c, m, 0, false, (long)m * I.n, tiles, I.form, 0, false);
        CGArgs g;
        memset(&g, 0, sizeof(g));
        g.nsys = m;
        g.sys = a.sys;
        g.inst = c->d_inst.as<InstDev>();
        g.part[0] = (double *)(w + Lo.part_a);
        g.part[1] = (double *)(w + Lo.part_b);
        g.pstride = (int)tiles;
        g.bar = (unsigned long long *)ctl;
        g.abort_flag = (int *)(ctl + 256);
        g.out_iters = out_iters;
        g.out_status = out_status;
        g.out_rho = out_rho;
        g.out_alpha = out_alpha;
        g.maxit = d->maxit > 0 ? d->maxit : (int)std::min<long>(10 * I.n, 1 << 30);
        g.form = L.form;
        g.G = L.G;
        g.timeout_ticks = (long long)(c->wall_khz * 1000.0 * c->bar_timeout_s);
        g.tile_lds = L.tl;
        g.taps_lds = L.taps;
        g.msys = L.msys;
        g.stamps = nullptr;
        {
            const hipError_t e = launch_cg(g, L.qt, false, L.G, L.lds, s);
            if (e != hipSuccess) fail(RSR_E_HIP, std::string("persistent CG launch: ") + hipGetErrorString(e));
        }
        // x += alpha p, rt = B x, ||b - rt||, statistics
        HIPCHK(launch_async_elem(a, 2, s));
        HIPCHK(launch_apply(c->d_inst.as<InstDev>(), D, a.jobs + m, nullptr, m, alds, s));
        HIPCHK(launch_async_elem(a, 3, s));
        HIPCHK(launch_async_stats(a, stats_dev, s));
    });
}

rsr_status rsr_workspace_size(rsr_ctx *c, const rsr_solve_desc *d, int kind, size_t *bytes, void *stream)
{
    return guard(c, [&] {
        if (!d || !bytes) fail(RSR_E_ARG, "null descriptor or output");
        if (c->inst.empty()) fail(RSR_E_STATE, "operators not set");
        if (d->n_sys <= 0 || !d->inst) fail(RSR_E_ARG, "n_sys must be positive with inst");
        if (d->n_ritz < 0 || d->n_ritz > QMAX) fail(RSR_E_ARG, "n_ritz out of range");
        set_device(c);
        if (kind < RSR_WS_SOLVE || kind > RSR_WS_DEVICE) fail(RSR_E_ARG, "unknown workspace kind");
        if (kind == RSR_WS_DEVICE) {   // the device-only solve keeps nothing between calls
            *bytes = async_layout(c, d).bytes;
            return;
        }
        *bytes = solve_ws_bytes(c, d, kind == RSR_WS_ADJOINT);
        reserve_persistent(c, d, kind == RSR_WS_ADJOINT, S(stream));
    });
}

rsr_status rsr_adjoint(rsr_ctx *c, const rsr_solve_desc *d, const double *X, const double *Gbar, double *Lambda,
                       double *dgamma_host, double *dw_h, double *dw_v, double *db, void *ws, size_t ws_bytes,
                       rsr_shift_stats *stats, void *stream)
{
    bool all = true;
    rsr_status st = guard(c, [&] {
        if (!d || !X || !Gbar || !Lambda) fail(RSR_E_ARG, "null argument");
        if (ws && ((uintptr_t)ws & 255)) fail(RSR_E_ARG, "workspace must be 256-byte aligned");
        WsScope scope(c, ws, ws_bytes, S(stream));
        if (d->n_sys <= 0 || !d->inst || !d->gammas) fail(RSR_E_ARG, "n_sys must be positive with inst and gammas");
        const int m = d->n_sys;
        const int ii = d->inst[0];
        for (int i = 1; i < m; ++i)
            if (d->inst[i] != ii) fail(RSR_E_ARG, "adjoint expects one instance");
        Instance &I = get_inst(c, ii);
        if (m > 1 && d->ld_x < I.n) fail(RSR_E_ARG, "ld_x smaller than ny*nx");
        // B_l lambda_l = Gbar_l with the same recycled solver (B_l symmetric); the
        // adjoint systems keep their corrections in slots of their own
        rsr_solve_desc ad = *d;
        ad.ld_b = d->ld_x;
        if (ad.init == RSR_INIT_GIVEN) ad.init = RSR_INIT_ZERO;
        ad.seed_lanczos = 0;
        hipStream_t s = S(stream);
        all = solve_set(c, &ad, Gbar, Lambda, stats, s, 1 << 20);
        // gradients: one pass over X and Lambda, partial sums of dL/dgamma per chunk
        const int nch = 512;
        const long n = I.n;
        double *dg = (double *)dscratch(c, c->d_grad, sizeof(double) * ((size_t)nch * m + ((dw_h && dw_v) ? 0 : 2 * (size_t)n)));
        double *wh = dw_h, *wv = dw_v;
        if (!wh || !wv) {
            wh = dg + (size_t)nch * m;
            wv = wh + n;
        }
        const double *gam = stage(c, std::vector<double>(d->gammas, d->gammas + m), s);
        HIPCHK(launch_grad(X, Lambda, d->ld_x, gam, m, I.d_wh.as<double>(), I.d_wv.as<double>(), I.ny, I.nx, wh, wv,
                           db, dg, nch, s));
        std::vector<double> h((size_t)nch * m);
        read_back(c, {ReadBack{h.data(), dg, sizeof(double) * h.size()}}, s);
        if (dgamma_host)
            for (int l = 0; l < m; ++l) {
                double sm = 0.0;
                for (int k = 0; k < nch; ++k) sm += h[(size_t)k * m + l];
                dgamma_host[l] = sm;
            }
    });
    if (st == RSR_OK && !all) {
        c->err = "some adjoint systems did not reach tol";
        return RSR_NOT_CONVERGED;
    }
    return st;
}

rsr_status rsr_get_tile(const rsr_ctx *c, int ii, int *ty, int *tx)
{
    if (!c || ii < 0 || ii >= (int)c->inst.size()) return RSR_E_ARG;
    if (ty) *ty = c->inst[ii]->ty;
    if (tx) *tx = c->inst[ii]->tx;
    return RSR_OK;
}

rsr_status rsr_set_tile(rsr_ctx *c, int ii, int ty, int tx)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (I.ct) fail(RSR_E_ARG, "tomography instances have no stencil tiles");
        if (ty < 4 || tx < 4 || ty > 64 || tx > 64 || (ty & (ty - 1)) || (tx & (tx - 1)))
            fail(RSR_E_ARG, "tile sides must be powers of two in [4, 64]");
        const int tl = tile_lds_doubles(ty, tx, eff_sy(I), eff_sx(I), I.sep);
        if (cg_lds_bytes(cg_tile_lds(tl, 8), taps_lds_doubles(eff_sy(I), I.sep), 8) > 160 * 1024)
            fail(RSR_E_ARG, "tile too large for LDS");
        set_device(c);
        I.ty = ty;
        I.tx = tx;
        upload_inst(c);
    });
}

rsr_status rsr_autotune(rsr_ctx *c, int ii, int n_vec, const char *cache_path)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (I.ct) fail(RSR_E_ARG, "nothing to tune on a tomography instance");
        if (n_vec <= 0) n_vec = 1;
        if (n_vec > MAXSYS) fail(RSR_E_ARG, "n_vec above the systems of one launch");
        set_device(c);
        std::ostringstream key;
        key << "gfx950 " << I.ny << " " << I.nx << " " << I.sy << " " << I.sx << " " << n_vec;
        auto apply_choice = [&](int ty, int tx, int gc, int form, int sep) {
            I.ty = ty;
            I.tx = tx;
            c->cg_gmax = gc;
            I.form = form;
            I.sep = (sep == 1 && I.sep_ok) ? 1 : (sep == 2 && I.rank) ? 2 : 0;
            upload_inst(c);
        };
        if (cache_path) {
            std::ifstream f(cache_path);
            std::string line;
            while (std::getline(f, line)) {
                if (line.rfind(key.str() + " ->", 0) == 0) {
                    int ty = 0, tx = 0, gc = 0, form = -1, sep = 1;
                    const int got = sscanf(line.c_str() + key.str().size() + 3, "%d %d %d %d %d", &ty, &tx, &gc, &form,
                                           &sep);
                    if (got >= 3) {
                        apply_choice(ty, tx, gc, got >= 4 ? form : -1, got >= 5 ? sep : 1);
                        return;
                    }
                }
            }
        }
        // Time the hot kernel itself: a bounded persistent-CG solve of n_vec systems
        // (shifts spread over 1e-3..1e-1) per candidate, keeping the fastest per
        // iteration, in stages: tile shape x workgroup cap (the single-system
        // kernel for one system, else the fused form); then the other iteration
        // forms (fused with coherent loads, fused with an agent acquire,
        // two-pass); then, for a rank-1 PSF of at most 9 x 9 taps, the direct 2-D
        // stencil against the banded separable one.
        const long n = I.n;
        DBuf bx;
        bx.ensure(sizeof(double) * n * 2 * n_vec);
        double *bvec = bx.as<double>(), *xvec = bvec + n * n_vec;
        hipStream_t s = nullptr;
        HIPCHK(launch_fill(bvec, 1.0, n * n_vec, s));
        std::vector<SysHost> sys(n_vec);
        for (int j = 0; j < n_vec; ++j) {
            SysHost &Y = sys[j];
            Y.inst = ii;
            Y.slot = j;
            Y.gamma = std::pow(10.0, -3.0 + 2.0 * j / std::max(1, n_vec - 1));
            Y.n = n;
            Y.b = bvec + (size_t)j * n;
            Y.x = xvec + (size_t)j * n;
            Y.bnorm = std::sqrt((double)n);
        }
        alloc_ws(c, sys);
        const long mvA = c->mv_A, mvE = c->mv_E;
        const int saved_mode = c->cg_mode;
        const int iters = 24;
        Opts o{0.0, iters, RSR_INIT_ZERO, 0, 0, 0, 0, 0.0, 0.0};
        auto time_it = [&]() {
            for (auto &Y : sys) {
                HIPCHK(launch_fill(Y.x, 0.0, n, s));
                HIPCHK(hipMemcpyAsync(Y.r, Y.b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
                Y.q = 0;
                Y.iters = 0;
            }
            std::vector<SysHost *> ptrs;
            for (auto &Y : sys) ptrs.push_back(&Y);
            c->last_cg_ms = 0.0;
            run_cg(c, ptrs, o, s);
            int its = 0;
            for (auto &Y : sys) its = std::max(its, Y.iters);
            return c->last_cg_ms / std::max(1, its);
        };
        const int cand[][2] = {{16, 16}, {16, 32}, {32, 16}, {32, 32}, {8, 64}, {16, 64}};
        const int gcaps[] = {128, 256, 512, 1024};
        double best = 1e30;
        // stage 1 in the single-system kernel for one system (where a launch
        // does not fit it, the launch falls back by size), else the fused form
        // with coherent loads
        const int form1 = n_vec == 1 ? 3 : 0;
        int bty = I.ty, btx = I.tx, bg = c->cg_gmax, bform = form1, bsep = I.sep;
        c->cg_mode = form1 + 1;
        for (auto &cd : cand) {
            const int tl = tile_lds_doubles(cd[0], cd[1], eff_sy(I), eff_sx(I), I.sep);
            const int ms8 = (n_vec + 7) & ~7;
            if (cg_lds_bytes(cg_tile_lds(tl, ms8), taps_lds_doubles(eff_sy(I), I.sep), ms8) > 160 * 1024) continue;
            I.ty = cd[0];
            I.tx = cd[1];
            upload_inst(c);
            for (int gc : gcaps) {
                c->cg_gmax = gc;
                const double per = time_it();
                if (per < best) {
                    best = per;
                    bty = cd[0];
                    btx = cd[1];
                    bg = gc;
                }
            }
        }
        I.ty = bty;
        I.tx = btx;
        c->cg_gmax = bg;
        upload_inst(c);
        for (int form = 0; form <= 2; ++form) {
            if (form == form1) continue;
            c->cg_mode = form + 1;
            const double per = time_it();
            if (per < best) {
                best = per;
                bform = form;
            }
        }
        c->cg_mode = bform + 1;
        if ((I.sep_ok && I.ssq <= 9) || I.rank) {
            const int keep = I.sep;
            I.sep = 0;
            upload_inst(c);
            const int tl = tile_lds_doubles(bty, btx, eff_sy(I), eff_sx(I), 0);
            const int ms8 = (n_vec + 7) & ~7;
            if (cg_lds_bytes(cg_tile_lds(tl, ms8), taps_lds_doubles(eff_sy(I), 0), ms8) <= 160 * 1024) {
                const double per = time_it();
                if (per < best) {
                    best = per;
                    bsep = 0;
                }
            }
            I.sep = keep;
        }
        c->mv_A = mvA;
        c->mv_E = mvE;
        c->cg_mode = saved_mode;
        apply_choice(bty, btx, bg, bform, bsep);
        bx.release();
        if (cache_path) {
            std::ofstream f(cache_path, std::ios::app);
            f << key.str() << " -> " << bty << " " << btx << " " << bg << " " << bform << " " << bsep << "\n";
        }
    });
}

rsr_status rsr_get_recycle_info(const rsr_ctx *c, int ii, int *p, double *Ahat, double *Ehat)
{
    if (!c || ii < 0 || ii >= (int)c->inst.size()) return RSR_E_ARG;
    const Instance &I = *c->inst[ii];
    if (p) *p = I.p;
    if (Ahat && !I.Ahat.empty()) memcpy(Ahat, I.Ahat.data(), sizeof(double) * I.p * I.p);
    if (Ehat && !I.Ehat.empty()) memcpy(Ehat, I.Ehat.data(), sizeof(double) * I.p * I.p);
    return RSR_OK;
}

rsr_status rsr_get_recycle_basis(rsr_ctx *c, int ii, double *U_out, long ld, void *stream)
{
    return guard(c, [&] {
        Instance &I = get_inst(c, ii);
        if (I.p > 0 && (!U_out || ld < I.n)) fail(RSR_E_ARG, "null output or ld < ny*nx");
        set_device(c);
        for (int j = 0; j < I.p; ++j)
            HIPCHK(hipMemcpyAsync(U_out + (size_t)j * ld, I.d_U.as<double>() + (size_t)j * I.n, sizeof(double) * I.n,
                                  hipMemcpyDeviceToDevice, S(stream)));
        HIPCHK(hipStreamSynchronize(S(stream)));
    });
}

rsr_status rsr_last_solve_timing(const rsr_ctx *c, double *ms, int *launches, long *items)
{
    if (!c) return RSR_E_ARG;
    if (ms) *ms = c->last_cg_ms;
    if (launches) *launches = c->last_launches;
    if (items) *items = c->last_items;
    return RSR_OK;
}

long long rsr_allocation_count(void) { return g_alloc_calls.load(); }

rsr_status rsr_get_counters(const rsr_ctx *c, long *matvec_A, long *matvec_E)
{
    if (!c) return RSR_E_ARG;
    if (matvec_A) *matvec_A = c->mv_A;
    if (matvec_E) *matvec_E = c->mv_E;
    return RSR_OK;
}

}  // extern "C"
