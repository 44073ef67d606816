// Internal declarations shared by the device kernels and the host engine.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rsr {

// Global-memory views.  Pointers read out of descriptors are generic to the
// compiler, which then emits flat instructions; a flat load counts against
// both the vector-memory and the LDS wait counters, so every LDS wait would
// also wait for the global loads in flight.  Kernels read and write global
// data through these address-space-1 views instead.
typedef __attribute__((address_space(1))) double gdbl;
__device__ __forceinline__ gdbl *gp(double *p) { return (gdbl *)p; }
__device__ __forceinline__ const gdbl *gp(const double *p) { return (const gdbl *)p; }

constexpr int NT = 256;        // threads per workgroup (4 wave64)
constexpr int QMAX = 8;        // widest local (deflation) space per system
constexpr int NVP = 4 + 2 * QMAX;   // values per chunk partial: p.w, r.r, r.w, w.w, Z^T r[QMAX], Z^T w[QMAX]
constexpr int MAXSYS = 512;    // systems per persistent launch
constexpr int RB = 8;          // register-blocked outputs per thread in the stencil passes
constexpr int MAXS = 31;       // largest separable PSF extent with a compiled path
constexpr int RMAX = 4;        // largest PSF rank with the rank-R path (terms of the separable sum)
constexpr int TAPS = 64;       // LDS slots per staged band (4r + 1 <= 61 taps)

// Device view of one instance (image geometry, PSF, weights, tiling).
struct InstDev {
    int ny, nx;
    int ty, tx;        // tile (outputs per workgroup item), powers of two
    int lty, ltx;      // log2 of ty, tx
    int nty, ntx;      // tiles per dimension
    int sep;           // 1: rank-1 separable PSF (banded K^T K), 2: rank-R sum of separable terms,
                       // 0: direct 2-D stencil
    int rank;          // terms of the rank-R path (sep 2)
    int rsv;
    int sy, sx;        // PSF extent (odd); for sep 1 both equal the zero-padded square size
    const double *fy;  // [sy] column factor (sep)
    const double *fx;  // [sx] row factor (sep)
    const double *band; // sep 1: banded factors of K^T K and their end corrections (layout in band_tables);
                        // sep 2: per term [fy reversed][fx reversed][fy][fx]
    const double *psf; // [sy*sx] (direct)
    const double *wh;  // [ny*nx] weights of x[i,j+1]-x[i,j]; 0 in the last column
    const double *wv;  // [ny*nx] weights of x[i+1,j]-x[i,j]; 0 in the last row
};

// Device view of one shifted system inside a persistent CG launch.
struct SysDev {
    int inst;
    int q;             // local space width (0..QMAX)
    int ntiles;
    int tile_base;     // offset of this system's partial slots
    double gamma;
    double tolabs;     // tol * ||b||
    double *x;
    double *rb[2];     // residual r_j in rb[j & 1] (rb[0] holds the starting residual)
    double *wb[2];     // w_j = B p_j in wb[j & 1]
    double *pb[2];     // undeflated direction ph_j in pb[j & 1]
    double *pa;        // search direction p_j = ph_j - W c_j
    double *cbuf;      // [2][QMAX] deflation coefficients c_j, double-buffered by iteration parity
    const double *W;   // [q][ldw] local basis (deflation), column-major
    const double *Z;   // [q][ldw] B W
    long ldw;
    double Ginv[QMAX * QMAX];   // pseudo-inverse of W^T Z (row-major q x q)
    // optional Lanczos capture (nlz > 0): residuals r_j, j < nlz, into lz[j * ldw + i]
    // and the coefficients alpha_j, beta_j, rho_j into lzc[0..nlz), [nlz..2 nlz), [2 nlz..3 nlz)
    double *lz;
    double *lzc;
    long nlz;
};

struct CGArgs {
    int nsys;
    const SysDev *sys;
    const InstDev *inst;
    double *part[2];               // [NVP][pstride] chunk partials (value-major), double-buffered by iteration parity
    int pstride;                   // slots per value plane (>= total tiles of the launch)
    unsigned long long *bar;       // barrier control block (BAR_BYTES, zero at launch): global counter,
                                   // per-group arrival counters and release epochs, 256-byte lines
    int *abort_flag;               // set on barrier timeout
    int *out_iters;                // [nsys]
    int *out_status;               // [nsys] 1 converged, 2 maxit, -3 nonfinite, -4 not SPD
    double *out_rho;               // [nsys] final recursive r.r
    double *out_alpha;             // [nsys] step still to apply after the launch: x += alpha p (p in pa)
    int maxit;
    int form;                      // iteration form: 0 fused (one phase per iteration that recomputes r,
                                   // ph on the halo from r, w, ph of step j-1; other workgroups' cells
                                   // read with coherent loads), 1 fused with an agent-scope acquire per
                                   // barrier and plain loads, 2 two-pass (r, ph updated elementwise, a
                                   // barrier, then the stencil pass reads ph alone) with that acquire
    int G;                         // workgroups in the grid
    long long timeout_ticks;       // barrier wait limit in s_memrealtime ticks (100 MHz)
    int tile_lds;                  // doubles of dynamic LDS used by the stencil buffers
    int taps_lds;                  // doubles of dynamic LDS for an instance's bands and end corrections
    int msys;                      // capacity of the per-system LDS arrays (>= nsys)
    unsigned long long *stamps;    // optional [DBG_ITERS][8] phase timestamps of workgroup 0 (or null)
};
constexpr int DBG_ITERS = 1024, DBG_SLOTS = 16;   // workgroup 0's stamps: [DBG_ITERS][DBG_SLOTS]
constexpr int DBG_WG_IT0 = 100, DBG_WG_NIT = 8, DBG_WG_MAX = 1024;   // per-workgroup stamps: [DBG_WG_NIT][DBG_WG_MAX][8]
constexpr size_t DBG_WORDS = (size_t)DBG_ITERS * DBG_SLOTS + (size_t)DBG_WG_NIT * DBG_WG_MAX * 8;

// Launch plumbing implemented in kernels.hip.
int tile_lds_doubles(int ty, int tx, int sy, int sx, int sep);
int taps_lds_doubles(int s, int sep);         // an instance's bands and end corrections (PSF extent s)
int cg_tile_lds(int tile_lds, int msys);      // tile LDS rounded up to the reduction scratch
size_t cg_lds_bytes(int tile_lds, int taps_lds, int msys);
constexpr int BAR_GROUPS = 8;                          // barrier groups (one per XCD when G % 8 == 0)
constexpr size_t BAR_BYTES = 256 * (2 + 2 * BAR_GROUPS);
constexpr size_t FLAG_BYTES = 8 * NT;                  // step flags of the single-system kernel, after the
                                                       // barrier block (one per tile, at most NT tiles)
int cg_width(int qmax);                           // compiled local-space width for a widest q
// Form 3 takes its one system's descriptor as a second kernel argument (sys1,
// with a.sys null): no upload before the launch.  It is not a field of CGArgs,
// whose copies the general kernel keeps in scratch.
hipError_t launch_cg(const CGArgs &a, int qt, bool lz, int G, size_t lds, hipStream_t s,
                     const SysDev *sys1 = nullptr);
int cg_max_blocks_per_cu(size_t lds, int qt, bool lz, int form);
// Form 3: the single-system kernel k_cg1 (cg1.hip), for one system whose tiles
// (at most NT, of at most 4 NT pixels each) each get a workgroup of their own.
const void *cg1_kernel(int qt, bool lz);   // lz: the variant that records CG-Lanczos data (qt 0 or QMAX)

// The job descriptors of a launch: carried in the kernel arguments when there
// are at most KJ of them, so the launch needs no upload of its own, else read
// from a device array.
constexpr int KJ = 8;
template <class J>
struct Jobs {
    const J *dev;              // device array (used when n == 0)
    int n;                     // jobs held in inl
    J inl[KJ];
    // the descriptor of job i, the same in every lane: read through a
    // uniform branch and kept in scalar registers
    __device__ J operator[](int i) const
    {
        static_assert(sizeof(J) % 4 == 0, "descriptor size");
        J v;
        if (n) v = inl[i];
        else v = dev[i];
        unsigned w[sizeof(J) / 4];
        __builtin_memcpy(w, &v, sizeof(J));
#pragma unroll
        for (int k = 0; k < (int)(sizeof(J) / 4); ++k) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
        __builtin_memcpy(&v, w, sizeof(J));
        return v;
    }
};
template <class J>
Jobs<J> make_jobs(const J *dev, const J *host, int njobs)
{
    Jobs<J> a;
    a.dev = dev;
    a.n = 0;
    if (!dev)
        for (int i = 0; i < njobs; ++i) a.inl[a.n++] = host[i];
    return a;
}

struct ApplyJob {              // y = cA K^T K v + cE E v   (or K / K^T alone)
    int inst;
    int op;                    // 0: cA*A + cE*E ; 3: K ; 4: K^T
    double cA, cE;
    const double *v;
    double *y;
};
// jobs_dev == nullptr: the njobs (at most KJ) jobs of jobs_host go in the
// kernel arguments.
hipError_t launch_apply(const InstDev *inst_dev, const InstDev &inst_host, const ApplyJob *jobs_dev,
                        const ApplyJob *jobs_host, int njobs, size_t lds, hipStream_t s);

hipError_t launch_blur(const InstDev *inst_dev, const InstDev &inst_host, const ApplyJob *jobs_dev,
                       int njobs, hipStream_t s);

hipError_t launch_weights(const double *x, double beta, double *wh, double *wv, int ny, int nx,
                          hipStream_t s);
hipError_t launch_copy_weights(const double *wh_in, const double *wv_in, double *wh, double *wv,
                               int ny, int nx, hipStream_t s);
hipError_t launch_fill(double *p, double v, long n, hipStream_t s);

// Tall-skinny products over n rows:
//   C[i][j] = sum_r X[r + i*ldx] * Y[r + j*ldy],  i < a, j < c      (gram)
//   Y[r + j*ldy] = beta*Y + sum_k X[r + k*ldx] * Q[k + j*ldq]       (combo)
struct GramJob {
    const double *X; long ldx; int a;
    const double *Y; long ldy; int c;
    long n;
    double *C;                 // device [a][c] row-major (result)
    long sc_off;               // offset of this job's chunk partials in the scratch buffer
};
hipError_t launch_gram(const GramJob *jobs_dev, const GramJob *jobs_host, int njobs, double *scratch,
                       size_t scratch_doubles, hipStream_t s);
size_t gram_scratch_doubles(const GramJob *jobs_host, int njobs);

struct ComboJob {
    const double *X; long ldx; int a;
    const double *Q; int ldq;  // device [c][ldq] column-major coefficients (k fast)
    double *Y; long ldy; int c;
    double beta;               // Y = beta*Y + X Q   (beta = 0: Y is not read)
    const double *Y0;          // optional: Y = Y0 + X Q when non-null (beta ignored)
    long ldy0;
    long n;
    int qoff = -1;             // >= 0: Q is at this offset of the launch's inline coefficients
};
// The coefficients of a combination launch whose jobs are inline, when they
// fit: a launch without any upload.
constexpr int KQ = 256;
struct ComboArgs {
    Jobs<ComboJob> jobs;
    double q[KQ];
};
// jobs_dev == nullptr: the jobs (at most KJ) go in the kernel arguments, and so
// do Qs (column-major a x c each, at most KQ doubles in all) when qs is given;
// otherwise each job's Q points to device memory.
hipError_t launch_combo(const ComboJob *jobs_dev, const ComboJob *jobs_host, int njobs, hipStream_t s,
                        const double *const *qs = nullptr);

// Graph-capturable plain CG of a shift set on one instance (see kernels.hip).
constexpr int ASYNC_MAXSYS = 128;
struct AsyncArgs {
    int m;                     // systems (<= ASYNC_MAXSYS)
    int init;                  // 0: x0 = 0, 1: x0 given in X
    long n;                    // pixels per system
    int inst;                  // instance
    int ntiles;                // tiles per system
    int nb;                    // workgroups per system of the elementwise kernels
    double tol;
    const double *b;
    long ld_b;
    double *X;
    long ld_x;
    double *vec;               // per system: r, r1, w, w1, p0, p1, (unused), rt, pa (n each) at vec + i * vstride
    long vstride;
    double *cbuf;              // [m][2 QMAX]
    SysDev *sys;               // [m]
    ApplyJob *jobs;            // [2 m]: B x -> r (GIVEN start), B x -> rt (true residual)
    double *bn2;               // [m]
    double *part;              // [m][nb]
    double *clear;             // barrier block and outputs, zeroed by the setup kernel
    int clear_n;
    const int *out_iters, *out_status;
    const double *out_alpha;
    double gam[ASYNC_MAXSYS];
};
hipError_t launch_async_elem(const AsyncArgs &a, int stage, hipStream_t s);
hipError_t launch_async_setup(const AsyncArgs &a, hipStream_t s);
hipError_t launch_async_stats(const AsyncArgs &a, double *stats, hipStream_t s);

hipError_t launch_grad(const double *X, const double *Lam, long ld, const double *gammas_dev, int m,
                       const double *wh, const double *wv, int ny, int nx, double *dw_h, double *dw_v,
                       double *db, double *dg_partial, int nchunks, hipStream_t s);

// Parallel-beam tomography instances (ct.hip).  Pixel (i, j) is the unit square
// centred at x = j - (nx - 1) / 2, y = (ny - 1) / 2 - i; ray (a, k) is the line
// x cos(theta_a) + y sin(theta_a) = (k - (nd - 1) / 2) * spacing; K = scale * C
// with C the ray-pixel intersection lengths and scale = 1 / ||C||_F.
struct CtDev {
    int ny, nx;
    int na, nd;        // angles, detector bins (sinogram [na][nd], angle-major)
    double spacing;
    double scale;
    const double *cs;  // [na][4] cos, sin of the angles and the reciprocals 1/(-sin), 1/cos (0 for a 0)
    const double *wh;  // weight planes of E (layout of InstDev)
    const double *wv;
};
struct CtJob {         // op 0: y = cA K^T K v + cE E v; op 3: y = K v (sinogram); op 4: y = K^T v (v a sinogram)
    int inst;
    int op;
    double cA, cE;
    const double *v;
    double *y;
    double *sino;      // op 0 with cA != 0: [na*nd] scratch for K v; op 5: per-ray sums of squared lengths
};
hipError_t launch_ct_fwd(const CtDev *inst_dev, const CtJob *jobs_dev, int njobs, int max_rays, hipStream_t s);
hipError_t launch_ct_back(const CtDev *inst_dev, const CtJob *jobs_dev, int njobs, long max_px, hipStream_t s);

}  // namespace rsr
