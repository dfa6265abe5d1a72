// Implicit diffusion (Sec. II.B.3b, Scheme 2): per diffusing pool, solve
// (I + a L_w) y = x with the conjugate gradient method preconditioned by the
// inverse diagonal of the system matrix (Sec. III).  Matrix-free: the
// Laplacian is applied as a gather over the neighbours (the explicit step's
// neighbour source: table or packed).  Vectors,
// dot products and scalars are FP64 whatever the field type.
//
// Per iteration two streaming kernels, each followed by a one-block kernel
// that reduces the per-block partials in a fixed order and updates the
// scalars on the device:
//  - SpMV: the new direction p = z + beta p_old, q = B p and p.q partials;
//    also x += alpha p_old, the previous iteration's x update, done here
//    where p_old is read anyway (the last one is added on write-back);
//  - update: r -= alpha q, z = M^-1 r, r.z and r.r partials (without region
//    weights M^-1 comes from a table indexed by the voxel's neighbour count,
//    1 byte per voxel instead of an FP64 vector).
// q = B p is formed as B z + beta q_old (linearity), so the SpMV gathers one
// vector instead of two; this adds rounding to the gap between the recursive
// and the true residual, orders of magnitude below the tolerances in use.
// The host reads the scalars only every few iterations; kernels launched
// after convergence return at once.
//
// Multigrid option (not in the paper, whose preconditioner is the diagonal):
// M^-1 is one V-cycle over a hierarchy of aggregates.  Level l+1 has one cell
// per occupied 2x2x2 block of level l's grid and the piecewise-constant
// prolongation P; its operator P^T B_l P keeps the form mass + a L_w (the
// mass of a cell is its number of voxels, the weight between two cells the
// sum of the weights of the level-l edges between them), so every level
// runs the same kind of kernel.  Pre-smoothing is one damped Jacobi sweep
// from zero, x = w D^-1 r, post-smoothing the same sweep after the coarse
// correction, and the coarsest level gets kMgSweeps damped Jacobi sweeps:
// a fixed linear map, symmetric (the post-smoother is the transpose of the
// pre-smoother; k Jacobi sweeps from zero are D^-1/2 p(D^-1/2 B D^-1/2)
// D^-1/2 for a polynomial p) and positive definite (w times the largest
// eigenvalue of D^-1 B stays below 2 because every row's weights sum to less
// than its diagonal).  The restriction is computed per coarse cell from its
// children (found with the level's rank index in a fixed order) and the
// prolongation per fine cell from its parent, so no sum depends on
// scheduling.  Every level's kernels are one thread per cell: residual,
// restriction (sum over the children), prolongation (add the parent's
// value), post-smoothing.  In MG mode the update kernel also forms the
// pre-smoothed iterate w D^-1 r (in z); the V-cycle's last kernel writes z
// and the r.z partials.
#include "vg_internal.h"

namespace vg {
namespace {

enum { S_RZ = 0, S_RR, S_BB, S_ALPHA, S_BETA, S_DONE, S_ITER, S_RTOL2, S_NSCAL = 8 };

// multigrid V-cycle
constexpr double kMgOmega = 0.8;        // damping of the Jacobi smoother
constexpr int64_t kMgCoarsest = 1024;   // a level this small is solved by sweeps alone
constexpr int kMgSweeps = 8;            // damped Jacobi sweeps on the coarsest level
constexpr int kMgCoarseThreads = 1024;  // the coarsest level's single block
constexpr int kMgCoarseMax = 4096;      // cells the coarsest kernel holds in LDS

__device__ __forceinline__ double weight(const uint16_t *rcode, const double *cl, int64_t i, int k,
                                         bool reg) {
    if (!reg) return 1.0;
    const uint32_t code = rcode[i];
    const uint32_t own = code & 7u;
    const uint32_t other = own ^ (((code >> (3 + k)) & 1u) << (k >> 1));
    return 0.5 * (cl[own] + cl[other]);
}

struct CgArgs {
    const int32_t *nbr = nullptr;
    const uint16_t *rcode = nullptr;
    PackedNbr pk;                // packed neighbour sources (when built)
    int64_t n = 0;
    int64_t ntiles = 0;
    double a = 0;
    double c[VG_NREG] = {};
};

// Neighbour sources of the CG kernels (the explicit step's): the table, or
// a packed source; an absent neighbour comes back as the voxel itself.
enum { NS_TABLE = 0, NS_REL = 1, NS_OFF = 2 };

template <int NS>
__device__ __forceinline__ void cg_neighbours(const CgArgs &A, int64_t i, int64_t (&j)[6], bool (&pres)[6]) {
    if constexpr (NS == NS_TABLE) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const int32_t jk = A.nbr[(int64_t)k * A.n + i];
            pres[k] = jk >= 0;
            j[k] = pres[k] ? (int64_t)jk : i;
        }
    } else {
        uint32_t jp[6];
        const PackedWords W = packed_words<NS == NS_REL>(A.pk, (uint32_t)i);
        packed_decode<NS == NS_REL>(A.pk, (uint32_t)i, W, jp);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            j[k] = (int64_t)jp[k];
            pres[k] = j[k] != i;      // no periodic wrap: a neighbour is never the voxel itself
        }
    }
}

template <typename F, bool REG, int NS, bool MG>
__global__ __launch_bounds__(kBlock) void k_cg_init(CgArgs A, F field,
                                                    double *__restrict__ y, double *__restrict__ r,
                                                    double *__restrict__ z, double *__restrict__ p,
                                                    double *__restrict__ m, double *__restrict__ part,
                                                    double *__restrict__ q) {
    __shared__ double lds[kWaves * 3];
    __shared__ double cl[VG_NREG];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = A.c[threadIdx.x];
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};   // r.z, r.r, b.b
    for (int64_t it = 0;; it++) {
    const int64_t t = xcd_stride_tile(blockIdx.x, gridDim.x, it, A.ntiles);
    if (t >= A.ntiles) break;
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = t * kTile + v * kBlock + threadIdx.x;
        if (i >= A.n) continue;
        const double b = field.get(i);
        int64_t j[6];
        bool pres[6];
        cg_neighbours<NS>(A, i, j, pres);
        double fj[6];
#pragma unroll
        for (int k = 0; k < 6; k++) fj[k] = field.get(j[k]);
        double s = 0.0, deg = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            if (!pres[k]) continue;
            const double w = weight(A.rcode, cl, i, k, REG);
            deg += w;
            s += w * (b - fj[k]);
        }
        const double mi = 1.0 / (1.0 + A.a * deg);
        const double ri = b - (b + A.a * s);
        const double zi = mi * ri;
        y[i] = b;
        r[i] = ri;
        // MG: z holds the V-cycle's pre-smoothed iterate w D^-1 r until the
        // cycle overwrites it; the first direction is then z + 0 * p
        z[i] = MG ? kMgOmega * ri * mi : zi;
        p[i] = MG ? 0.0 : zi;
        if (REG) m[i] = mi;
        else ((uint8_t *)m)[i] = (uint8_t)deg;   // 1/diag is then one of 7 values
        q[i] = 0.0;    // B p of no direction: the first q is B z alone (beta = 0)
        acc[0] += ri * zi;
        acc[1] += ri * ri;
        acc[2] += b * b;
    }
    }
    block_sum<3>(acc, lds);
    if (threadIdx.x == 0) {
        for (int u = MG ? 1 : 0; u < 3; u++) part[(int64_t)blockIdx.x * 4 + u] = acc[u];
    }
}

// p' = z + beta p (the new search direction, written out) and q' = B p',
// formed as B z + beta q by linearity so that only z is gathered (q holds
// B p from the previous iteration and 0 before the first, where beta = 0)
template <bool REG, int NS>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(CgArgs A, const double *__restrict__ z,
                                                    const double *__restrict__ pold, double *__restrict__ pnew,
                                                    double *__restrict__ y,
                                                    double *__restrict__ q, const double *__restrict__ scal,
                                                    double *__restrict__ part) {
    if (scal[S_DONE] != 0.0) return;
    __shared__ double lds[kWaves];
    __shared__ double cl[VG_NREG];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = A.c[threadIdx.x];
    __syncthreads();
    const double beta = scal[S_BETA], alpha = scal[S_ALPHA];
    double acc[1] = {0.0};
    for (int64_t it = 0;; it++) {
    const int64_t t = xcd_stride_tile(blockIdx.x, gridDim.x, it, A.ntiles);
    if (t >= A.ntiles) break;
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = t * kTile + v * kBlock + threadIdx.x;
        if (i >= A.n) continue;
        const double zi = z[i], po = pold[i];
        y[i] += alpha * po;   // the previous iteration's x update (alpha = 0 before the first)
        const double pi = zi + beta * po;
        int64_t j[6];
        bool pres[6];
        cg_neighbours<NS>(A, i, j, pres);
        double zj[6];
#pragma unroll
        for (int k = 0; k < 6; k++) zj[k] = z[j[k]];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            if (!pres[k]) continue;
            s += weight(A.rcode, cl, i, k, REG) * (zi - zj[k]);
        }
        const double qi = (zi + A.a * s) + beta * q[i];
        pnew[i] = pi;
        q[i] = qi;
        acc[0] += pi * qi;
    }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 4] = acc[0];
}

// m: 1/diag per voxel with region weights; without them the number of
// neighbours per voxel (uint8), and 1/diag = 1 / (1 + a deg) from a table
// (the same division as in the init kernel, so the same values)
template <bool REG, bool MG>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, int64_t ntiles, double a,
                                                      const double *__restrict__ q, const double *__restrict__ m,
                                                      double *__restrict__ r,
                                                      double *__restrict__ z, const double *__restrict__ scal,
                                                      double *__restrict__ part) {
    if (scal[S_DONE] != 0.0) return;
    __shared__ double lds[kWaves * 2];
    __shared__ double mtab[8];
    if (!REG) {
        if (threadIdx.x < 7) mtab[threadIdx.x] = 1.0 / (1.0 + a * (double)threadIdx.x);
        __syncthreads();
    }
    const double alpha = scal[S_ALPHA];
    double acc[2] = {0.0, 0.0};
    for (int64_t it = 0;; it++) {
    const int64_t t = xcd_stride_tile(blockIdx.x, gridDim.x, it, ntiles);
    if (t >= ntiles) break;
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = t * kTile + v * kBlock + threadIdx.x;
        if (i >= n) continue;
        const double ri = r[i] - alpha * q[i];
        const double mi = REG ? m[i] : mtab[((const uint8_t *)m)[i]];
        r[i] = ri;
        if (MG) {
            z[i] = kMgOmega * ri * mi;   // the V-cycle's pre-smoothed iterate
        } else {
            const double zi = mi * ri;
            z[i] = zi;
            acc[0] += ri * zi;
        }
        acc[1] += ri * ri;
    }
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        if (!MG) part[(int64_t)blockIdx.x * 4] = acc[0];   // MG: the V-cycle writes r.z
        part[(int64_t)blockIdx.x * 4 + 1] = acc[1];
    }
}

// stage 0: after init; 1: alpha after spmv; 2: beta/convergence after update
__global__ __launch_bounds__(kBlock) void k_cg_scalars(const double *__restrict__ part, int nblocks, int stage,
                                                       double *__restrict__ scal) {
    if (stage != 0 && scal[S_DONE] != 0.0) return;
    __shared__ double lds[kWaves * 3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
        v[0] += part[(int64_t)b * 4];
        v[1] += part[(int64_t)b * 4 + 1];
        v[2] += part[(int64_t)b * 4 + 2];
    }
    block_sum<3>(v, lds);
    if (threadIdx.x != 0) return;
    if (stage == 0) {
        scal[S_RZ] = v[0];
        scal[S_RR] = v[1];
        scal[S_BB] = v[2];
        scal[S_BETA] = 0.0;
        scal[S_ITER] = 0.0;
        scal[S_DONE] = (v[1] <= scal[S_RTOL2] * v[2]) ? 1.0 : 0.0;
    } else if (stage == 1) {
        scal[S_ALPHA] = scal[S_RZ] / v[0];
    } else {
        scal[S_BETA] = v[0] / scal[S_RZ];
        scal[S_RZ] = v[0];
        scal[S_RR] = v[1];
        scal[S_ITER] = scal[S_ITER] + 1.0;
        if (v[1] <= scal[S_RTOL2] * scal[S_BB]) scal[S_DONE] = 1.0;
    }
}

// the solution with the last direction's update still to add, rounded to the
// field storage
template <typename F>
__global__ __launch_bounds__(kBlock) void k_cg_writeback(int64_t n, const double *__restrict__ y,
                                                         const double *__restrict__ p,
                                                         const double *__restrict__ scal, F field) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) field.put(i, y[i] + scal[S_ALPHA] * p[i]);
}

// ---------------------------------------------------------------- multigrid

// One level of the hierarchy as the kernels see it (levels >= 1).
struct MgView {
    const int32_t *nbr;
    const float *w, *mass;
    const double *invd;
    double *r, *x, *e;
    const int32_t *parent;
    const RankWord *rank;
    const int32_t *vox;
    int64_t n, ld;
    Geom g;
};

// Diagonal inverse of the fine level, 1 / (1 + a sum_j w_ij): from the
// vector the init kernel wrote (region weights) or from the neighbour count.
template <bool REG>
__device__ __forceinline__ double fine_minv(const double *m, const double *mtab, int64_t i) {
    return REG ? m[i] : mtab[((const uint8_t *)m)[i]];
}

// Calls f(i, d) for the cells i of level l inside cell (X, Y, Z) of level
// l + 1, in the fixed order z, y, x ascending; d = dx | dy << 1 | dz << 2 is
// the child's offset inside the 2x2x2 block.
template <typename Fn>
__device__ __forceinline__ void mg_children(const RankWord *rank, const Geom &g, int X, int Y, int Z, Fn &&f) {
    for (int dz = 0; dz < 2; dz++) {
        const int z = 2 * Z + dz;
        if (z >= g.nz) break;
        for (int dy = 0; dy < 2; dy++) {
            const int y = 2 * Y + dy;
            if (y >= g.ny) break;
            for (int dx = 0; dx < 2; dx++) {
                const int x = 2 * X + dx;
                if (x >= g.nx) break;
                const int64_t p = geom_pos(g, x, y, z);
                const int32_t i = rank_lookup(rank[p >> 5], (uint32_t)p);
                if (i >= 0) f((int64_t)i, dx | (dy << 1) | (dz << 2));
            }
        }
    }
}

__device__ __forceinline__ void mg_cell_xyz(const int32_t *vox, int64_t i, int nx, int ny, int &x, int &y, int &z) {
    const int v = vox[i];
    x = v % nx;
    y = (v / nx) % ny;
    z = v / (nx * ny);
}

// set-up: occupancy of the next grid (every writer writes 1)
__global__ __launch_bounds__(kBlock) void k_mg_mark(const int32_t *__restrict__ vox, int64_t n, int nx, int ny,
                                                    int cnx, int cny, uint8_t *__restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int x, y, z;
    mg_cell_xyz(vox, i, nx, ny, x, y, z);
    mask[(x >> 1) + (int64_t)cnx * ((y >> 1) + (int64_t)cny * (z >> 1))] = 1;
}

// set-up: the cell of the next level that holds each cell
__global__ __launch_bounds__(kBlock) void k_mg_parent(const int32_t *__restrict__ vox, int64_t n, int nx, int ny,
                                                      const RankWord *__restrict__ crank, Geom cg,
                                                      int32_t *__restrict__ parent) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int x, y, z;
    mg_cell_xyz(vox, i, nx, ny, x, y, z);
    const int64_t p = geom_pos(cg, x >> 1, y >> 1, z >> 1);
    parent[i] = rank_lookup(crank[p >> 5], (uint32_t)p);
}

// set-up: mass and face weights of the cells of level l + 1 from level l
// (fine level: unit masses and the step's edge weights).  The weight of face
// k sums, over the children on that face (fixed order), the weight of their
// edge in direction k; the neighbour cell sums the same edges in the same
// order from its side, so both ends hold the same float.
template <bool FINE, bool REG>
__global__ __launch_bounds__(kBlock) void k_mg_coarse_op(const RankWord *__restrict__ rank, Geom g,
                                                         const int32_t *__restrict__ nbr, int64_t ld,
                                                         const float *__restrict__ w, const float *__restrict__ mass,
                                                         const uint16_t *__restrict__ rcode, CgArgs A,
                                                         const int32_t *__restrict__ cvox, int64_t cn, int cnx,
                                                         int cny, float *__restrict__ cmass,
                                                         float *__restrict__ cw, int64_t cld) {
    __shared__ double cl[VG_NREG];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = A.c[threadIdx.x];
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= cn) return;
    int X, Y, Z;
    mg_cell_xyz(cvox, c, cnx, cny, X, Y, Z);
    double m = 0.0, wk[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    mg_children(rank, g, X, Y, Z, [&](int64_t i, int d) {
        m += FINE ? 1.0 : (double)mass[i];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const int axis = k >> 1, plus = k & 1;
            if (((d >> axis) & 1) != plus) continue;   // not on face k of the block
            if (nbr[(int64_t)k * ld + i] < 0) continue;
            if (FINE) wk[k] += weight(rcode, cl, i, k, REG);
            else wk[k] += (double)w[(int64_t)k * ld + i];
        }
    });
    cmass[c] = (float)m;
#pragma unroll
    for (int k = 0; k < 6; k++) cw[(int64_t)k * cld + c] = (float)wk[k];
}

// per solve: 1 / diag of every cell, mass + a sum_k w_k
__global__ __launch_bounds__(kBlock) void k_mg_invd(const float *__restrict__ w, const float *__restrict__ mass,
                                                    int64_t n, int64_t ld, double a, double *__restrict__ invd) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) s += (double)w[(int64_t)k * ld + i];
    invd[i] = 1.0 / ((double)mass[i] + a * s);
}

// Fine-level residual of the pre-smoothed iterate: t = r - B x0 (x0 = w D^-1 r,
// written by the update kernel), one thread per voxel.
template <bool REG, int NS>
__global__ __launch_bounds__(kBlock) void k_mg_res0(CgArgs A, const double *__restrict__ r,
                                                    const double *__restrict__ x0, double *__restrict__ t,
                                                    const double *__restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    __shared__ double cl[VG_NREG];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = A.c[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.n) return;
    const double xi = x0[i];
    int64_t j[6];
    bool pres[6];
    cg_neighbours<NS>(A, i, j, pres);
    double xj[6];
#pragma unroll
    for (int k = 0; k < 6; k++) xj[k] = x0[j[k]];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        if (!pres[k]) continue;
        s += weight(A.rcode, cl, i, k, REG) * (xi - xj[k]);
    }
    t[i] = r[i] - (xi + A.a * s);
}

// Residual on level l >= 1 (into e, free until the upward pass): r - B x.
__global__ __launch_bounds__(kBlock) void k_mg_res(MgView L, double a, const double *__restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= L.n) return;
    const double xi = L.x[i];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int32_t j = L.nbr[(int64_t)k * L.ld + i];
        if (j >= 0) s += (double)L.w[(int64_t)k * L.ld + i] * (xi - L.x[j]);
    }
    L.e[i] = L.r[i] - ((double)L.mass[i] * xi + a * s);
}

// Restriction, one thread per cell of the coarser level C: the sum of the
// finer level's residuals over its children (fixed order); also C's
// pre-smoothed iterate w D^-1 r.  (Eight lanes per cell with a butterfly sum
// measured twice as slow at 512^3.)
__global__ __launch_bounds__(kBlock) void k_mg_sum(const RankWord *__restrict__ rank, Geom g,
                                                   const double *__restrict__ res, MgView C,
                                                   const double *__restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= C.n) return;
    int X, Y, Z;
    mg_cell_xyz(C.vox, c, C.g.nx, C.g.ny, X, Y, Z);
    double sum = 0.0;
    mg_children(rank, g, X, Y, Z, [&](int64_t i, int) { sum += res[i]; });
    C.r[c] = sum;
    C.x[c] = kMgOmega * sum * C.invd[c];
}

// The coarsest level (at most kMgCoarseMax cells): kMgSweeps damped Jacobi
// sweeps from zero (the first is the x the restriction wrote) in one block,
// the iterate in LDS; the result goes to e.
__global__ __launch_bounds__(kMgCoarseThreads) void k_mg_coarsest(MgView L, double a,
                                                                  const double *__restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    __shared__ double xs[2][kMgCoarseMax];
    constexpr int kPer = kMgCoarseMax / kMgCoarseThreads;
    for (int u = 0; u < kPer; u++) {
        const int64_t i = threadIdx.x + (int64_t)u * kMgCoarseThreads;
        if (i < L.n) xs[0][i] = L.x[i];
    }
    __syncthreads();
    int src = 0;
    for (int sweep = 1; sweep < kMgSweeps; sweep++) {
        for (int u = 0; u < kPer; u++) {
            const int64_t i = threadIdx.x + (int64_t)u * kMgCoarseThreads;
            if (i >= L.n) continue;
            const double xi = xs[src][i];
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int32_t j = L.nbr[(int64_t)k * L.ld + i];
                if (j >= 0) s += (double)L.w[(int64_t)k * L.ld + i] * (xi - xs[src][j]);
            }
            xs[src ^ 1][i] = xi + kMgOmega * (L.r[i] - ((double)L.mass[i] * xi + a * s)) * L.invd[i];
        }
        __syncthreads();
        src ^= 1;
    }
    for (int u = 0; u < kPer; u++) {
        const int64_t i = threadIdx.x + (int64_t)u * kMgCoarseThreads;
        if (i < L.n) L.e[i] = xs[src][i];
    }
}

// Prolongation: y = x + sol_c[parent] (any level; streaming).
__global__ __launch_bounds__(kBlock) void k_mg_pro(int64_t n, const double *__restrict__ x,
                                                   const int32_t *__restrict__ parent,
                                                   const double *__restrict__ solc, double *__restrict__ y,
                                                   const double *__restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = x[i] + solc[parent[i]];
}

// Post-smoothing on level l >= 1: x = y + w D^-1 (r - B y), y in e.
__global__ __launch_bounds__(kBlock) void k_mg_post(MgView L, double a, const double *__restrict__ scal) {
    if (scal[S_DONE] != 0.0) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= L.n) return;
    const double yi = L.e[i];
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int32_t j = L.nbr[(int64_t)k * L.ld + i];
        if (j >= 0) s += (double)L.w[(int64_t)k * L.ld + i] * (yi - L.e[j]);
    }
    L.x[i] = yi + kMgOmega * (L.r[i] - ((double)L.mass[i] * yi + a * s)) * L.invd[i];
}

// Post-smoothing on the fine level: z = y + w D^-1 (r - B y), y in t; writes
// z and the per-block r.z partials (slot 0, the grid-stride blocks of the
// other CG kernels).
template <bool REG, int NS>
__global__ __launch_bounds__(kBlock) void k_mg_post0(CgArgs A, const double *__restrict__ r,
                                                     const double *__restrict__ m, const double *__restrict__ y,
                                                     double *__restrict__ z, const double *__restrict__ scal,
                                                     double *__restrict__ part) {
    if (scal[S_DONE] != 0.0) return;
    __shared__ double lds[kWaves];
    __shared__ double cl[VG_NREG];
    __shared__ double mtab[8];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = A.c[threadIdx.x];
    if (!REG && threadIdx.x < 7) mtab[threadIdx.x] = 1.0 / (1.0 + A.a * (double)threadIdx.x);
    __syncthreads();
    double acc[1] = {0.0};
    for (int64_t it = 0;; it++) {
    const int64_t t = xcd_stride_tile(blockIdx.x, gridDim.x, it, A.ntiles);
    if (t >= A.ntiles) break;
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = t * kTile + v * kBlock + threadIdx.x;
        if (i >= A.n) continue;
        const double yi = y[i];
        int64_t j[6];
        bool pres[6];
        cg_neighbours<NS>(A, i, j, pres);
        double yj[6];
#pragma unroll
        for (int k = 0; k < 6; k++) yj[k] = y[j[k]];
        const double ri = r[i], mi = fine_minv<REG>(m, mtab, i);
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            if (!pres[k]) continue;
            s += weight(A.rcode, cl, i, k, REG) * (yi - yj[k]);
        }
        const double zi = yi + kMgOmega * (ri - (yi + A.a * s)) * mi;
        z[i] = zi;
        acc[0] += ri * zi;
    }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 4] = acc[0];
}

// The pre-smoothed fine iterate for a given r (vg_precondition): x0 = w D^-1 r.
template <bool REG>
__global__ __launch_bounds__(kBlock) void k_mg_x0(int64_t n, double a, const double *__restrict__ r,
                                                  const double *__restrict__ m, double *__restrict__ x0) {
    __shared__ double mtab[8];
    if (!REG && threadIdx.x < 7) mtab[threadIdx.x] = 1.0 / (1.0 + a * (double)threadIdx.x);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x0[i] = kMgOmega * r[i] * fine_minv<REG>(m, mtab, i);
}

// Jacobi as a separate map (vg_precondition): z = D^-1 r.
template <bool REG>
__global__ __launch_bounds__(kBlock) void k_mg_jacobi(int64_t n, double a, const double *__restrict__ r,
                                                      const double *__restrict__ m, double *__restrict__ z) {
    __shared__ double mtab[8];
    if (!REG && threadIdx.x < 7) mtab[threadIdx.x] = 1.0 / (1.0 + a * (double)threadIdx.x);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) z[i] = fine_minv<REG>(m, mtab, i) * r[i];
}

// The fine diagonal for a given a (what the init kernel writes into m).
template <bool REG, int NS>
__global__ __launch_bounds__(kBlock) void k_mg_fine_diag(CgArgs A, double *__restrict__ m) {
    __shared__ double cl[VG_NREG];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = A.c[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= A.n) return;
    int64_t j[6];
    bool pres[6];
    cg_neighbours<NS>(A, i, j, pres);
    double deg = 0.0;
#pragma unroll
    for (int k = 0; k < 6; k++)
        if (pres[k]) deg += weight(A.rcode, cl, i, k, REG);
    if (REG) m[i] = 1.0 / (1.0 + A.a * deg);
    else ((uint8_t *)m)[i] = (uint8_t)deg;
}

inline unsigned mg_grid(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

MgView mg_view(vg_sim *h, int l) {
    vg_sim::MgLevel &L = h->mg[l];
    MgView v;
    v.nbr = L.nbr;
    v.w = L.w;
    v.mass = L.mass;
    v.invd = L.invd;
    v.r = L.r;
    v.x = L.x;
    v.e = L.e;
    v.parent = L.parent;
    v.rank = L.rank;
    v.vox = L.vox;
    v.n = L.n;
    v.ld = L.cap;
    make_geom(L.nx, L.ny, L.nz, 0, &v.g);
    return v;
}

Geom fine_geom(const vg_sim *h) {
    Geom g;
    make_geom(h->nx, h->ny, h->nz, h->brick, &g);
    return g;
}

CgArgs cg_args(const vg_sim *h, double a) {
    CgArgs A;
    A.nbr = h->nbr;
    A.rcode = h->rcode;
    A.pk = packed_of(h);
    A.n = h->n;
    A.ntiles = h->ntiles;
    A.a = a;
    for (int k = 0; k < VG_NREG; k++) A.c[k] = h->c[k];
    return A;
}

// coarse weights for the current region factors (the structure is fixed)
int mg_weights(vg_sim *h, hipStream_t s) {
    const bool reg = h->rcode != nullptr;
    const CgArgs A = cg_args(h, 0.0);
    const Geom g0 = fine_geom(h);
    for (int l = 0; l + 1 < h->mg_levels; l++) {
        const vg_sim::MgLevel &F = h->mg[l];
        vg_sim::MgLevel &C = h->mg[l + 1];
        if (l == 0) {
            if (reg) hipLaunchKernelGGL((k_mg_coarse_op<true, true>), dim3(mg_grid(C.n)), dim3(kBlock), 0, s,
                                        (const RankWord *)h->rank, g0, h->nbr, h->n, nullptr, nullptr, h->rcode, A,
                                        C.vox, C.n, C.nx, C.ny, C.mass, C.w, C.cap);
            else hipLaunchKernelGGL((k_mg_coarse_op<true, false>), dim3(mg_grid(C.n)), dim3(kBlock), 0, s,
                                    (const RankWord *)h->rank, g0, h->nbr, h->n, nullptr, nullptr, h->rcode, A,
                                    C.vox, C.n, C.nx, C.ny, C.mass, C.w, C.cap);
        } else {
            const MgView fv = mg_view(h, l);
            hipLaunchKernelGGL((k_mg_coarse_op<false, false>), dim3(mg_grid(C.n)), dim3(kBlock), 0, s, F.rank, fv.g,
                               F.nbr, F.cap, F.w, F.mass, nullptr, A, C.vox, C.n, C.nx, C.ny, C.mass, C.w, C.cap);
        }
        int rc = launch_status("k_mg_coarse_op");
        if (rc) return rc;
    }
    h->mg_wdone = true;
    return VG_OK;
}

// 1 / diag of every coarse level for this a (and the weights if stale)
int mg_prepare(vg_sim *h, double a, hipStream_t s) {
    int rc;
    if (!h->mg_wdone && (rc = mg_weights(h, s))) return rc;
    for (int l = 1; l < h->mg_levels; l++) {
        vg_sim::MgLevel &L = h->mg[l];
        hipLaunchKernelGGL(k_mg_invd, dim3(mg_grid(L.n)), dim3(kBlock), 0, s, L.w, L.mass, L.n, L.cap, a, L.invd);
        if ((rc = launch_status("k_mg_invd"))) return rc;
    }
    return VG_OK;
}

// z = V-cycle(r) on the fine level: z holds x0 = w D^-1 r on entry (the
// update or init kernel wrote it), m the fine diagonal as the init kernel
// wrote it; r.z partials go to part slot 0 of G blocks.  Each level's
// result: x (levels between), e (the coarsest).
template <bool REG, int NS>
int mg_vcycle(vg_sim *h, const CgArgs &A, const double *r, const double *m, double *z, int G, hipStream_t s) {
    const int L = h->mg_levels;
    const double a = A.a;
    double *t = h->mg[0].e;   // fine residual, then the prolongated iterate
    int rc;
    hipLaunchKernelGGL((k_mg_res0<REG, NS>), dim3(mg_grid(h->n)), dim3(kBlock), 0, s, A, r, (const double *)z, t,
                       h->cg_scal);
    if ((rc = launch_status("k_mg_res0"))) return rc;
    hipLaunchKernelGGL(k_mg_sum, dim3(mg_grid(h->mg[1].n)), dim3(kBlock), 0, s, (const RankWord *)h->rank,
                       fine_geom(h), (const double *)t, mg_view(h, 1), h->cg_scal);
    if ((rc = launch_status("k_mg_sum"))) return rc;
    for (int l = 1; l + 1 < L; l++) {
        const MgView F = mg_view(h, l);
        hipLaunchKernelGGL(k_mg_res, dim3(mg_grid(F.n)), dim3(kBlock), 0, s, F, a, h->cg_scal);
        if ((rc = launch_status("k_mg_res"))) return rc;
        hipLaunchKernelGGL(k_mg_sum, dim3(mg_grid(h->mg[l + 1].n)), dim3(kBlock), 0, s, F.rank, F.g,
                           (const double *)F.e, mg_view(h, l + 1), h->cg_scal);
        if ((rc = launch_status("k_mg_sum"))) return rc;
    }
    hipLaunchKernelGGL(k_mg_coarsest, dim3(1), dim3(kMgCoarseThreads), 0, s, mg_view(h, L - 1), a, h->cg_scal);
    if ((rc = launch_status("k_mg_coarsest"))) return rc;
    for (int l = L - 2; l >= 1; l--) {
        const MgView V = mg_view(h, l);
        const double *solc = l + 1 == L - 1 ? h->mg[l + 1].e : h->mg[l + 1].x;
        hipLaunchKernelGGL(k_mg_pro, dim3(mg_grid(V.n)), dim3(kBlock), 0, s, V.n, (const double *)V.x, V.parent,
                           solc, V.e, h->cg_scal);
        if ((rc = launch_status("k_mg_pro"))) return rc;
        hipLaunchKernelGGL(k_mg_post, dim3(mg_grid(V.n)), dim3(kBlock), 0, s, V, a, h->cg_scal);
        if ((rc = launch_status("k_mg_post"))) return rc;
    }
    const double *sol1 = L == 2 ? h->mg[1].e : h->mg[1].x;
    hipLaunchKernelGGL(k_mg_pro, dim3(mg_grid(h->n)), dim3(kBlock), 0, s, h->n, (const double *)z,
                       (const int32_t *)h->mg[0].parent, sol1, t, h->cg_scal);
    if ((rc = launch_status("k_mg_pro"))) return rc;
    hipLaunchKernelGGL((k_mg_post0<REG, NS>), dim3(G), dim3(kBlock), 0, s, A, r, m, (const double *)t, z, h->cg_scal,
                       h->cg_part);
    return launch_status("k_mg_post0");
}

// storage of one pool of the bound fields
template <typename F>
F pool_acc(vg_sim *h, int pool);
template <>
PlainAcc<float> pool_acc<PlainAcc<float>>(vg_sim *h, int pool) {
    return PlainAcc<float>{(float *)h->fields + (int64_t)pool * h->n};
}
template <>
PlainAcc<double> pool_acc<PlainAcc<double>>(vg_sim *h, int pool) {
    return PlainAcc<double>{(double *)h->fields + (int64_t)pool * h->n};
}
template <>
CompAcc pool_acc<CompAcc>(vg_sim *h, int pool) {
    return CompAcc{(float *)h->fields + (int64_t)pool * h->n, h->lo + (int64_t)pool * h->n};
}

template <typename F, int NS, bool REG, bool MG>
int cg_solve_t(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
               hipStream_t s) {
    const CgArgs A = cg_args(h, a);
    const int G = h->cg_blocks;
    const F field = pool_acc<F>(h, pool);
    int rc;
    // squared tolerance (compared with squared norms; rtol^2 is exact enough)
    double host_scal[S_NSCAL] = {0, 0, 0, 0, 0, 0, 0, rtol * rtol};
    if ((rc = hip_status(hipMemcpyAsync(h->cg_scal, host_scal, sizeof(host_scal), hipMemcpyHostToDevice, s),
                         "cg scalars"))) return rc;
    if (MG && (rc = mg_prepare(h, a, s))) return rc;
    hipLaunchKernelGGL((k_cg_init<F, REG, NS, MG>), dim3(G), dim3(kBlock), 0, s, A, field, h->cg_y, h->cg_r, h->cg_z,
                       h->cg_p[0], h->cg_m, h->cg_part, h->cg_q);
    if ((rc = launch_status("k_cg_init"))) return rc;
    if (MG && (rc = mg_vcycle<REG, NS>(h, A, h->cg_r, h->cg_m, h->cg_z, G, s))) return rc;
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kBlock), 0, s, h->cg_part, G, 0, h->cg_scal);
    if ((rc = launch_status("k_cg_scalars"))) return rc;

    int launched = 0, cur = 0;
    const int chunk = 8;
    double back[S_NSCAL];
    for (;;) {
        if ((rc = hip_status(hipMemcpyAsync(back, h->cg_scal, sizeof(back), hipMemcpyDeviceToHost, s),
                             "cg scalars back"))) return rc;
        if ((rc = hip_status(hipStreamSynchronize(s), "cg sync"))) return rc;
        if (back[S_DONE] != 0.0 || launched >= max_iter) break;
        const int todo = (max_iter - launched) < chunk ? (max_iter - launched) : chunk;
        for (int it = 0; it < todo; it++) {
            hipLaunchKernelGGL((k_cg_spmv<REG, NS>), dim3(G), dim3(kBlock), 0, s, A, h->cg_z, h->cg_p[cur],
                               h->cg_p[cur ^ 1], h->cg_y, h->cg_q, h->cg_scal, h->cg_part);
            if ((rc = launch_status("k_cg_spmv"))) return rc;
            hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kBlock), 0, s, h->cg_part, G, 1, h->cg_scal);
            if ((rc = launch_status("k_cg_scalars"))) return rc;
            hipLaunchKernelGGL((k_cg_update<REG, MG>), dim3(G), dim3(kBlock), 0, s, h->n, h->ntiles, a, h->cg_q,
                               h->cg_m, h->cg_r, h->cg_z, h->cg_scal, h->cg_part);
            if ((rc = launch_status("k_cg_update"))) return rc;
            if (MG && (rc = mg_vcycle<REG, NS>(h, A, h->cg_r, h->cg_m, h->cg_z, G, s))) return rc;
            hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kBlock), 0, s, h->cg_part, G, 2, h->cg_scal);
            if ((rc = launch_status("k_cg_scalars"))) return rc;
            cur ^= 1;   // p ping-pong (iteration k writes p[k & 1]); after convergence the kernels return early
        }
        launched += todo;
    }
    hipLaunchKernelGGL((k_cg_writeback<F>), dim3((unsigned)((h->n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       h->n, h->cg_y, h->cg_p[(int)back[S_ITER] & 1], h->cg_scal, field);
    if ((rc = launch_status("k_cg_writeback"))) return rc;
    if (iters) *iters = (int)back[S_ITER];
    if (relres) *relres = back[S_BB] > 0.0 ? __builtin_sqrt(back[S_RR] / back[S_BB]) : 0.0;
    return back[S_DONE] != 0.0 ? VG_OK : VG_ENOCONV;
}

template <typename F, int NS>
int cg_solve_ns(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
                hipStream_t s) {
    const bool reg = h->rcode != nullptr;
    const bool mg = h->precond == VG_PRECOND_MG && h->mg_levels >= 2;
    if (reg) return mg ? cg_solve_t<F, NS, true, true>(h, pool, a, rtol, max_iter, iters, relres, s)
                       : cg_solve_t<F, NS, true, false>(h, pool, a, rtol, max_iter, iters, relres, s);
    return mg ? cg_solve_t<F, NS, false, true>(h, pool, a, rtol, max_iter, iters, relres, s)
              : cg_solve_t<F, NS, false, false>(h, pool, a, rtol, max_iter, iters, relres, s);
}

template <int NS>
int mg_apply_ns(vg_sim *h, double a, const double *r, double *z, hipStream_t s) {
    const CgArgs A = cg_args(h, a);
    const bool reg = h->rcode != nullptr;
    const bool mg = h->precond == VG_PRECOND_MG && h->mg_levels >= 2;
    int rc;
    if (reg) hipLaunchKernelGGL((k_mg_fine_diag<true, NS>), dim3(mg_grid(h->n)), dim3(kBlock), 0, s, A, h->cg_m);
    else hipLaunchKernelGGL((k_mg_fine_diag<false, NS>), dim3(mg_grid(h->n)), dim3(kBlock), 0, s, A, h->cg_m);
    if ((rc = launch_status("k_mg_fine_diag"))) return rc;
    if (!mg) {
        if (reg) hipLaunchKernelGGL(k_mg_jacobi<true>, dim3(mg_grid(h->n)), dim3(kBlock), 0, s, h->n, a, r, h->cg_m, z);
        else hipLaunchKernelGGL(k_mg_jacobi<false>, dim3(mg_grid(h->n)), dim3(kBlock), 0, s, h->n, a, r, h->cg_m, z);
        return launch_status("k_mg_jacobi");
    }
    // the V-cycle's kernels check the convergence flag: clear it
    if ((rc = hip_status(hipMemsetAsync(h->cg_scal, 0, sizeof(double) * S_NSCAL, s), "cg scalars"))) return rc;
    if ((rc = mg_prepare(h, a, s))) return rc;
    if (reg) hipLaunchKernelGGL(k_mg_x0<true>, dim3(mg_grid(h->n)), dim3(kBlock), 0, s, h->n, a, r, h->cg_m, z);
    else hipLaunchKernelGGL(k_mg_x0<false>, dim3(mg_grid(h->n)), dim3(kBlock), 0, s, h->n, a, r, h->cg_m, z);
    if ((rc = launch_status("k_mg_x0"))) return rc;
    return reg ? mg_vcycle<true, NS>(h, A, r, h->cg_m, z, h->cg_blocks, s)
               : mg_vcycle<false, NS>(h, A, r, h->cg_m, z, h->cg_blocks, s);
}

// the explicit step's neighbour source
template <typename F>
int cg_solve(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
             hipStream_t s) {
    if (use_relative(h)) return cg_solve_ns<F, NS_REL>(h, pool, a, rtol, max_iter, iters, relres, s);
    if (use_offsets(h)) return cg_solve_ns<F, NS_OFF>(h, pool, a, rtol, max_iter, iters, relres, s);
    return cg_solve_ns<F, NS_TABLE>(h, pool, a, rtol, max_iter, iters, relres, s);
}

}  // namespace

void mg_plan(vg_sim *h) {
    h->mg[0].nx = h->nx;
    h->mg[0].ny = h->ny;
    h->mg[0].nz = h->nz;
    h->mg[0].cap = h->n;
    int l = 0;
    while (l + 1 < VG_MG_MAX_LEVELS) {
        const vg_sim::MgLevel &F = h->mg[l];
        if (F.nx <= 1 && F.ny <= 1 && F.nz <= 1) break;
        vg_sim::MgLevel &C = h->mg[l + 1];
        C.nx = (F.nx + 1) / 2;
        C.ny = (F.ny + 1) / 2;
        C.nz = (F.nz + 1) / 2;
        const int64_t cells = (int64_t)C.nx * C.ny * C.nz;
        C.cap = cells < F.cap ? cells : F.cap;   // every cell holds at least one cell of the level below
        l++;
    }
    h->mg_plan_levels = l + 1;
}

int mg_build(vg_sim *h, hipStream_t s) {
    h->mg_levels = 0;
    h->mg_wdone = false;
    if (h->n == 0) return VG_OK;
    h->mg[0].n = h->n;
    int l = 0, rc;
    while (l + 1 < h->mg_plan_levels) {
        const vg_sim::MgLevel &F = h->mg[l];
        if (l > 0 && F.n <= kMgCoarsest) break;
        vg_sim::MgLevel &C = h->mg[l + 1];
        const int32_t *fvox = l == 0 ? h->vox : F.vox;
        int32_t *fparent = l == 0 ? h->mg[0].parent : F.parent;
        const size_t cells = (size_t)C.nx * C.ny * C.nz;
        if ((rc = hip_status(hipMemsetAsync(h->mg_mask, 0, cells, s), "clear occupancy"))) return rc;
        hipLaunchKernelGGL(k_mg_mark, dim3(mg_grid(F.n)), dim3(kBlock), 0, s, fvox, F.n, F.nx, F.ny, C.nx, C.ny,
                           h->mg_mask);
        if ((rc = launch_status("k_mg_mark"))) return rc;
        int64_t cn = 0;
        if ((rc = vg_count_pores(h->mg_mask, C.nx, C.ny, C.nz, 0, C.rank, &cn, s))) return rc;
        if (cn < 1 || cn > C.cap) { set_error("multigrid level %d: %lld cells", l + 1, (long long)cn); return VG_EHIP; }
        C.n = cn;
        if ((rc = vg_build_graph(C.rank, C.nx, C.ny, C.nz, 0, 0u, 0, cn, C.cap, C.vox, C.nbr, s))) return rc;
        Geom cg;
        make_geom(C.nx, C.ny, C.nz, 0, &cg);
        hipLaunchKernelGGL(k_mg_parent, dim3(mg_grid(F.n)), dim3(kBlock), 0, s, fvox, F.n, F.nx, F.ny,
                           (const RankWord *)C.rank, cg, fparent);
        if ((rc = launch_status("k_mg_parent"))) return rc;
        l++;
    }
    h->mg_levels = l + 1;
    if (h->mg_levels >= 2 && h->mg[l].n > kMgCoarseMax) {
        set_error("multigrid: coarsest level of %lld cells", (long long)h->mg[l].n);
        return VG_EINVAL;
    }
    return mg_weights(h, s);
}

int mg_apply(vg_sim *h, double a, const double *r, double *z, hipStream_t s) {
    if (h->n == 0) return VG_OK;
    if (use_relative(h)) return mg_apply_ns<NS_REL>(h, a, r, z, s);
    if (use_offsets(h)) return mg_apply_ns<NS_OFF>(h, a, r, z, s);
    return mg_apply_ns<NS_TABLE>(h, a, r, z, s);
}

int run_cg(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
           hipStream_t s) {
    if (h->n == 0) {
        if (iters) *iters = 0;
        if (relres) *relres = 0.0;
        return VG_OK;
    }
    if (h->prec == VG_F32C) return cg_solve<CompAcc>(h, pool, a, rtol, max_iter, iters, relres, s);
    if (h->prec == VG_F64) return cg_solve<PlainAcc<double>>(h, pool, a, rtol, max_iter, iters, relres, s);
    return cg_solve<PlainAcc<float>>(h, pool, a, rtol, max_iter, iters, relres, s);
}

}  // namespace vg
