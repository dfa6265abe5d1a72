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
#include "vg_internal.h"

namespace vg {
namespace {

enum { S_RZ = 0, S_RR, S_BB, S_ALPHA, S_BETA, S_DONE, S_ITER, S_RTOL2, S_NSCAL = 8 };

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

template <typename F, bool REG, int NS>
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
        z[i] = zi;
        p[i] = zi;
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
        for (int u = 0; u < 3; u++) part[(int64_t)blockIdx.x * 4 + u] = acc[u];
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
template <bool REG>
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
        const double zi = (REG ? m[i] : mtab[((const uint8_t *)m)[i]]) * ri;
        r[i] = ri;
        z[i] = zi;
        acc[0] += ri * zi;
        acc[1] += ri * ri;
    }
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * 4] = acc[0];
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

template <typename F, int NS>
int cg_solve_ns(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
                hipStream_t s) {
    CgArgs A;
    A.nbr = h->nbr;
    A.rcode = h->rcode;
    A.pk = packed_of(h);
    A.n = h->n;
    A.ntiles = h->ntiles;
    A.a = a;
    for (int k = 0; k < VG_NREG; k++) A.c[k] = h->c[k];
    const bool reg = h->rcode != nullptr;
    const int G = h->cg_blocks;
    const F field = pool_acc<F>(h, pool);
    int rc;
    // squared tolerance (compared with squared norms; rtol^2 is exact enough)
    double host_scal[S_NSCAL] = {0, 0, 0, 0, 0, 0, 0, rtol * rtol};
    if ((rc = hip_status(hipMemcpyAsync(h->cg_scal, host_scal, sizeof(host_scal), hipMemcpyHostToDevice, s),
                         "cg scalars"))) return rc;
    if (reg) hipLaunchKernelGGL((k_cg_init<F, true, NS>), dim3(G), dim3(kBlock), 0, s, A, field, h->cg_y, h->cg_r,
                                h->cg_z, h->cg_p[0], h->cg_m, h->cg_part, h->cg_q);
    else hipLaunchKernelGGL((k_cg_init<F, false, NS>), dim3(G), dim3(kBlock), 0, s, A, field, h->cg_y, h->cg_r,
                            h->cg_z, h->cg_p[0], h->cg_m, h->cg_part, h->cg_q);
    if ((rc = launch_status("k_cg_init"))) return rc;
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
            if (reg) hipLaunchKernelGGL((k_cg_spmv<true, NS>), dim3(G), dim3(kBlock), 0, s, A, h->cg_z, h->cg_p[cur],
                                        h->cg_p[cur ^ 1], h->cg_y, h->cg_q, h->cg_scal, h->cg_part);
            else hipLaunchKernelGGL((k_cg_spmv<false, NS>), dim3(G), dim3(kBlock), 0, s, A, h->cg_z, h->cg_p[cur],
                                    h->cg_p[cur ^ 1], h->cg_y, h->cg_q, h->cg_scal, h->cg_part);
            if ((rc = launch_status("k_cg_spmv"))) return rc;
            hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(kBlock), 0, s, h->cg_part, G, 1, h->cg_scal);
            if ((rc = launch_status("k_cg_scalars"))) return rc;
            if (reg) hipLaunchKernelGGL(k_cg_update<true>, dim3(G), dim3(kBlock), 0, s, h->n, h->ntiles, a, h->cg_q,
                                        h->cg_m, h->cg_r, h->cg_z, h->cg_scal, h->cg_part);
            else hipLaunchKernelGGL(k_cg_update<false>, dim3(G), dim3(kBlock), 0, s, h->n, h->ntiles, a, h->cg_q,
                                    h->cg_m, h->cg_r, h->cg_z, h->cg_scal, h->cg_part);
            if ((rc = launch_status("k_cg_update"))) return rc;
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

// the explicit step's neighbour source
template <typename F>
int cg_solve(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
             hipStream_t s) {
    if (use_relative(h)) return cg_solve_ns<F, NS_REL>(h, pool, a, rtol, max_iter, iters, relres, s);
    if (use_offsets(h)) return cg_solve_ns<F, NS_OFF>(h, pool, a, rtol, max_iter, iters, relres, s);
    return cg_solve_ns<F, NS_TABLE>(h, pool, a, rtol, max_iter, iters, relres, s);
}

}  // namespace

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
