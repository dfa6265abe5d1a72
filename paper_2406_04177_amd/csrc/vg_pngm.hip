// Pore-network (PNGM) objectives of Sec. V on a coarse partition of the
// voxel graph: the primitives are the bricks of side b (pore voxels of one
// brick), adjacent when a pore-voxel face joins them.
//
//   k_brick_stats    per brick: pore voxels, coordinate sums (centres of
//                    gravity) and pore-voxel faces shared with the next
//                    brick along +x, +y, +z (contact surface S)
//   k_pngm_loss_grad objective L1 (explicit scheme 3 residual) or L2
//                    (implicit scheme 4 residual) over data pairs of
//                    primitive masses, and its gradient per directed edge
//   k_pngm_step      one explicit PNGM step (scheme 3)
//   k_pngm_jacobi    one Jacobi sweep of the implicit PNGM step (scheme 4)
//                    on the concentrations, with the row residuals
//   k_sign_update    the normalised-gradient update of Sec. V.A
//
// Inner term x_j / v_j (the printed x_i / v_j is read as a slip); theta is
// one parameter per ordered pair; dL2/dtheta carries the minus sign of
// d r2 / d theta, which the printed formula drops.
#include <cmath>
#include <mutex>

#include "vg_internal.h"

#pragma clang fp contract(off)

namespace vg {
namespace {

inline unsigned blocks_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *__restrict__ p, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < cnt) p[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long *__restrict__ p, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < cnt) p[i] = 0ull;
}

struct BrickGeom {
    int nx, ny, nz, b, nbx, nby, nbz;
};

__device__ __forceinline__ int64_t brick_of(const BrickGeom &G, int x, int y, int z) {
    return ((int64_t)(z / G.b) * G.nby + y / G.b) * G.nbx + x / G.b;
}

// Integer sums (atomic adds of integers are exact and order-free, so the
// result is deterministic).
__global__ __launch_bounds__(kBlock) void k_brick_stats(const int32_t *__restrict__ vox,
                                                        const int32_t *__restrict__ nbr, int64_t n, BrickGeom G,
                                                        uint32_t *__restrict__ contact,
                                                        unsigned long long *__restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t p = vox[i];
    const int x = (int)(p % G.nx), y = (int)((p / G.nx) % G.ny), z = (int)(p / ((int64_t)G.nx * G.ny));
    const int64_t k = brick_of(G, x, y, z);
    atomicAdd(&sums[k * 4 + 0], 1ull);
    atomicAdd(&sums[k * 4 + 1], (unsigned long long)x);
    atomicAdd(&sums[k * 4 + 2], (unsigned long long)y);
    atomicAdd(&sums[k * 4 + 3], (unsigned long long)z);
    // +x, +y, +z slots: a face shared with the next brick along that axis
    const int axis_coord[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int32_t j = nbr[(int64_t)(2 * a + 1) * n + i];
        if (j >= 0 && (axis_coord[a] + 1) % G.b == 0) atomicAdd(&contact[k * 3 + a], 1u);
    }
}

// ---------------------------------------------------------------- partition
// The primitive graph of the brick partition from the brick statistics:
// primitive i = the i-th brick (raster order of bricks) holding pore voxels;
// v_i its pore voxels; offsets_i the start of its range in a brick-ordered
// compact list; adjacency in CSR with ascending columns: a brick's
// neighbours -z, -y, -x, +x, +y, +z have ascending brick (so primitive)
// indices; S = the pore-voxel faces between the two bricks, d = the distance
// of their centres of gravity (coordinate sums / count, exact integer sums).

__device__ __forceinline__ void brick_xyz(const BrickGeom &G, int64_t k, int64_t &bx, int64_t &by, int64_t &bz) {
    bx = k % G.nbx;
    by = (k / G.nbx) % G.nby;
    bz = k / ((int64_t)G.nbx * G.nby);
}

// Neighbour brick of k in order o = 0..5 (-z, -y, -x, +x, +y, +z) and the
// faces between them (0: none or outside the box).
__device__ __forceinline__ uint32_t brick_link(const BrickGeom &G, const uint32_t *__restrict__ contact, int64_t k,
                                               int o, int64_t &kn) {
    int64_t bx, by, bz;
    brick_xyz(G, k, bx, by, bz);
    const int64_t sx = 1, sy = G.nbx, sz = (int64_t)G.nbx * G.nby;
    switch (o) {
        case 0: kn = k - sz; return bz > 0 ? contact[kn * 3 + 2] : 0u;
        case 1: kn = k - sy; return by > 0 ? contact[kn * 3 + 1] : 0u;
        case 2: kn = k - sx; return bx > 0 ? contact[kn * 3 + 0] : 0u;
        case 3: kn = k + sx; return contact[k * 3 + 0];   // faces exist only when brick k + 1 does
        case 4: kn = k + sy; return contact[k * 3 + 1];
        default: kn = k + sz; return contact[k * 3 + 2];
    }
}

constexpr int kScanThreads = 1024;

// One block: each thread takes a contiguous chunk of bricks, counts its
// primitives, edges and pore voxels, the block scans the counts (exclusive,
// in LDS), and each thread numbers its chunk's primitives and writes their
// volume, range start, first edge and brick; scal = {q, E}.
__global__ __launch_bounds__(kScanThreads) void k_prim_scan(const uint32_t *__restrict__ contact,
                                                            const unsigned long long *__restrict__ sums,
                                                            BrickGeom G, int64_t nb, int32_t *__restrict__ pid,
                                                            double *__restrict__ v, int64_t *__restrict__ offsets,
                                                            int32_t *__restrict__ bricks, int64_t *__restrict__ row,
                                                            int64_t *__restrict__ scal) {
    __shared__ int64_t sc[3][kScanThreads];
    const int t = threadIdx.x;
    const int64_t chunk = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t k0 = t * chunk < nb ? t * chunk : nb, k1 = k0 + chunk < nb ? k0 + chunk : nb;
    int64_t cnt[3] = {0, 0, 0};   // primitives, edges, pore voxels
    for (int64_t k = k0; k < k1; k++) {
        const unsigned long long c = sums[k * 4];
        if (!c) continue;
        cnt[0] += 1;
        cnt[2] += (int64_t)c;
        for (int o = 0; o < 6; o++) {
            int64_t kn;
            cnt[1] += brick_link(G, contact, k, o, kn) ? 1 : 0;
        }
    }
    for (int a = 0; a < 3; a++) sc[a][t] = cnt[a];
    __syncthreads();
    for (int w = 1; w < kScanThreads; w <<= 1) {   // inclusive scan (Hillis-Steele)
        int64_t add[3] = {0, 0, 0};
        if (t >= w)
            for (int a = 0; a < 3; a++) add[a] = sc[a][t - w];
        __syncthreads();
        for (int a = 0; a < 3; a++) sc[a][t] += add[a];
        __syncthreads();
    }
    int64_t base[3];
    for (int a = 0; a < 3; a++) base[a] = sc[a][t] - cnt[a];
    for (int64_t k = k0; k < k1; k++) {
        const unsigned long long c = sums[k * 4];
        if (!c) {
            pid[k] = -1;
            continue;
        }
        const int64_t i = base[0]++;
        pid[k] = (int32_t)i;
        v[i] = (double)c;
        offsets[i] = base[2];
        base[2] += (int64_t)c;
        bricks[i] = (int32_t)k;
        row[i] = base[1];
        for (int o = 0; o < 6; o++) {
            int64_t kn;
            base[1] += brick_link(G, contact, k, o, kn) ? 1 : 0;
        }
    }
    if (t == kScanThreads - 1) {
        const int64_t q = sc[0][t], E = sc[1][t];
        row[q] = E;
        offsets[q] = sc[2][t];
        scal[0] = q;
        scal[1] = E;
    }
}

// One thread per brick: the CSR row of its primitive.
__global__ __launch_bounds__(kBlock) void k_prim_fill(const uint32_t *__restrict__ contact,
                                                      const unsigned long long *__restrict__ sums, BrickGeom G,
                                                      int64_t nb, const int32_t *__restrict__ pid,
                                                      const int64_t *__restrict__ row, int32_t *__restrict__ col,
                                                      double *__restrict__ S, double *__restrict__ dist) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= nb || !sums[k * 4]) return;
    const double ck = (double)sums[k * 4];
    const double cx = (double)sums[k * 4 + 1] / ck, cy = (double)sums[k * 4 + 2] / ck,
                 cz = (double)sums[k * 4 + 3] / ck;
    int64_t e = row[pid[k]];
    for (int o = 0; o < 6; o++) {
        int64_t kn;
        const uint32_t f = brick_link(G, contact, k, o, kn);
        if (!f) continue;
        const double cn = (double)sums[kn * 4];
        const double dx = cx - (double)sums[kn * 4 + 1] / cn, dy = cy - (double)sums[kn * 4 + 2] / cn,
                     dz = cz - (double)sums[kn * 4 + 3] / cn;
        col[e] = pid[kn];
        S[e] = (double)f;
        dist[e] = sqrt((dx * dx + dy * dy) + dz * dz);
        e++;
    }
}

// One thread per primitive row i: for every data pair p the residual of row
// i, then the gradient terms of the row's edges (each edge belongs to one
// row, so no two threads write the same entry) and the row's share of the
// loss.
__global__ __launch_bounds__(kBlock) void k_pngm_loss_grad(const double *__restrict__ X, const double *__restrict__ Y,
                                                           int64_t l, int64_t q, const double *__restrict__ v,
                                                           const int64_t *__restrict__ row,
                                                           const int32_t *__restrict__ col,
                                                           const double *__restrict__ theta, double c, int objective,
                                                           double *__restrict__ rowloss, double *__restrict__ grad) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    const int64_t e0 = row[i], e1 = row[i + 1];
    const double inv = 1.0 / (double)(l * q);
    for (int64_t e = e0; e < e1; e++) grad[e] = 0.0;
    double acc = 0.0;
    for (int64_t p = 0; p < l; p++) {
        const double *x = X + p * q, *y = Y + p * q;
        const double *zz = objective == 1 ? x : y;       // the concentrations of the flux term
        const double si = zz[i] / v[i];
        double s = 0.0;
        for (int64_t e = e0; e < e1; e++) {
            const int32_t j = col[e];
            s += theta[e] * (si - zz[j] / v[j]);
        }
        const double r = objective == 1 ? y[i] - x[i] + c * s : x[i] - y[i] - c * s;
        for (int64_t e = e0; e < e1; e++) {
            const int32_t j = col[e];
            const double t = 2.0 * inv * r * c * (si - zz[j] / v[j]);
            grad[e] = objective == 1 ? grad[e] + t : grad[e] - t;
        }
        acc += r * r * inv;
    }
    rowloss[i] = acc;
}

__global__ __launch_bounds__(kBlock) void k_sum_rows(const double *__restrict__ rowloss, int64_t q,
                                                     double *__restrict__ out) {
    __shared__ double lds[kWaves];
    double v[1] = {0.0};
    for (int64_t i = threadIdx.x; i < q; i += kBlock) v[0] += rowloss[i];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[0] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_pngm_step(const double *__restrict__ m, double *__restrict__ out,
                                                      int64_t q, const double *__restrict__ v,
                                                      const int64_t *__restrict__ row,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ theta, double c) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    const double si = m[i] / v[i];
    double s = 0.0;
    for (int64_t e = row[i]; e < row[i + 1]; e++) {
        const int32_t j = col[e];
        s += theta[e] * (si - m[j] / v[j]);
    }
    out[i] = m[i] - c * s;
}

// Scheme 4 in concentrations s = m / v: (v_i + c sum_e theta_e) s_i -
// c sum_e theta_e s_j = m_i.  Every row is strictly diagonally dominant
// (v_i >= 1), so Jacobi converges.  One sweep writes s_out from s_in and the
// squared residual of s_in per row (mass units) into rowres.
__global__ __launch_bounds__(kBlock) void k_pngm_jacobi(const double *__restrict__ m,
                                                        const double *__restrict__ s_in,
                                                        double *__restrict__ s_out, int64_t q,
                                                        const double *__restrict__ v,
                                                        const int64_t *__restrict__ row,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ theta, double c,
                                                        double *__restrict__ rowres) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    double sum_t = 0.0, sum_ts = 0.0;
    for (int64_t e = row[i]; e < row[i + 1]; e++) {
        sum_t += theta[e];
        sum_ts += theta[e] * s_in[col[e]];
    }
    const double diag = v[i] + c * sum_t;
    const double r = m[i] - (diag * s_in[i] - c * sum_ts);
    s_out[i] = (m[i] + c * sum_ts) / diag;
    rowres[i] = r * r;
}

__global__ __launch_bounds__(kBlock) void k_pngm_conc(const double *__restrict__ m, const double *__restrict__ v,
                                                      double *__restrict__ s, double *__restrict__ msq, int64_t q) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q) return;
    s[i] = m[i] / v[i];
    msq[i] = m[i] * m[i];
}

__global__ __launch_bounds__(kBlock) void k_pngm_mass(const double *__restrict__ s, const double *__restrict__ v,
                                                      double *__restrict__ out, int64_t q) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < q) out[i] = s[i] * v[i];
}

// theta_e <- clamp(theta_e - lr * scale_e * sign(g_e), lo_e, hi_e); a zero
// derivative gives no move.
__global__ __launch_bounds__(kBlock) void k_sign_update(double *__restrict__ theta, const double *__restrict__ g,
                                                        int64_t cnt, double lr, const double *__restrict__ scale,
                                                        const double *__restrict__ lo,
                                                        const double *__restrict__ hi) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= cnt) return;
    double t = theta[e];
    if (g[e] > 0.0) t -= lr * scale[e];
    else if (g[e] < 0.0) t += lr * scale[e];
    t = t < lo[e] ? lo[e] : t;
    t = t > hi[e] ? hi[e] : t;
    theta[e] = t;
}

}  // namespace
}  // namespace vg

using namespace vg;

extern "C" int vg_brick_stats(const int32_t *vox_d, const int32_t *nbr_d, int64_t n, int nx, int ny, int nz, int b,
                              uint32_t *contact_d, unsigned long long *sums_d, void *stream) {
    if (n < 0 || nx <= 0 || ny <= 0 || nz <= 0 || b <= 0 || !contact_d || !sums_d || (n > 0 && (!vox_d || !nbr_d))) {
        set_error("bad brick-statistics arguments");
        return VG_EINVAL;
    }
    BrickGeom G{nx, ny, nz, b, (nx + b - 1) / b, (ny + b - 1) / b, (nz + b - 1) / b};
    const int64_t nb = (int64_t)G.nbx * G.nby * G.nbz;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(nb * 3)), dim3(kBlock), 0, s, contact_d, nb * 3);
    int rc = launch_status("k_fill_u32");
    if (rc) return rc;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(nb * 4)), dim3(kBlock), 0, s, sums_d, nb * 4);
    if ((rc = launch_status("k_fill_u64"))) return rc;
    if (n == 0) return VG_OK;
    hipLaunchKernelGGL(k_brick_stats, dim3(blocks_for(n)), dim3(kBlock), 0, s, vox_d, nbr_d, n, G, contact_d, sums_d);
    return launch_status("k_brick_stats");
}

namespace {
// Brick grid, bricks, primitive and edge capacities of a partition.
int partition_sizes(int nx, int ny, int nz, int b, BrickGeom *G, int64_t *nb, int64_t *max_edges) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || b <= 0) {
        set_error("bad partition shape or brick size");
        return VG_EINVAL;
    }
    *G = BrickGeom{nx, ny, nz, b, (nx + b - 1) / b, (ny + b - 1) / b, (nz + b - 1) / b};
    const int64_t X = G->nbx, Y = G->nby, Z = G->nbz;
    *nb = X * Y * Z;
    *max_edges = 2 * ((X - 1) * Y * Z + X * (Y - 1) * Z + X * Y * (Z - 1));   // both directions of every pair
    if (*nb >= ((int64_t)1 << 31)) {
        set_error("too many bricks (%lld)", (long long)*nb);
        return VG_EINVAL;
    }
    return VG_OK;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t partition_work(int64_t nb) {
    return align256(sizeof(uint32_t) * 3 * (size_t)nb) + align256(sizeof(unsigned long long) * 4 * (size_t)nb) +
           align256(sizeof(int32_t) * (size_t)nb) + align256(sizeof(int64_t) * 2);
}
}  // namespace

extern "C" int vg_pngm_partition_bytes(int nx, int ny, int nz, int b, size_t *work_bytes, int64_t *max_prims,
                                       int64_t *max_edges) {
    if (!work_bytes || !max_prims || !max_edges) {
        set_error("null pointer argument");
        return VG_EINVAL;
    }
    BrickGeom G;
    int64_t nb = 0, me = 0;
    const int rc = partition_sizes(nx, ny, nz, b, &G, &nb, &me);
    if (rc) return rc;
    *work_bytes = partition_work(nb);
    *max_prims = nb;
    *max_edges = me;
    return VG_OK;
}

extern "C" int vg_pngm_partition(const int32_t *vox_d, const int32_t *nbr_d, int64_t n, int nx, int ny, int nz, int b,
                                 void *work_d, size_t work_bytes, double *v_d, int64_t *offsets_d, int32_t *bricks_d,
                                 int64_t *row_d, int32_t *col_d, double *S_d, double *dist_d, int64_t *q_out,
                                 int64_t *e_out, void *stream) {
    BrickGeom G;
    int64_t nb = 0, me = 0;
    int rc = partition_sizes(nx, ny, nz, b, &G, &nb, &me);
    if (rc) return rc;
    if (n < 0 || !q_out || !e_out || !work_d || !v_d || !offsets_d || !bricks_d || !row_d ||
        (me > 0 && (!col_d || !S_d || !dist_d)) || (n > 0 && (!vox_d || !nbr_d))) {
        set_error("bad partition arguments");
        return VG_EINVAL;
    }
    if (work_bytes < partition_work(nb)) {
        set_error("partition workspace too small: %zu < %zu bytes", work_bytes, partition_work(nb));
        return VG_EINVAL;
    }
    char *w = (char *)work_d;
    uint32_t *contact = (uint32_t *)w;
    w += align256(sizeof(uint32_t) * 3 * (size_t)nb);
    unsigned long long *sums = (unsigned long long *)w;
    w += align256(sizeof(unsigned long long) * 4 * (size_t)nb);
    int32_t *pid = (int32_t *)w;
    w += align256(sizeof(int32_t) * (size_t)nb);
    int64_t *scal = (int64_t *)w;
    if ((rc = vg_brick_stats(vox_d, nbr_d, n, nx, ny, nz, b, contact, sums, stream))) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_prim_scan, dim3(1), dim3(kScanThreads), 0, s, contact, sums, G, nb, pid, v_d, offsets_d,
                       bricks_d, row_d, scal);
    if ((rc = launch_status("k_prim_scan"))) return rc;
    hipLaunchKernelGGL(k_prim_fill, dim3(blocks_for(nb)), dim3(kBlock), 0, s, contact, sums, G, nb, pid, row_d, col_d,
                       S_d, dist_d);
    if ((rc = launch_status("k_prim_fill"))) return rc;
    int64_t host[2] = {0, 0};
    if ((rc = hip_status(hipMemcpyAsync(host, scal, sizeof(host), hipMemcpyDeviceToHost, s), "partition sizes")))
        return rc;
    if ((rc = hip_status(hipStreamSynchronize(s), "partition sync"))) return rc;
    *q_out = host[0];
    *e_out = host[1];
    return VG_OK;
}

extern "C" int vg_pngm_loss_grad(const double *X_d, const double *Y_d, int64_t l, int64_t q, const double *v_d,
                                 const int64_t *row_d, const int32_t *col_d, const double *theta_d, double c,
                                 int objective, double *rowloss_d, double *loss_d, double *grad_d, void *stream) {
    if (l <= 0 || q <= 0 || (objective != 1 && objective != 2) || !std::isfinite(c) || !X_d || !Y_d || !v_d ||
        !row_d || !col_d || !theta_d || !rowloss_d || !loss_d || !grad_d) {
        set_error("bad PNGM objective arguments");
        return VG_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pngm_loss_grad, dim3(blocks_for(q)), dim3(kBlock), 0, s, X_d, Y_d, l, q, v_d, row_d, col_d,
                       theta_d, c, objective, rowloss_d, grad_d);
    int rc = launch_status("k_pngm_loss_grad");
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kBlock), 0, s, rowloss_d, q, loss_d);
    return launch_status("k_sum_rows");
}

extern "C" int vg_pngm_step(const double *m_d, double *out_d, int64_t q, const double *v_d, const int64_t *row_d,
                            const int32_t *col_d, const double *theta_d, double c, void *stream) {
    if (q < 0 || !std::isfinite(c) || (q > 0 && (!m_d || !out_d || !v_d || !row_d || !col_d || !theta_d)) ||
        (q > 0 && m_d == out_d)) {
        set_error("bad PNGM step arguments");
        return VG_EINVAL;
    }
    if (q == 0) return VG_OK;
    hipLaunchKernelGGL(k_pngm_step, dim3(blocks_for(q)), dim3(kBlock), 0, (hipStream_t)stream, m_d, out_d, q, v_d,
                       row_d, col_d, theta_d, c);
    return launch_status("k_pngm_step");
}

namespace {

// The implicit PNGM step with its 3 q + 2 FP64 scratch entries at work_d
// (arguments already checked): sa, sb (concentration iterates), the row
// residuals and two scalars.  Every entry is written before it is read, so
// the scratch needs no clearing.
int pngm_implicit(const double *m_d, double *out_d, int64_t q, const double *v_d, const int64_t *row_d,
                  const int32_t *col_d, const double *theta_d, double c, double rtol, int max_iter, double *work_d,
                  int *iters_out, double *relres_out, void *stream) {
    *iters_out = 0;
    *relres_out = 0.0;
    if (q == 0) return VG_OK;
    hipStream_t s = (hipStream_t)stream;
    double *sa = work_d, *sb = work_d + q, *rowres = work_d + 2 * q, *scal = work_d + 3 * q;
    const unsigned nb = blocks_for(q);
    hipLaunchKernelGGL(k_pngm_conc, dim3(nb), dim3(kBlock), 0, s, m_d, v_d, sa, rowres, q);
    int rc = launch_status("k_pngm_conc");
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kBlock), 0, s, rowres, q, scal + 1);
    if ((rc = launch_status("k_sum_rows"))) return rc;
    double host[2] = {0.0, 0.0};
    if (hipMemcpyAsync(&host[1], scal + 1, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("PNGM implicit step: reading the right-hand side norm failed");
        return VG_EHIP;
    }
    const double bnorm = std::sqrt(host[1]);
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_pngm_mass, dim3(nb), dim3(kBlock), 0, s, sa, v_d, out_d, q);
        return launch_status("k_pngm_mass");
    }
    // sweeps in groups of 8; the residual read after a group is that of the
    // last sweep's input (sb after the swap), and that input is the result,
    // so the reported residual is the result's own
    int it = 0;
    double rel = INFINITY;
    while (it < max_iter) {
        for (int k = 0; k < 8 && it < max_iter; k++, it++) {
            hipLaunchKernelGGL(k_pngm_jacobi, dim3(nb), dim3(kBlock), 0, s, m_d, sa, sb, q, v_d, row_d, col_d,
                               theta_d, c, rowres);
            if ((rc = launch_status("k_pngm_jacobi"))) return rc;
            double *t = sa;
            sa = sb;
            sb = t;
        }
        hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(kBlock), 0, s, rowres, q, scal);
        if ((rc = launch_status("k_sum_rows"))) return rc;
        if (hipMemcpyAsync(&host[0], scal, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("PNGM implicit step: reading the residual failed");
            return VG_EHIP;
        }
        rel = std::sqrt(host[0]) / bnorm;
        if (rel <= rtol) break;
    }
    hipLaunchKernelGGL(k_pngm_mass, dim3(nb), dim3(kBlock), 0, s, sb, v_d, out_d, q);
    if ((rc = launch_status("k_pngm_mass"))) return rc;
    *iters_out = it;
    *relres_out = rel;
    if (!(rel <= rtol)) {
        set_error("PNGM implicit step did not reach rtol within max_iter sweeps");
        return VG_ENOCONV;
    }
    return VG_OK;
}

bool pngm_implicit_args_ok(const double *m_d, const double *out_d, int64_t q, const double *v_d,
                           const int64_t *row_d, const int32_t *col_d, const double *theta_d, double c, double rtol,
                           int max_iter, const int *iters_out, const double *relres_out) {
    return !(q < 0 || !std::isfinite(c) || c < 0 || !(rtol > 0) || max_iter < 1 || !iters_out || !relres_out ||
             (q > 0 && (!m_d || !out_d || !v_d || !row_d || !col_d || !theta_d || out_d == m_d)));
}

// Scratch of vg_pngm_implicit_step_noalloc: a file-scope device array, one
// copy per GPU the library runs on, held until the process ends.  In host
// code its name is only a stand-in; the device address of each GPU's copy is
// looked up once per device (that device current) and kept.
static __device__ __align__(256) double scratch[3 * VG_PNGM_NOALLOC_MAX_Q + 2];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(double **out) {
    int dev = -1;
    int rc = hip_status(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the static scratch tracks", dev, kMaxDevices);
        return VG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *p = nullptr;
        rc = hip_status(hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc) return rc;
        if (!p) {
            set_error("hipGetSymbolAddress(scratch) returned a null address");
            return VG_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VG_OK;
}

}  // namespace

extern "C" int vg_pngm_implicit_step(const double *m_d, double *out_d, int64_t q, const double *v_d,
                                     const int64_t *row_d, const int32_t *col_d, const double *theta_d, double c,
                                     double rtol, int max_iter, double *work_d, int *iters_out, double *relres_out,
                                     void *stream) {
    if (!pngm_implicit_args_ok(m_d, out_d, q, v_d, row_d, col_d, theta_d, c, rtol, max_iter, iters_out, relres_out) ||
        (q > 0 && (!work_d || (out_d < work_d + 3 * q + 2 && work_d < out_d + q)))) {
        set_error("bad PNGM implicit-step arguments");
        return VG_EINVAL;
    }
    return pngm_implicit(m_d, out_d, q, v_d, row_d, col_d, theta_d, c, rtol, max_iter, work_d, iters_out, relres_out,
                         stream);
}

extern "C" int vg_pngm_implicit_step_noalloc(const double *m_d, double *out_d, int64_t q, const double *v_d,
                                             const int64_t *row_d, const int32_t *col_d, const double *theta_d,
                                             double c, double rtol, int max_iter, int *iters_out, double *relres_out,
                                             void *stream) {
    if (!pngm_implicit_args_ok(m_d, out_d, q, v_d, row_d, col_d, theta_d, c, rtol, max_iter, iters_out, relres_out)) {
        set_error("bad PNGM implicit-step arguments");
        return VG_EINVAL;
    }
    if (q > VG_PNGM_NOALLOC_MAX_Q) {
        set_error("q = %lld primitives exceeds the static scratch (at most %d)", (long long)q, VG_PNGM_NOALLOC_MAX_Q);
        return VG_EINVAL;
    }
    double *work = nullptr;
    int rc = scratch_of_current_device(&work);
    if (rc) return rc;
    return pngm_implicit(m_d, out_d, q, v_d, row_d, col_d, theta_d, c, rtol, max_iter, work, iters_out, relres_out,
                         stream);
}

extern "C" int vg_sign_update(double *theta_d, const double *grad_d, int64_t count, double lr, const double *scale_d,
                              const double *lo_d, const double *hi_d, void *stream) {
    if (count < 0 || !(lr >= 0) || !std::isfinite(lr) ||
        (count > 0 && (!theta_d || !grad_d || !scale_d || !lo_d || !hi_d))) {
        set_error("bad sign-update arguments");
        return VG_EINVAL;
    }
    if (count == 0) return VG_OK;
    hipLaunchKernelGGL(k_sign_update, dim3(blocks_for(count)), dim3(kBlock), 0, (hipStream_t)stream, theta_d, grad_d,
                       count, lr, scale_d, lo_d, hi_d);
    return launch_status("k_sign_update");
}
