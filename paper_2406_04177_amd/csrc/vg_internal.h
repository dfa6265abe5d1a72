// Internal declarations shared by the translation units of libvgsim.
// Device helpers (wave/block reductions, enumeration geometry, XCD-aware block
// mapping) and the host-side launch entry points of each kernel file.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "vgsim.h"

namespace vg {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, 32 CUs each

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int hip_status(hipError_t e, const char *what);   // VG_OK or VG_EHIP
int launch_status(const char *what);              // checks hipGetLastError

// ---------------------------------------------------------------- geometry
// Enumeration of voxel positions: raster (b == 0) or brick-major (b > 0).
struct Geom {
    int nx, ny, nz, b;
    int nbx, nby, nbz;
    int64_t npos;      // positions in the enumeration (bricks padded)
    int64_t nwords;    // 32-position words of the rank index
};

int make_geom(int nx, int ny, int nz, int brick, Geom *g);

__host__ __device__ inline int64_t geom_pos(const Geom &g, int x, int y, int z) {
    if (g.b <= 0) return x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
    const int b = g.b;
    const int bx = x / b, by = y / b, bz = z / b;
    const int lx = x - bx * b, ly = y - by * b, lz = z - bz * b;
    const int64_t blin = ((int64_t)bz * g.nby + by) * g.nbx + bx;
    return blin * (int64_t)(b * b * b) + (lz * b + ly) * b + lx;
}

__host__ __device__ inline void geom_xyz(const Geom &g, int64_t p, int &x, int &y, int &z) {
    if (g.b <= 0) {
        x = (int)(p % g.nx);
        const int64_t r = p / g.nx;
        y = (int)(r % g.ny);
        z = (int)(r / g.ny);
        return;
    }
    const int b = g.b;
    const int64_t b3 = (int64_t)b * b * b;
    const int64_t blin = p / b3;
    const int loc = (int)(p - blin * b3);
    const int bx = (int)(blin % g.nbx);
    const int64_t r = blin / g.nbx;
    const int by = (int)(r % g.nby);
    const int bz = (int)(r / g.nby);
    x = bx * b + loc % b;
    y = by * b + (loc / b) % b;
    z = bz * b + loc / (b * b);
}

// Rank index word: pore bitmap of 32 consecutive positions and the number of
// pore positions before the word.
struct RankWord {
    uint32_t bits;
    uint32_t before;
};

// ---------------------------------------------------------------- mapping
// Block index -> tile index such that each XCD (blocks are dealt round-robin
// to the 8 XCDs) works on one contiguous range of tiles, so the neighbour
// gathers of a tile hit the L2 that already holds its neighbours.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    const int64_t x = b % kNumXcd, k = b / kNumXcd;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums M doubles over the block in a fixed order; the result is valid in
// thread 0.  `lds` must hold kWaves * M doubles.
template <int M>
__device__ inline void block_sum(double (&v)[M], double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < M; m++) v[m] = wave_sum(v[m]);
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < M; m++) lds[wave * M + m] = v[m];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < M; m++) {
            double s = lds[m];
            for (int w = 1; w < kWaves; w++) s += lds[w * M + m];
            v[m] = s;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- kernels
// Coefficients of one step, rounded once to the field type R.
template <typename R>
struct Coef {
    R a[VG_NPOOL];       // D_s dt / h^2
    R v_dom, k_dom, rho, mu, beta, omb, v_som, v_p4, dt;   // omb = 1 - beta
    int route;           // 0 paper, 1 all mortality to pool 3
    R c[VG_NREG];        // region conductance factors
};

// Segment bookkeeping of the reduction tiles: tile t holds pieces
// [piece_first[t], piece_first[t+1]); piece p covers compact voxels
// [piece_lo[p], piece_lo[p+1]) of segment piece_seg[p].
struct Pieces {
    const int32_t *piece_first;
    const int64_t *piece_lo;
    const int32_t *piece_seg;
    int32_t npieces;
};

constexpr int kTile = kBlock;   // voxels per step-kernel tile (one per thread)


}  // namespace vg

// ---------------------------------------------------------------- handle
// Definition of the opaque handle declared in vgsim.h.
struct vg_sim {
    // graph
    int64_t n = 0;
    int nseg = 0;
    int prec = VG_F32;
    int mobile_all = 0;
    int features = 0;
    std::vector<int64_t> seg_off;
    const int32_t *nbr = nullptr;
    const uint16_t *rcode = nullptr;
    // model
    vg_params params{};
    double c[VG_NREG] = {1, 1, 1, 1, 1, 1, 1, 1};
    // bound buffers
    bool bound = false;
    char *fields = nullptr;
    char *alt = nullptr;
    char *work = nullptr;
    int cur = 0;                 // mobile pools live in fields (0) or alt (1)
    // reduction tiles and pieces (host copies and device views)
    int64_t ntiles = 0;
    int32_t npieces = 0;
    std::vector<int32_t> piece_first_h, piece_seg_h, seg_first_h;
    std::vector<int64_t> piece_lo_h;
    int32_t *piece_first = nullptr, *piece_seg = nullptr, *seg_first = nullptr;
    int64_t *piece_lo = nullptr;
    double *part = nullptr;      // [npieces][5]
    double *tot_tmp = nullptr;   // [nseg][6]
    // implicit CG (FP64 vectors)
    double *cg_y = nullptr, *cg_r = nullptr, *cg_z = nullptr, *cg_q = nullptr, *cg_m = nullptr;
    double *cg_p[2] = {nullptr, nullptr};
    double *cg_part = nullptr;   // [cg_blocks][4]
    double *cg_scal = nullptr;   // scalars (see vg_cg.hip)
    int cg_blocks = 0;
    // adjoint
    char *lam_alt = nullptr;     // [5][n] field type
    double *adj_part = nullptr;  // [adj_blocks][VG_NGRAD]
    int adj_blocks = 0;

    size_t elem() const { return prec == VG_F64 ? sizeof(double) : sizeof(float); }
    int mobile_mode() const { return mobile_all ? 2 : 1; }
};

namespace vg {

// launchers (vg_step.hip)
enum { MODE_T = 0, MODE_D = 1, MODE_DT = 2, MODE_NONE = 3 };
enum { TOT_NONE = 0, TOT_IN = 1, TOT_MID = 2, TOT_OUT = 3 };
int launch_pass(vg_sim *h, int mode, int tot, double dt, hipStream_t s);
int launch_pass_bufs(vg_sim *h, int mode, int tot, double dt, const void *const src[VG_NPOOL],
                     void *const dst[VG_NPOOL], hipStream_t s);
int launch_totals_finalize(vg_sim *h, double *out_rows, hipStream_t s);
int restore_canonical(vg_sim *h, hipStream_t s);
// vg_cg.hip
int run_cg(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
           hipStream_t s);
// vg_adjoint.hip
int launch_record(vg_sim *h, int64_t nsteps, double dt, void *states, hipStream_t s);
int launch_adjoint(vg_sim *h, int64_t nsteps, double dt, const void *states, const double *seeds,
                   void *lambda, double *grad, hipStream_t s);
int launch_seed(vg_sim *h, const double *seed, void *lambda, int zero, hipStream_t s);

template <typename R>
Coef<R> make_coef(const vg_sim *h, double dt) {
    Coef<R> c;
    const vg_params &p = h->params;
    for (int s = 0; s < VG_NPOOL; s++) c.a[s] = (R)(p.D[s] * dt / (p.h * p.h));
    c.v_dom = (R)p.v_dom; c.k_dom = (R)p.k_dom; c.rho = (R)p.rho; c.mu = (R)p.mu;
    c.beta = (R)p.beta; c.omb = (R)(1.0 - p.beta); c.v_som = (R)p.v_som; c.v_p4 = (R)p.v_p4;
    c.dt = (R)dt;
    c.route = p.mort_to_p4 ? 1 : 0;
    for (int r = 0; r < VG_NREG; r++) c.c[r] = (R)h->c[r];
    return c;
}

}  // namespace vg
