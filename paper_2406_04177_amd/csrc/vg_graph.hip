// Graph construction on the GPU (Sec. II.A, Fig. 2; Sec. III): pore voxels
// become graph nodes, face-adjacent pore voxels are joined.  Integer only and
// deterministic: the compact index of a pore voxel is its rank in the chosen
// enumeration (raster or brick-major), found with a pore bitmap plus per-word
// prefix counts ("rank index"), so no atomics or sorting are involved.
#include "vg_internal.h"

namespace vg {

int make_geom(int nx, int ny, int nz, int brick, Geom *g) {
    if (nx <= 0 || ny <= 0 || nz <= 0) {
        set_error("volume shape must be positive (got %d x %d x %d)", nx, ny, nz);
        return VG_EINVAL;
    }
    if ((int64_t)nx * ny * nz > INT32_MAX) {
        set_error("volume has more than 2^31-1 voxels");
        return VG_EINVAL;
    }
    if (brick < 0 || brick > 64) {
        set_error("brick size must be in [0, 64]");
        return VG_EINVAL;
    }
    g->nx = nx; g->ny = ny; g->nz = nz; g->b = brick;
    if (brick > 0) {
        g->nbx = (nx + brick - 1) / brick;
        g->nby = (ny + brick - 1) / brick;
        g->nbz = (nz + brick - 1) / brick;
        g->npos = (int64_t)g->nbx * g->nby * g->nbz * brick * brick * brick;
    } else {
        g->nbx = g->nby = g->nbz = 0;
        g->npos = (int64_t)nx * ny * nz;
    }
    if (g->npos > (int64_t)1 << 34) {
        set_error("padded brick enumeration too large");
        return VG_EINVAL;
    }
    g->nwords = (g->npos + 31) / 32;
    return VG_OK;
}

namespace {

constexpr int kScanItems = 8;                      // words per thread in the block scan
constexpr int kScanTile = kBlock * kScanItems;     // words per scan block

// One thread per enumeration position; a wave64 covers two 32-bit words.
__global__ __launch_bounds__(kBlock) void k_pack(const uint8_t *__restrict__ mask, Geom g,
                                                 RankWord *__restrict__ rank) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool pore = false;
    if (p < g.npos) {
        int x, y, z;
        geom_xyz(g, p, x, y, z);
        if (x < g.nx && y < g.ny && z < g.nz)
            pore = mask[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)] != 0;
    }
    const uint64_t ball = __ballot(pore);
    const int lane = threadIdx.x & 63;
    if ((lane & 31) == 0) {
        const int64_t w = p >> 5;
        if (w < g.nwords) {
            const uint32_t bits = (uint32_t)(ball >> lane);
            rank[w].bits = bits;
            rank[w].before = (uint32_t)__popc(bits);   // count; scanned below
        }
    }
}

// Exclusive scan of the per-word counts, pass 1: within tiles of kScanTile
// words; tile totals go to tsum.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(RankWord *__restrict__ rank, int64_t nwords,
                                                       uint32_t *__restrict__ tsum) {
    __shared__ uint32_t lds[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t c[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const int64_t w = base + k;
        c[k] = w < nwords ? rank[w].before : 0u;
        s += c[k];
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the thread sums
    for (int o = 1; o < kBlock; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0u;
        __syncthreads();
        lds[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = lds[threadIdx.x] - s;   // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const int64_t w = base + k;
        if (w < nwords) rank[w].before = run;
        run += c[k];
    }
    if (threadIdx.x == kBlock - 1) tsum[blockIdx.x] = lds[kBlock - 1];
}

// Pass 2: one block scans the tile totals (exclusive, in place); the grand
// total goes to tsum[ntiles].
__global__ __launch_bounds__(kBlock) void k_scan_totals(uint32_t *__restrict__ tsum, int64_t ntiles) {
    __shared__ uint32_t lds[kBlock];
    const int64_t per = (ntiles + kBlock - 1) / kBlock;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < ntiles ? lo + per : ntiles;
    uint32_t s = 0;
    for (int64_t t = lo; t < hi; t++) s += tsum[t];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0u;
        __syncthreads();
        lds[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = lds[threadIdx.x] - s;
    for (int64_t t = lo; t < hi; t++) {
        const uint32_t c = tsum[t];
        tsum[t] = run;
        run += c;
    }
    if (threadIdx.x == kBlock - 1) tsum[ntiles] = lds[kBlock - 1];
}

// Pass 3: add the tile offsets.
__global__ __launch_bounds__(kBlock) void k_scan_add(RankWord *__restrict__ rank, int64_t nwords,
                                                     const uint32_t *__restrict__ tsum) {
    const int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (w < nwords) rank[w].before += tsum[w / kScanTile];
}

// Compact index of enumeration position p, or -1 if it is not a pore voxel.
__device__ inline int32_t rank_of(const RankWord *__restrict__ rank, int64_t p) {
    const RankWord wd = rank[p >> 5];
    const uint32_t bit = (uint32_t)(p & 31);
    if (!((wd.bits >> bit) & 1u)) return -1;
    return (int32_t)(wd.before + (uint32_t)__popc(wd.bits & ((1u << bit) - 1u)));
}

__global__ __launch_bounds__(kBlock) void k_build(const RankWord *__restrict__ rank, Geom g,
                                                  unsigned periodic, int32_t base, int64_t ld,
                                                  int32_t *__restrict__ vox, int32_t *__restrict__ nbr) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= g.npos) return;
    const int32_t i = rank_of(rank, p);
    if (i < 0) return;
    int x, y, z;
    geom_xyz(g, p, x, y, z);
    vox[i] = x + g.nx * (y + g.ny * z);
    const int dims[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int k = 0; k < 6; k++) {
        int q[3] = {x, y, z};
        const int axis = k >> 1;
        q[axis] += (k & 1) ? 1 : -1;
        bool inside = true;
        if (q[axis] < 0 || q[axis] >= dims[axis]) {
            if (periodic & (1u << axis)) q[axis] = (q[axis] + dims[axis]) % dims[axis];
            else inside = false;
        }
        int32_t j = -1;
        if (inside) {
            const int32_t r = rank_of(rank, geom_pos(g, q[0], q[1], q[2]));
            if (r >= 0) j = base + r;
        }
        nbr[(int64_t)k * ld + i] = j;
    }
}

__global__ __launch_bounds__(kBlock) void k_lookup(const RankWord *__restrict__ rank, Geom g,
                                                   const int64_t *__restrict__ lin, int64_t count,
                                                   int32_t base, int32_t *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= count) return;
    const int64_t v = lin[q];
    int32_t r = -1;
    if (v >= 0 && v < (int64_t)g.nx * g.ny * g.nz) {
        const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
        r = rank_of(rank, geom_pos(g, x, y, z));
    }
    out[q] = r >= 0 ? base + r : -1;
}

__device__ inline int octant(int x, int y, int z, int nx, int ny, int nz) {
    return 4 * (z >= nz / 2) + 2 * (y >= ny / 2) + (x >= nx / 2);
}

__global__ __launch_bounds__(kBlock) void k_region_codes(const int32_t *__restrict__ vox, int64_t n,
                                                         int nx, int ny, int nz, unsigned periodic,
                                                         uint16_t *__restrict__ codes) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int v = vox[i];
    const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
    const int own = octant(x, y, z, nx, ny, nz);
    const int dims[3] = {nx, ny, nz};
    uint32_t code = (uint32_t)own;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        int q[3] = {x, y, z};
        const int axis = k >> 1;
        q[axis] += (k & 1) ? 1 : -1;
        if (q[axis] < 0 || q[axis] >= dims[axis]) {
            if (!(periodic & (1u << axis))) continue;
            q[axis] = (q[axis] + dims[axis]) % dims[axis];
        }
        if (octant(q[0], q[1], q[2], nx, ny, nz) != own) code |= 1u << (3 + k);
    }
    codes[i] = (uint16_t)code;
}

inline unsigned grid_for(int64_t work) { return (unsigned)((work + kBlock - 1) / kBlock); }

}  // namespace
}  // namespace vg

using namespace vg;

extern "C" int vg_rank_bytes(int nx, int ny, int nz, int brick, size_t *bytes) {
    if (!bytes) { set_error("bytes is NULL"); return VG_EINVAL; }
    Geom g;
    int rc = make_geom(nx, ny, nz, brick, &g);
    if (rc) return rc;
    const int64_t ntiles = (g.nwords + kScanTile - 1) / kScanTile;
    *bytes = (size_t)g.nwords * sizeof(RankWord) + (size_t)(ntiles + 1) * sizeof(uint32_t) + 64;
    return VG_OK;
}

extern "C" int vg_count_pores(const uint8_t *mask_d, int nx, int ny, int nz, int brick, void *rank_d,
                              int64_t *n_out, void *stream) {
    if (!mask_d || !rank_d || !n_out) { set_error("null pointer argument"); return VG_EINVAL; }
    Geom g;
    int rc = make_geom(nx, ny, nz, brick, &g);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    RankWord *rank = (RankWord *)rank_d;
    const int64_t ntiles = (g.nwords + kScanTile - 1) / kScanTile;
    uint32_t *tsum = (uint32_t *)(rank + g.nwords);
    // words beyond npos (the last partial word) are written by k_pack as well
    hipLaunchKernelGGL(k_pack, dim3(grid_for(g.nwords * 32)), dim3(kBlock), 0, s, mask_d, g, rank);
    if ((rc = launch_status("k_pack"))) return rc;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kBlock), 0, s, rank, g.nwords, tsum);
    if ((rc = launch_status("k_scan_tiles"))) return rc;
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kBlock), 0, s, tsum, ntiles);
    if ((rc = launch_status("k_scan_totals"))) return rc;
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(g.nwords)), dim3(kBlock), 0, s, rank, g.nwords, tsum);
    if ((rc = launch_status("k_scan_add"))) return rc;
    uint32_t total = 0;
    if ((rc = hip_status(hipMemcpyAsync(&total, tsum + ntiles, sizeof(total), hipMemcpyDeviceToHost, s),
                         "copy pore count"))) return rc;
    if ((rc = hip_status(hipStreamSynchronize(s), "synchronise"))) return rc;
    *n_out = (int64_t)total;
    return VG_OK;
}

extern "C" int vg_build_graph(const void *rank_d, int nx, int ny, int nz, int brick, unsigned periodic,
                              int32_t index_base, int64_t n, int64_t ld, int32_t *vox_d, int32_t *nbr_d,
                              void *stream) {
    if (!rank_d || (n > 0 && (!vox_d || !nbr_d))) { set_error("null pointer argument"); return VG_EINVAL; }
    if (n < 0 || ld < n || index_base < 0 || (int64_t)index_base + n > INT32_MAX || periodic > 7u) {
        set_error("bad n / ld / index_base / periodic");
        return VG_EINVAL;
    }
    Geom g;
    int rc = make_geom(nx, ny, nz, brick, &g);
    if (rc) return rc;
    if (n == 0) return VG_OK;
    hipLaunchKernelGGL(k_build, dim3(grid_for(g.npos)), dim3(kBlock), 0, (hipStream_t)stream,
                       (const RankWord *)rank_d, g, periodic, index_base, ld, vox_d, nbr_d);
    return launch_status("k_build");
}

extern "C" int vg_lookup(const void *rank_d, int nx, int ny, int nz, int brick, const int64_t *lin_d,
                         int64_t count, int32_t index_base, int32_t *idx_d, void *stream) {
    if (count < 0 || (count > 0 && (!rank_d || !lin_d || !idx_d))) {
        set_error("bad lookup arguments");
        return VG_EINVAL;
    }
    Geom g;
    int rc = make_geom(nx, ny, nz, brick, &g);
    if (rc) return rc;
    if (count == 0) return VG_OK;
    hipLaunchKernelGGL(k_lookup, dim3(grid_for(count)), dim3(kBlock), 0, (hipStream_t)stream,
                       (const RankWord *)rank_d, g, lin_d, count, index_base, idx_d);
    return launch_status("k_lookup");
}

extern "C" int vg_region_codes(const int32_t *vox_d, int64_t n, int nx, int ny, int nz, unsigned periodic,
                               uint16_t *codes_d, void *stream) {
    if (n < 0 || (n > 0 && (!vox_d || !codes_d)) || periodic > 7u) {
        set_error("bad region-code arguments");
        return VG_EINVAL;
    }
    Geom g;
    int rc = make_geom(nx, ny, nz, 0, &g);
    if (rc) return rc;
    if (n == 0) return VG_OK;
    hipLaunchKernelGGL(k_region_codes, dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, vox_d, n,
                       nx, ny, nz, periodic, codes_d);
    return launch_status("k_region_codes");
}
