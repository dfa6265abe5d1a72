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
// Block index -> tile index.  Blocks are dealt round-robin to the 8 XCDs,
// each with its own L2; runs of kXcdRun consecutive tiles go to the XCDs in
// turn and each XCD works through its run in order, so the +-x / +-y
// neighbours of a tile mostly sit in its own L2 while the whole chip still
// sweeps memory in one front; the tiles after the last full round of runs
// are split into one contiguous share per XCD.  (Measured on the 512^3 step:
// ~1 % faster than the identity map; one contiguous eighth per XCD ~5 %
// slower.)
constexpr int64_t kXcdRun = 64;
__device__ inline int64_t xcd_split(int64_t b, int64_t nb) {
    const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    const int64_t x = b % kNumXcd, k = b / kNumXcd;
    return x * q + (x < r ? x : r) + k;
}
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
    constexpr int64_t S = kXcdRun, R = S * kNumXcd;
    const int64_t full = nb / R * R;
    if (b >= full) return full + xcd_split(b - full, nb - full);
    const int64_t x = b % kNumXcd, k = b / kNumXcd;
    return ((k / S) * kNumXcd + x) * S + k % S;
}

// Tile of iteration `it` of block b in a grid-stride kernel of nb blocks.
// With nb a multiple of 8 the blocks of one XCD (b % 8) walk that XCD's own
// runs of kXcdRun consecutive tiles (the runs xcd_tile deals to it), then
// its contiguous share of the tiles after the last full round of runs, so a
// grid-stride kernel keeps the locality of the one-tile-per-block kernels;
// otherwise plain striding.  Returns ntiles once the block's list is done.
__device__ inline int64_t xcd_stride_tile(int64_t b, int64_t nb, int64_t it, int64_t ntiles) {
    if (nb % kNumXcd != 0) {
        const int64_t t = b + it * nb;
        return t < ntiles ? t : ntiles;
    }
    constexpr int64_t S = kXcdRun, R = S * kNumXcd;
    const int64_t x = b % kNumXcd, m = it * (nb / kNumXcd) + b / kNumXcd;
    const int64_t nfull = ntiles / R * R, own_full = nfull / kNumXcd;
    if (m < own_full) return ((m / S) * kNumXcd + x) * S + m % S;
    const int64_t u = m - own_full, tail = ntiles - nfull;
    const int64_t q = tail / kNumXcd, r = tail % kNumXcd;
    if (u >= q + (x < r ? 1 : 0)) return ntiles;
    return nfull + x * q + (x < r ? x : r) + u;
}

// Blocks of kBlock threads of `kernel` that fit on the device at once (so a
// grid-stride launch has no second, partial round), rounded down to a
// multiple of the XCD count, at most cap (cached per kernel and device).
int resident_blocks(const void *kernel, int cap);

// Barrier that orders the block's LDS accesses only: global loads issued
// before it may still be in flight after it (a full __syncthreads waits for
// them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- reductions
// A double moved across lanes by a DPP control (the two 32-bit halves in
// turn).  Only controls whose source lane lies in the same 16-lane row are
// used, so every lane has a source.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave, the same value in every lane, in a fixed
// order: within each 16-lane row pairs (lane ^ 1), then pairs of pairs
// (lane ^ 2), then the row's quads by rotations of 4 and 8 lanes (DPP: no
// LDS traffic), then the four row sums read from lanes 0, 16, 32, 48 and
// added as (r0 + r1) + (r2 + r3).
__device__ inline double wave_sum(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x124>(v);   // row_ror:4
    v += dpp_move<0x128>(v);   // row_ror:8
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Per-tile sums of M doubles written straight to out[0..M-1] in a fixed
// order: each 16-lane row is reduced by DPP (the first four steps of
// wave_sum), one lane per row stores the row sums in LDS, and thread m < M
// adds the block's kRows row sums of value m pairwise.  `lds` must hold
// kRows * M doubles; it may be reused after the call.
constexpr int kRows = kWaves * 4;

template <int M>
__device__ inline void tile_sum_to(double (&v)[M], double *lds, double *__restrict__ out) {
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 4;
#pragma unroll
    for (int m = 0; m < M; m++) {
        double x = v[m];
        x += dpp_move<0xB1>(x);
        x += dpp_move<0x4E>(x);
        x += dpp_move<0x124>(x);
        x += dpp_move<0x128>(x);
        v[m] = x;
    }
    if ((lane & 15) == 0) {
#pragma unroll
        for (int m = 0; m < M; m++) lds[row * M + m] = v[m];
    }
    __syncthreads();
    if (threadIdx.x < M) {
        const int m = threadIdx.x;
        double r[kRows];
#pragma unroll
        for (int k = 0; k < kRows; k++) r[k] = lds[k * M + m];
#pragma unroll
        for (int w = 1; w < kRows; w <<= 1)
#pragma unroll
            for (int k = 0; k + w < kRows; k += 2 * w) r[k] += r[k + w];
        out[m] = r[0];
    }
    __syncthreads();
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

// ---------------------------------------------------------------- storage
// Compensated float32 (VG_F32C): a value x is stored as hi = the float nearest
// to x and lo = (x - hi) / ulp(hi) * 2^15 rounded to an int16.  |x - hi| is at
// most half an ulp of hi, so |lo| <= 2^14, and x - hi is exact in FP64
// (Sterbenz), as is the scaling by a power of two: the only rounding is lo's,
// at most ulp(hi) * 2^-16, i.e. 2^-39 relative.  ulp(hi) = 2^(e - 150) for the
// biased exponent e of hi, with e taken as 1 for zero and subnormal hi (their
// ulp is 2^-149), so ulp(hi) * 2^-15 = 2^(e - 165), a normal double.
__device__ __forceinline__ double comp_get(float hi, int16_t lo) {
    uint32_t e = (__float_as_uint(hi) >> 23) & 0xffu;
    e = e < 1u ? 1u : e;
    const double scale = __longlong_as_double((long long)((uint64_t)(e + 858u) << 52));   // 2^(e - 165)
    return (double)hi + (double)lo * scale;
}

__device__ __forceinline__ void comp_put(double x, float &hi, int16_t &lo) {
    const float h = (float)x;
    uint32_t e = (__float_as_uint(h) >> 23) & 0xffu;
    e = e < 1u ? 1u : e;
    const double inv = __longlong_as_double((long long)((uint64_t)(1188u - e) << 52));    // 2^(165 - e)
    hi = h;
    lo = (int16_t)__double2int_rn((x - (double)h) * inv);
}

// One pool's storage as the kernels that work in FP64 see it (the implicit
// solve, state conversions): plain R, or compensated float32.
template <typename R>
struct PlainAcc {
    R *p;
    __device__ __forceinline__ double get(int64_t i) const { return (double)p[i]; }
    __device__ __forceinline__ void put(int64_t i, double v) const { p[i] = (R)v; }
};
struct CompAcc {
    float *hi;
    int16_t *lo;
    __device__ __forceinline__ double get(int64_t i) const { return comp_get(hi[i], lo[i]); }
    __device__ __forceinline__ void put(int64_t i, double v) const {
        float h;
        int16_t l;
        comp_put(v, h, l);
        hi[i] = h;
        lo[i] = l;
    }
};

// ---------------------------------------------------------------- kernels
// Coefficients of one step, rounded once to the field type R.
template <typename R>
struct Coef {
    R a[VG_NPOOL];       // D_s dt / h^2
    R v_dom, k_dom, rho, mu, beta, omb, v_som, v_p4, dt;   // omb = 1 - beta
    int route;           // 0 paper, 1 all mortality to pool 3
    int seq;             // 0 Algorithm 1, 1 Algorithm 2
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

constexpr int kVPT = 1;                 // voxels per thread in a tile
constexpr int kTile = kBlock * kVPT;    // voxels per tile (one tile per block)
constexpr int kChunk = 256;             // pieces per first-stage totals chunk

// Division by a run-time invariant 32-bit divisor with one multiply-high
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Fig. 4.1).  Exact for every n < 2^32.
struct FastDiv {
    uint32_t d = 1, m = 1, s1 = 0, s2 = 0;
    __host__ void init(uint32_t div) {
        d = div;
        uint32_t l = 0;
        while (l < 32 && (1ull << l) < div) l++;
        m = (uint32_t)((((1ull << 32) * ((1ull << l) - div)) / div) + 1);
        s1 = l < 1 ? l : 1;
        s2 = l > 1 ? l - 1 : 0;
    }
    __device__ __forceinline__ uint32_t div(uint32_t n) const {
        const uint32_t t1 = __umulhi(m, n);
        return (t1 + ((n - t1) >> s1)) >> s2;
    }
};

// Geometry of the enumeration with fast divisions, for the kernels that find
// neighbours through the rank index instead of the neighbour table.
struct RGeom {
    Geom g;
    FastDiv fnx, fny, fb, fb2, fb3, fnbx, fnby;
    unsigned periodic;
    const RankWord *rank;
};

__device__ __forceinline__ void rg_xyz(const RGeom &G, uint32_t p, int &x, int &y, int &z) {
    if (G.g.b <= 0) {
        const uint32_t q1 = G.fnx.div(p);
        x = (int)(p - q1 * G.fnx.d);
        const uint32_t q2 = G.fny.div(q1);
        y = (int)(q1 - q2 * G.fny.d);
        z = (int)q2;
        return;
    }
    const uint32_t blin = G.fb3.div(p);
    const uint32_t loc = p - blin * G.fb3.d;
    const uint32_t r1 = G.fnbx.div(blin);
    const int bx = (int)(blin - r1 * G.fnbx.d);
    const uint32_t r2 = G.fnby.div(r1);
    const int by = (int)(r1 - r2 * G.fnby.d);
    const int bz = (int)r2;
    const uint32_t lz = G.fb2.div(loc);
    const uint32_t rem = loc - lz * G.fb2.d;
    const uint32_t ly = G.fb.div(rem);
    const uint32_t lx = rem - ly * G.fb.d;
    const int b = G.g.b;
    x = bx * b + (int)lx;
    y = by * b + (int)ly;
    z = bz * b + (int)lz;
}

__device__ __forceinline__ uint32_t rg_pos(const RGeom &G, int x, int y, int z) {
    if (G.g.b <= 0) return (uint32_t)x + G.fnx.d * ((uint32_t)y + G.fny.d * (uint32_t)z);
    const uint32_t b = (uint32_t)G.g.b;
    const uint32_t bx = G.fb.div((uint32_t)x), by = G.fb.div((uint32_t)y), bz = G.fb.div((uint32_t)z);
    const uint32_t lx = (uint32_t)x - bx * b, ly = (uint32_t)y - by * b, lz = (uint32_t)z - bz * b;
    const uint32_t blin = (bz * (uint32_t)G.g.nby + by) * (uint32_t)G.g.nbx + bx;
    return blin * G.fb3.d + (lz * b + ly) * b + lx;
}

__device__ __forceinline__ int32_t rank_lookup(const RankWord &wd, uint32_t p) {
    const uint32_t bit = p & 31u;
    if (!((wd.bits >> bit) & 1u)) return -1;
    return (int32_t)(wd.before + (uint32_t)__popc(wd.bits & ((1u << bit) - 1u)));
}


// Packed neighbour offsets: two 32-bit words per voxel, one for the minus-side
// neighbours (compact index i - d) and one for the plus side (i + d).  In
// both, the z offset occupies bits [0, bz), y the next by bits and x the next
// bx bits; an offset of 0 means the neighbour is absent.  Valid when every
// minus-side neighbour precedes the voxel in the enumeration and every
// plus-side one follows it (no periodic wrap) and the widths fit 32 bits.
struct DLayout {
    uint32_t bz = 0, by = 0, sx = 0;   // shifts of the y and x fields
    uint32_t mz = 0, my = 0, mx = 0;   // field masks
};

// Relative neighbour codes: one 32-bit word per voxel with a code per slot
// k (0..5 = -x, +x, -y, +y, -z, +z) in bits [sh[k], sh[k] + width), and per
// group of kGroup consecutive voxels one base distance per slot (8 words,
// the last two unused).  Code 0 = absent, code c >= 1 = distance base + c - 1
// (minus side: neighbour i - distance, plus side: i + distance).  The bases
// are the smallest distances in the group, so the codes only have to span the
// spread of the distances within 64 voxels (a few dozen in raster order).
constexpr int kGroup = 64;
struct RLayout {
    uint32_t sh[6] = {0, 0, 0, 0, 0, 0};
    uint32_t mk[6] = {0, 0, 0, 0, 0, 0};
};

__device__ __forceinline__ void unpack_offsets(const DLayout &L, uint32_t w, uint32_t (&d)[3]) {
    d[0] = (w >> L.sx) & L.mx;
    d[1] = (w >> L.bz) & L.my;
    d[2] = w & L.mz;
}

// Element idx of an array whose base is uniform across the wave: a 32-bit
// byte offset from the base, so that the whole address arithmetic of a voxel
// is one shift (valid while n * sizeof(T) < 2^32, which the host checks
// before it enables a packed neighbour source).
template <typename T>
__device__ __forceinline__ const T &at(const T *base, uint32_t idx) {
    return *(const T *)((const char *)base + (idx * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T &at(T *base, uint32_t idx) {
    return *(T *)((char *)base + (idx * (uint32_t)sizeof(T)));
}

// The two packed neighbour sources as the kernels see them.
struct PackedNbr {
    const uint32_t *rel_w = nullptr;     // [n] relative codes
    const uint32_t *rel_base = nullptr;  // [groups][8] base distances
    RLayout rl;
    const uint32_t *off_m = nullptr;     // [n] packed offsets, minus side
    const uint32_t *off_p = nullptr;     // [n] packed offsets, plus side
    DLayout dl;
};

// Compact indices of the six neighbours of voxel i from a packed source
// (RELC: relative codes, else packed offsets), in two steps so that the
// caller can issue its other loads between them: packed_words loads the
// voxel's words, packed_decode turns them into indices.  An absent neighbour
// gives i itself, so that every difference x_j - x_i of an absent slot is
// exactly +0 for finite values and the slot needs no select.  With relative
// codes all active lanes of the wave must hold voxels of the same group.
struct PackedWords {
    uint32_t a, b;
};

template <bool RELC>
__device__ __forceinline__ PackedWords packed_words(const PackedNbr &P, uint32_t i) {
    PackedWords W;
    if (RELC) {
        W.a = at(P.rel_w, i);
        W.b = 0;
    } else {
        W.a = at(P.off_m, i);
        W.b = at(P.off_p, i);
    }
    return W;
}

template <bool RELC>
__device__ __forceinline__ void packed_decode(const PackedNbr &P, uint32_t i, PackedWords W, uint32_t (&j)[6]) {
    if (RELC) {
        // the six base distances of the group: one uniform 32-byte load
        const uint32_t grp = __builtin_amdgcn_readfirstlane(i / (uint32_t)kGroup);
        const uint32_t *bp = P.rel_base + (size_t)grp * 8;
        uint32_t base[6];
#pragma unroll
        for (int k = 0; k < 6; k++) base[k] = bp[k];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const uint32_t c = (W.a >> P.rl.sh[k]) & P.rl.mk[k];
            const uint32_t d = c ? base[k] + (c - 1u) : 0u;
            j[k] = (k & 1) ? i + d : i - d;
        }
    } else {
        uint32_t dm[3], dp[3];
        unpack_offsets(P.dl, W.a, dm);
        unpack_offsets(P.dl, W.b, dp);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            j[2 * a] = i - dm[a];
            j[2 * a + 1] = i + dp[a];
        }
    }
}

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
    int16_t *lo = nullptr;       // VG_F32C: [5][n] compensation words of the fields
    int16_t *lo_alt = nullptr;   // VG_F32C: compensation words of alt
    // reduction tiles and pieces (host copies and device views)
    int64_t ntiles = 0;
    int32_t npieces = 0;
    int32_t nchunks = 0;
    int32_t max_seg_pieces = 0;  // most pieces in one segment (one-stage totals up to 4096)
    std::vector<int32_t> chunk_first_h, seg_chunk_h;
    int32_t *chunk_first = nullptr, *seg_chunk = nullptr;
    double *chunk_part = nullptr;   // [tot_batch][nchunks][5]
    // rank-index neighbours (single volume)
    const void *rank = nullptr;
    int nx = 0, ny = 0, nz = 0, brick = 0;
    unsigned periodic = 0;
    const int32_t *vox = nullptr;   // compacted list (linear indices)
    uint32_t *geo = nullptr;        // [n] geometry words of the rank-index kernel
    int kernel = 0;                 // VG_KERNEL_*
    // packed neighbour offsets (any volume or batch without periodic wrap)
    uint32_t *off_m = nullptr, *off_p = nullptr;   // [n] each
    uint32_t *off_stat = nullptr;                  // [8] max offset per axis, violation flag, code spans
    bool off_ok = false;
    vg::DLayout off_layout;
    // relative neighbour codes (4 B per voxel plus 32 B per 64 voxels)
    uint32_t *rel_w = nullptr;      // [n]
    uint32_t *rel_base = nullptr;   // [ceil(n / 64)][8]
    bool rel_ok = false;
    vg::RLayout rel_layout;
    // two-pass band kernel (single raster volume; see vg_step.hip)
    int32_t *band_rs = nullptr;     // [nz * ny + 1] compact index of the first voxel of each row
    char *band_alt = nullptr;       // [5][n] field type: the pass pair's intermediate fields
    bool band_ok = false;           // built and fits the LDS
    bool band_auto = false;         // chunks long enough for AUTO to take it
    int band_h = 0, band_z = 0, band_nbands = 0, band_nchunks = 0, band_cap = 0;
    std::vector<int32_t> piece_first_h, piece_seg_h, seg_first_h;
    std::vector<int64_t> piece_lo_h;
    int32_t *piece_first = nullptr, *piece_seg = nullptr, *seg_first = nullptr;
    int64_t *piece_lo = nullptr;
    double *part = nullptr;      // [tot_batch][npieces][5]: partials of up to tot_batch logged passes
    int tot_batch = 1;           // logged passes whose totals are reduced by one launch
    int part_slot = 0;           // the slot the next pass with totals writes
    double *tot_tmp = nullptr;   // [nseg][6]
    // implicit CG (FP64 vectors)
    double *cg_y = nullptr, *cg_r = nullptr, *cg_z = nullptr, *cg_q = nullptr, *cg_m = nullptr;
    double *cg_p[2] = {nullptr, nullptr};
    double *cg_part = nullptr;   // [cg_blocks][4]
    double *cg_scal = nullptr;   // scalars (see vg_cg.hip)
    int cg_blocks = 0;
    // multigrid preconditioner of the CG (VG_FEAT_MG; vg_cg.hip).  Level 0 is
    // the pore voxels (the CG's own vectors); levels >= 1 are aggregates.
    struct MgLevel {
        int64_t n = 0, cap = 0;          // cells; capacity reserved in the workspace
        int nx = 0, ny = 0, nz = 0;      // grid of the level
        int32_t *vox = nullptr;          // [cap] linear index of each cell in its grid (levels >= 1)
        int32_t *nbr = nullptr;          // [6][cap] neighbour cells, -1 if absent (levels >= 1)
        float *w = nullptr;              // [6][cap] edge weights, 0 if absent (levels >= 1)
        float *mass = nullptr;           // [cap] voxels in the cell (levels >= 1)
        double *invd = nullptr, *r = nullptr, *x = nullptr, *e = nullptr;   // [cap] (levels >= 1)
        int32_t *parent = nullptr;       // [cap] cell of the next level (all but the coarsest)
        vg::RankWord *rank = nullptr;    // rank index of the grid (levels >= 1; level 0 uses the handle's)
    };
    MgLevel mg[VG_MG_MAX_LEVELS];
    int mg_levels = 0;                   // levels built (0: none)
    int mg_plan_levels = 0;              // levels the workspace reserves
    bool mg_wdone = false;               // coarse weights follow the current region factors
    uint8_t *mg_mask = nullptr;          // set-up scratch: occupancy of the next coarser grid
    int precond = VG_PRECOND_JACOBI;
    // adjoint
    unsigned adj_flags = 0;      // VG_ADJ_* options
    char *lam_alt = nullptr;     // [5][n] field type
    double *adj_part = nullptr;  // [adj_blocks][VG_NGRAD]
    char *adj_co2 = nullptr;     // [2][nseg] field type: the CO2 adjoint of each volume (uniform case)
    int32_t *adj_flag = nullptr; // [nseg] nonzero: the CO2 adjoint of the volume is not uniform
    int adj_blocks = 0;

    // replayed runs of fused passes (HIP graphs; see vg_step_explicit)
    unsigned launch_flags = 0;      // VG_LAUNCH_*
    hipStream_t capture_stream = nullptr;   // private stream the runs are captured on
    uint64_t graph_version = 0;     // bumped by every change a captured run depends on
    struct RunGraph {
        hipGraphExec_t exec = nullptr;
        int cur = 0, passes = 0, band = 0;
        double dt = 0;
        uint64_t version = 0;
    };
    RunGraph run_graph[2];          // one per parity of the mobile pools' ping-pong

    size_t elem() const { return prec == VG_F64 ? sizeof(double) : sizeof(float); }   // float for VG_F32C
    int mobile_mode() const { return mobile_all ? 2 : 1; }
};

namespace vg {

// launchers (vg_step.hip)
enum { MODE_T = 0, MODE_D = 1, MODE_DT = 2, MODE_NONE = 3 };
enum { TOT_NONE = 0, TOT_IN = 1, TOT_MID = 2, TOT_OUT = 3 };
int launch_pass(vg_sim *h, int mode, int tot, double dt, hipStream_t s);
int launch_pass2(vg_sim *h, int mode, int tot, double dt_t, double dt_d, hipStream_t s);
int launch_pass_bufs(vg_sim *h, int mode, int tot, double dt, const void *const src[VG_NPOOL],
                     void *const dst[VG_NPOOL], hipStream_t s, void *xdom = nullptr);
// Reduces the partials of slots 0 .. rows-1 into rows consecutive totals
// rows out_rows[r][nseg][6].
int launch_totals_finalize(vg_sim *h, double *out_rows, int rows, hipStream_t s);
// The partials the next pass with totals writes (slot part_slot).
inline double *part_of(const vg_sim *h) { return h->part + (size_t)h->part_slot * VG_NPOOL * (size_t)h->npieces; }
int launch_geometry(vg_sim *h, hipStream_t s);
bool use_rank(const vg_sim *h);
bool use_offsets(const vg_sim *h);
bool use_relative(const vg_sim *h);
bool band_geometry(const vg_sim *h);   // the graph and features allow the band kernel
bool use_band(const vg_sim *h);        // the next pass pairs run on the band kernel
bool tape_keeps_dom(const vg_sim *h);  // recordings keep each state's diffused DOM (VG_ADJ_TAPE_DOM)
int tape_rows(const vg_sim *h);        // rows per recorded state: 4 with the kept DOM, else 5
// The source pools of a recording pass from recorded state j, the
// destination pools of state j + 1, and where state j's diffused DOM goes
// (null without the kept DOM or for j = 0).
void tape_pass_bufs(const vg_sim *h, void *states, int64_t j, const void *src[VG_NPOOL], void *dst[VG_NPOOL],
                    void **xdom);
int build_band(vg_sim *h, hipStream_t s);
int launch_band_quad(vg_sim *h, double dt, hipStream_t s);
PackedNbr packed_of(const vg_sim *h);
int build_offsets(vg_sim *h, hipStream_t s);
int restore_canonical(vg_sim *h, hipStream_t s);
// vg_cg.hip
int run_cg(vg_sim *h, int pool, double a, double rtol, int max_iter, int *iters, double *relres,
           hipStream_t s);
// grids and capacities of the multigrid levels the workspace reserves
// (fills h->mg[*].nx/ny/nz/cap and h->mg_plan_levels)
void mg_plan(vg_sim *h);
int mg_build(vg_sim *h, hipStream_t s);    // the hierarchy (structure and weights), at vg_init_state
int mg_apply(vg_sim *h, double a, const double *r, double *z, hipStream_t s);   // vg_precondition
// vg_adjoint.hip
int launch_record(vg_sim *h, int64_t nsteps, double dt, void *states, hipStream_t s);
int launch_adjoint(vg_sim *h, int64_t nsteps, double dt, const void *states, const double *seeds,
                   void *lambda, double *grad, hipStream_t s);
int launch_seed(vg_sim *h, const double *seed, void *lambda, int zero, hipStream_t s);
int launch_load_state(vg_sim *h, const void *x, int xprec, hipStream_t s);
int launch_store_state(vg_sim *h, void *x, int xprec, hipStream_t s);

// Coefficients of a pass whose transformation step is dt_t and whose
// diffusion step is dt_d (equal except in sub-cycled runs).
template <typename R>
Coef<R> make_coef2(const vg_sim *h, double dt_t, double dt_d) {
    Coef<R> c;
    const vg_params &p = h->params;
    for (int s = 0; s < VG_NPOOL; s++) c.a[s] = (R)(p.D[s] * dt_d / (p.h * p.h));
    c.v_dom = (R)p.v_dom; c.k_dom = (R)p.k_dom; c.rho = (R)p.rho; c.mu = (R)p.mu;
    c.beta = (R)p.beta; c.omb = (R)(1.0 - p.beta); c.v_som = (R)p.v_som; c.v_p4 = (R)p.v_p4;
    c.dt = (R)dt_t;
    c.route = p.mort_to_p4 ? 1 : 0;
    c.seq = p.sequential ? 1 : 0;
    for (int r = 0; r < VG_NREG; r++) c.c[r] = (R)h->c[r];
    return c;
}

template <typename R>
Coef<R> make_coef(const vg_sim *h, double dt) {
    Coef<R> c;
    const vg_params &p = h->params;
    for (int s = 0; s < VG_NPOOL; s++) c.a[s] = (R)(p.D[s] * dt / (p.h * p.h));
    c.v_dom = (R)p.v_dom; c.k_dom = (R)p.k_dom; c.rho = (R)p.rho; c.mu = (R)p.mu;
    c.beta = (R)p.beta; c.omb = (R)(1.0 - p.beta); c.v_som = (R)p.v_som; c.v_p4 = (R)p.v_p4;
    c.dt = (R)dt;
    c.route = p.mort_to_p4 ? 1 : 0;
    c.seq = p.sequential ? 1 : 0;
    for (int r = 0; r < VG_NREG; r++) c.c[r] = (R)h->c[r];
    return c;
}

}  // namespace vg
