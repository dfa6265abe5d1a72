// Explicit time stepping: the per-voxel transformation (Sec. II.C eq. (3) with
// the clamps of Appendix A, Algorithm 1) and explicit diffusion on the voxel
// graph (Sec. II.B.3a, Scheme 1), fused into one bandwidth-bound pass over
// the compacted pore list, plus the FP64 mass totals.
//
// One pass reads each pool of a voxel once, gathers the mobile pools of its
// six neighbours (mostly cache hits: +-x are adjacent entries, +-y and +-z lie
// one row / one plane away in the enumeration), and writes each pool once.
// Immobile pools are updated in place; mobile pools ping-pong between the
// caller's field buffer and its alt buffer because neighbours read them.
//
// Two ways to find the neighbours of compact voxel i:
//   table  the 6-slot int32 table nbr[6][n] (24 B per voxel and pass);
//   rank   the rank index of the enumeration: a block decodes the positions of
//          its tile of compact voxels from the pore bitmap words into LDS, and
//          each neighbour's compact index is the rank of its position
//          (bitmap word + popcount).  The words of a tile are ~1.5 B per voxel
//          and the neighbour words are cache hits, so a pass moves ~41 B per
//          voxel instead of 64 B.  Single volume only.
//
// The paper's step is T then D.  The pass computes K = T o D (diffuse, then
// transform), so n paper steps run as T, K^(n-1), D.  Inside a K pass the
// state between its D and T halves is exactly the paper state after a full
// step, which is where the totals of that step are taken.
#include "vg_internal.h"

#pragma clang fp contract(off)

namespace vg {
namespace {

// Transformation of one voxel, Appendix A Algorithm 1: fluxes from the
// pre-step masses, each clamped to what its source pool holds, then applied.
template <typename R>
__device__ __forceinline__ void transform(const Coef<R> &C, R &m1, R &m2, R &m3, R &m4, R &m5) {
    R uptake = C.v_dom * m2 / (C.k_dom + m2) * m1 * C.dt;
    if (uptake > m2) uptake = m2;
    R resp = C.rho * m1 * C.dt;
    R morta = C.mu * m1 * C.dt;
    if (resp + morta > m1) {
        if (morta > m1) {
            morta = m1;
            resp = R(0);
        } else {
            resp = m1 - morta;
        }
    }
    R turn_p4 = C.v_p4 * m4 * C.dt;
    if (turn_p4 > m4) turn_p4 = m4;
    R turn_som = C.v_som * m3 * C.dt;
    if (turn_som > m3) turn_som = m3;
    const R n1 = m1 + (uptake - morta - resp);
    R n2, n3, n4;
    if (C.route == 0) {
        const R to_som = C.omb * morta;
        const R to_dom = C.beta * morta;
        n2 = m2 + (to_dom - uptake + turn_p4 + turn_som);
        n3 = m3 + (to_som - turn_som);
        n4 = m4 - turn_p4;
    } else {
        n2 = m2 + (R(0) - uptake + turn_p4 + turn_som);
        n3 = m3 + (R(0) - turn_som);
        n4 = m4 + (morta - turn_p4);
    }
    m1 = n1;
    m2 = n2;
    m3 = n3;
    m4 = n4;
    m5 = m5 + resp;
}

template <typename R>
struct StepBufs {
    const int32_t *nbr;     // [6][n]
    const uint16_t *rcode;  // [n] or null
    const R *src[VG_NPOOL];
    R *dst[VG_NPOOL];
    int64_t n;
};

#ifndef VG_NT
#define VG_NT 0
#endif
// Loads and stores of data used once per pass (the neighbour table, the
// immobile pools) may bypass cache allocation so that the gathered pools stay
// resident.
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) {
#if VG_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <typename T>
__device__ __forceinline__ void st_once(T *p, T v) {
#if VG_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// MOB: 1 = only DOM diffuses, 2 = every pool diffuses (a_s may be 0).
template <int MOB>
__device__ __forceinline__ constexpr bool mobile(int s) {
    return MOB == 2 || (MOB == 1 && s == 1);
}

template <int MODE, int MOB, int TOT>
__device__ __forceinline__ constexpr bool reads(int s) {
    // a diffusion-only pass reads the immobile pools only to total them
    return MODE != MODE_D || mobile<MOB>(s) || TOT != TOT_NONE;
}

// Scheme 1 for the mobile pools of one voxel: x_s += a_s * sum_k w_k (x_s,j - x_s,i),
// slot terms added as ((d0+d1)+(d2+d3))+(d4+d5).
template <typename R, int MOB, bool REG>
__device__ __forceinline__ void diffuse_voxel(const StepBufs<R> &B, const Coef<R> &C, int64_t i, const int32_t (&j)[6],
                                              const R (&w)[6], R (&x)[VG_NPOOL]) {
#pragma unroll
    for (int s = 0; s < VG_NPOOL; s++) {
        if (!mobile<MOB>(s)) continue;
        const R xi = x[s];
        // all six loads are issued before any is used (an absent neighbour
        // reads the voxel itself and contributes 0), so their latencies overlap
        R v[6];
#pragma unroll
        for (int k = 0; k < 6; k++) v[k] = B.src[s][j[k] >= 0 ? (int64_t)j[k] : i];
        R d[6];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const R diff = v[k] - xi;
            d[k] = j[k] >= 0 ? (REG ? w[k] * diff : diff) : R(0);
        }
        const R sum = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]);
        x[s] = xi + C.a[s] * sum;
    }
}

// A thread handles kVPT voxels of its tile.  The work is split into phases
// over all of them (indices, own loads, neighbour loads, arithmetic and
// stores) so that every load of the thread is in flight before the first
// result is needed; no store precedes a load of the same thread.

// own pools of every voxel of the thread (inactive lanes read a valid index)
template <typename R, int MODE, int MOB, int TOT>
__device__ __forceinline__ void load_own(const StepBufs<R> &B, const int64_t (&ic)[kVPT], R (&x)[kVPT][VG_NPOOL]) {
#pragma unroll
    for (int v = 0; v < kVPT; v++)
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++)
            x[v][s] = reads<MODE, MOB, TOT>(s) ? (mobile<MOB>(s) ? B.src[s][ic[v]] : ld_once(&B.src[s][ic[v]])) : R(0);
}

// Scheme 1 for DOM only, all gathers first: x_1 += a_1 * sum_k w_k (x_1,j - x_1,i).
template <typename R, bool REG>
__device__ __forceinline__ void diffuse_dom(const StepBufs<R> &B, const Coef<R> &C, const int64_t (&ic)[kVPT],
                                            const int32_t (&j)[kVPT][6], const R (&w)[kVPT][6],
                                            R (&x)[kVPT][VG_NPOOL]) {
    R g[kVPT][6];
#pragma unroll
    for (int v = 0; v < kVPT; v++)
#pragma unroll
        for (int k = 0; k < 6; k++) g[v][k] = B.src[1][j[v][k] >= 0 ? (int64_t)j[v][k] : ic[v]];
#pragma unroll
    for (int v = 0; v < kVPT; v++) {
        const R xi = x[v][1];
        R d[6];
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const R diff = g[v][k] - xi;
            d[k] = j[v][k] >= 0 ? (REG ? w[v][k] * diff : diff) : R(0);
        }
        const R sum = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]);
        x[v][1] = xi + C.a[1] * sum;
    }
}

// After the neighbours are known: diffuse, total, transform, store.
template <typename R, int MODE, int MOB, bool REG, int TOT>
__device__ __forceinline__ void finish(const StepBufs<R> &B, const Coef<R> &C, const int64_t (&ic)[kVPT],
                                       const bool (&act)[kVPT], const int32_t (&j)[kVPT][6], const R (&w)[kVPT][6],
                                       R (&x)[kVPT][VG_NPOOL], double (&acc)[kVPT][VG_NPOOL]) {
    constexpr bool do_d = MODE == MODE_D || MODE == MODE_DT;
    constexpr bool do_t = MODE == MODE_T || MODE == MODE_DT;
#pragma unroll
    for (int v = 0; v < kVPT; v++)
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) acc[v][s] = (TOT == TOT_IN && act[v]) ? (double)x[v][s] : 0.0;
    if (do_d) {
        if (MOB == 1) {
            diffuse_dom<R, REG>(B, C, ic, j, w, x);
        } else {
#pragma unroll
            for (int v = 0; v < kVPT; v++) diffuse_voxel<R, MOB, REG>(B, C, ic[v], j[v], w[v], x[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < kVPT; v++) {
        if (TOT == TOT_MID && act[v]) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[v][s] = (double)x[v][s];
        }
        if (do_t) transform(C, x[v][0], x[v][1], x[v][2], x[v][3], x[v][4]);
        if (TOT == TOT_OUT && act[v]) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[v][s] = (double)x[v][s];
        }
    }
    if (MODE != MODE_NONE) {
#pragma unroll
        for (int v = 0; v < kVPT; v++) {
            if (!act[v]) continue;
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) {
                if (mobile<MOB>(s)) B.dst[s][ic[v]] = x[v][s];
                else if (MODE != MODE_D) st_once(&B.dst[s][ic[v]], x[v][s]);
            }
        }
    }
}

template <typename R, int MODE, int MOB, bool REG, int TOT>
__global__ __launch_bounds__(kBlock) void k_step(StepBufs<R> B, Coef<R> C, Pieces pc, double *__restrict__ part) {
    __shared__ double lds[kWaves * VG_NPOOL];
    __shared__ R cl[VG_NREG];
    constexpr bool do_d = MODE == MODE_D || MODE == MODE_DT;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    if (REG) {
        if (threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];
        __syncthreads();
    }
    int64_t ic[kVPT];
    bool act[kVPT];
#pragma unroll
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = tile * kTile + v * kBlock + threadIdx.x;
        act[v] = i < B.n;
        ic[v] = act[v] ? i : B.n - 1;
    }
    int32_t j[kVPT][6];
    R w[kVPT][6];
    if (do_d) {
#pragma unroll
        for (int v = 0; v < kVPT; v++) {
#pragma unroll
            for (int k = 0; k < 6; k++) j[v][k] = ld_once(&B.nbr[(int64_t)k * B.n + ic[v]]);
            if (REG) {
                const uint32_t code = B.rcode[ic[v]];
                const uint32_t own = code & 7u;
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const uint32_t other = own ^ (((code >> (3 + k)) & 1u) << (k >> 1));
                    w[v][k] = R(0.5) * (cl[own] + cl[other]);
                }
            }
        }
    }
    R x[kVPT][VG_NPOOL];
    load_own<R, MODE, MOB, TOT>(B, ic, x);
    double acc[kVPT][VG_NPOOL];
    finish<R, MODE, MOB, REG, TOT>(B, C, ic, act, j, w, x, acc);
    if (TOT != TOT_NONE) {
        const int32_t p0 = pc.piece_first[tile], p1 = pc.piece_first[tile + 1];
        for (int32_t p = p0; p < p1; p++) {
            const int64_t lo = pc.piece_lo[p], hi = pc.piece_lo[p + 1];
            double v5[VG_NPOOL] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < kVPT; v++) {
                const int64_t i = tile * kTile + v * kBlock + threadIdx.x;
                const bool in = i >= lo && i < hi;
#pragma unroll
                for (int s = 0; s < VG_NPOOL; s++) v5[s] += in ? acc[v][s] : 0.0;
            }
            block_sum<VG_NPOOL>(v5, lds);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int s = 0; s < VG_NPOOL; s++) part[(int64_t)p * VG_NPOOL + s] = v5[s];
            }
        }
    }
}

// Rank-index variant (single volume: one piece per tile).  FAST: raster
// order, no periodic axis, every dimension <= 1024.  Then the decode also
// stores each voxel's coordinates and whether its -x / +x neighbours are pore
// (compact indices i - 1 / i + 1 in raster order), so only the four +-y / +-z
// neighbours need a bitmap word each.
template <typename R, int MODE, int MOB, bool REG, int TOT, bool FAST>
__global__ __launch_bounds__(kBlock) void k_step_rank(StepBufs<R> B, Coef<R> C, RGeom G, double *__restrict__ part) {
    __shared__ int32_t pos[kTile];
    __shared__ int32_t done;
    __shared__ double lds[kWaves * VG_NPOOL];
    __shared__ R cl[VG_NREG];
    constexpr bool do_d = MODE == MODE_D || MODE == MODE_DT;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t n = B.n;
    const uint32_t i0 = (uint32_t)(tile * kTile);
    const uint32_t i1 = (uint32_t)(i0 + kTile < n ? i0 + kTile : n);
    if (REG && threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];

    int64_t ic[kVPT];
    bool act[kVPT];
#pragma unroll
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = (int64_t)i0 + v * kBlock + threadIdx.x;
        act[v] = i < (int64_t)i1;
        ic[v] = act[v] ? i : n - 1;
    }
    // own pools first: their latency overlaps the decode below
    R x[kVPT][VG_NPOOL];
    load_own<R, MODE, MOB, TOT>(B, ic, x);

    if (do_d || REG) {
        // decode the enumeration positions of compact voxels [i0, i1) into LDS
        int64_t w = (int64_t)G.tile_word[tile] + threadIdx.x;
        for (;;) {
            uint32_t end = 0;
            if (w < G.g.nwords) {
                const RankWord wd = G.rank[w];
                uint32_t bits = wd.bits;
                const uint32_t before = wd.before;
                end = before + (uint32_t)__popc(bits);
                if (before < i1 && end > i0) {
                    uint32_t idx = before;
                    if (FAST) {
                        // coordinates of the word's first position, then per bit
                        const uint32_t p0 = (uint32_t)w << 5;
                        const uint32_t q1 = G.fnx.div(p0);
                        const uint32_t z0 = G.fny.div(q1);
                        const int x0 = (int)(p0 - q1 * G.fnx.d), y0 = (int)(q1 - z0 * G.fny.d);
                        const uint32_t lo_bit = w > 0 ? G.rank[w - 1].bits >> 31 : 0u;
                        const uint32_t hi_bit = w + 1 < G.g.nwords ? G.rank[w + 1].bits & 1u : 0u;
                        const uint32_t all = bits;
                        while (bits) {
                            const uint32_t b = (uint32_t)(__ffs(bits) - 1);
                            if (idx >= i0 && idx < i1) {
                                int x = x0 + (int)b, y = y0, z = (int)z0;
                                if (x >= G.g.nx) {   // a word spans at most two rows when nx >= 32
                                    x -= G.g.nx;
                                    if (++y >= G.g.ny) { y = 0; z++; }
                                }
                                const uint32_t left = b > 0 ? (all >> (b - 1)) & 1u : lo_bit;
                                const uint32_t right = b < 31 ? (all >> (b + 1)) & 1u : hi_bit;
                                const uint32_t mx = (x > 0 && left) ? 1u : 0u;
                                const uint32_t px = (x + 1 < G.g.nx && right) ? 1u : 0u;
                                pos[idx - i0] = (int32_t)((uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20) |
                                                          (mx << 30) | (px << 31));
                            }
                            idx++;
                            bits &= bits - 1u;
                        }
                    } else {
                        while (bits) {
                            const uint32_t b = (uint32_t)(__ffs(bits) - 1);
                            if (idx >= i0 && idx < i1) pos[idx - i0] = (int32_t)(((uint32_t)w << 5) + b);
                            idx++;
                            bits &= bits - 1u;
                        }
                    }
                }
            }
            if (threadIdx.x == kBlock - 1) done = (w >= G.g.nwords || end >= i1) ? 1 : 0;
            __syncthreads();
            if (done) break;
            w += kBlock;
            __syncthreads();
        }
    }

    int32_t j[kVPT][6];
    R w[kVPT][6];
    if (do_d && FAST) {
        const uint32_t nx = G.fnx.d, plane = G.fnx.d * G.fny.d;
        uint32_t pq[kVPT][4];
        bool ok[kVPT][4];
#pragma unroll
        for (int v = 0; v < kVPT; v++) {
            const uint32_t c = (uint32_t)pos[act[v] ? v * kBlock + threadIdx.x : 0];
            const int x = (int)(c & 1023u), y = (int)((c >> 10) & 1023u), z = (int)((c >> 20) & 1023u);
            const uint32_t p = (uint32_t)x + nx * ((uint32_t)y + G.fny.d * (uint32_t)z);
            // an inactive lane borrows voxel i0's coordinates; its +-x flags
            // would point past the tile, so they are dropped
            j[v][0] = (act[v] && ((c >> 30) & 1u)) ? (int32_t)ic[v] - 1 : -1;
            j[v][1] = (act[v] && (c >> 31)) ? (int32_t)ic[v] + 1 : -1;
            ok[v][0] = y > 0;
            ok[v][1] = y + 1 < G.g.ny;
            ok[v][2] = z > 0;
            ok[v][3] = z + 1 < G.g.nz;
            pq[v][0] = ok[v][0] ? p - nx : p;
            pq[v][1] = ok[v][1] ? p + nx : p;
            pq[v][2] = ok[v][2] ? p - plane : p;
            pq[v][3] = ok[v][3] ? p + plane : p;
            if (REG) {
                const int hx = G.g.nx / 2, hy = G.g.ny / 2, hz = G.g.nz / 2;
                const int oct = 4 * (z >= hz) + 2 * (y >= hy) + (x >= hx);
                const int nb[6] = {oct ^ ((x - 1 >= hx) != (x >= hx)), oct ^ ((x + 1 >= hx) != (x >= hx)),
                                   oct ^ (2 * ((y - 1 >= hy) != (y >= hy))), oct ^ (2 * ((y + 1 >= hy) != (y >= hy))),
                                   oct ^ (4 * ((z - 1 >= hz) != (z >= hz))), oct ^ (4 * ((z + 1 >= hz) != (z >= hz)))};
#pragma unroll
                for (int k = 0; k < 6; k++) w[v][k] = R(0.5) * (cl[oct] + cl[nb[k]]);
            }
        }
        uint32_t wb[kVPT][4], wbefore[kVPT][4];
#pragma unroll
        for (int v = 0; v < kVPT; v++)
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const RankWord t = G.rank[pq[v][k] >> 5];
                wb[v][k] = t.bits;
                wbefore[v][k] = t.before;
            }
#pragma unroll
        for (int v = 0; v < kVPT; v++)
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t bit = pq[v][k] & 31u;
                const bool pore = ok[v][k] && ((wb[v][k] >> bit) & 1u);
                j[v][k + 2] = pore ? (int32_t)(wbefore[v][k] + (uint32_t)__popc(wb[v][k] & ((1u << bit) - 1u))) : -1;
            }
    } else if (do_d) {
        const int dims[3] = {G.g.nx, G.g.ny, G.g.nz};
        // position strides of the three axes in raster order
        const uint32_t stride[3] = {1u, G.fnx.d, G.fnx.d * G.fny.d};
        uint32_t pq[kVPT][6];
        bool ok[kVPT][6];
#pragma unroll
        for (int v = 0; v < kVPT; v++) {
            const uint32_t p = act[v] ? (uint32_t)pos[v * kBlock + threadIdx.x] : (uint32_t)pos[0];
            int xyz[3];
            rg_xyz(G, p, xyz[0], xyz[1], xyz[2]);
            int oct = 0;
            if (REG) oct = 4 * (xyz[2] >= dims[2] / 2) + 2 * (xyz[1] >= dims[1] / 2) + (xyz[0] >= dims[0] / 2);
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int axis = k >> 1;
                const bool up = k & 1;
                int q[3] = {xyz[0], xyz[1], xyz[2]};
                q[axis] += up ? 1 : -1;
                bool inside = true, wrapped = false;
                if (q[axis] < 0 || q[axis] >= dims[axis]) {
                    if (G.periodic & (1u << axis)) {
                        q[axis] = q[axis] < 0 ? q[axis] + dims[axis] : q[axis] - dims[axis];
                        wrapped = true;
                    } else {
                        inside = false;
                    }
                }
                ok[v][k] = inside;
                if (!inside) pq[v][k] = p;         // any valid position: its word is loaded, not used
                else if (G.g.b <= 0 && !wrapped) pq[v][k] = up ? p + stride[axis] : p - stride[axis];
                else pq[v][k] = rg_pos(G, q[0], q[1], q[2]);
                if (REG) {
                    const int oq = 4 * (q[2] >= dims[2] / 2) + 2 * (q[1] >= dims[1] / 2) + (q[0] >= dims[0] / 2);
                    w[v][k] = R(0.5) * (cl[oct] + cl[oq]);
                }
            }
        }
        // all bitmap words of the thread are loaded before any is used
        uint32_t wb[kVPT][6], wbefore[kVPT][6];
#pragma unroll
        for (int v = 0; v < kVPT; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const RankWord t = G.rank[pq[v][k] >> 5];
                wb[v][k] = t.bits;
                wbefore[v][k] = t.before;
            }
#pragma unroll
        for (int v = 0; v < kVPT; v++)
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const uint32_t bit = pq[v][k] & 31u;
                const bool pore = ok[v][k] && ((wb[v][k] >> bit) & 1u);
                j[v][k] = pore ? (int32_t)(wbefore[v][k] + (uint32_t)__popc(wb[v][k] & ((1u << bit) - 1u))) : -1;
            }
    }
    double acc[kVPT][VG_NPOOL];
    finish<R, MODE, MOB, REG, TOT>(B, C, ic, act, j, w, x, acc);
    if (TOT != TOT_NONE) {
        double a5[VG_NPOOL] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < kVPT; v++)
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) a5[s] += acc[v][s];
        block_sum<VG_NPOOL>(a5, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) part[tile * VG_NPOOL + s] = a5[s];
        }
    }
}

// Word of the rank index that holds compact index t * kTile (binary search
// over the non-decreasing `before` counts).
__global__ __launch_bounds__(kBlock) void k_tile_words(const RankWord *__restrict__ rank, int64_t nwords,
                                                       int64_t ntiles, int32_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= ntiles) return;
    const uint32_t target = (uint32_t)(t * kTile);
    int64_t lo = 0, hi = nwords - 1;   // last word with before <= target
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (rank[mid].before <= target) lo = mid;
        else hi = mid - 1;
    }
    out[t] = (int32_t)lo;
}

// Totals, stage 1: chunks of up to kChunk pieces of one segment.
__global__ __launch_bounds__(kBlock) void k_tot_chunks(const double *__restrict__ part,
                                                       const int32_t *__restrict__ chunk_first,
                                                       double *__restrict__ chunk_part) {
    __shared__ double lds[kWaves * VG_NPOOL];
    const int c = blockIdx.x;
    const int32_t p = chunk_first[c] + (int32_t)threadIdx.x;
    double v[VG_NPOOL] = {0, 0, 0, 0, 0};
    if (p < chunk_first[c + 1]) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) v[s] = part[(int64_t)p * VG_NPOOL + s];
    }
    block_sum<VG_NPOOL>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) chunk_part[(int64_t)c * VG_NPOOL + s] = v[s];
    }
}

// Totals, stage 2: one block per segment sums its chunks in a fixed order,
// then the five pool totals into total carbon.
__global__ __launch_bounds__(kBlock) void k_tot_segments(const double *__restrict__ chunk_part,
                                                         const int32_t *__restrict__ seg_chunk,
                                                         double *__restrict__ out) {
    __shared__ double lds[kWaves * VG_NPOOL];
    const int g = blockIdx.x;
    double v[VG_NPOOL] = {0, 0, 0, 0, 0};
    for (int32_t c = seg_chunk[g] + (int32_t)threadIdx.x; c < seg_chunk[g + 1]; c += kBlock) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) v[s] += chunk_part[(int64_t)c * VG_NPOOL + s];
    }
    block_sum<VG_NPOOL>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) out[g * 6 + s] = v[s];
        out[g * 6 + 5] = ((v[0] + v[1]) + (v[2] + v[3])) + v[4];
    }
}

RGeom make_rgeom(const vg_sim *h) {
    RGeom G;
    make_geom(h->nx, h->ny, h->nz, h->brick, &G.g);
    G.fnx.init((uint32_t)h->nx);
    G.fny.init((uint32_t)h->ny);
    const uint32_t b = h->brick > 0 ? (uint32_t)h->brick : 1u;
    G.fb.init(b);
    G.fb2.init(b * b);
    G.fb3.init(b * b * b);
    G.fnbx.init(G.g.nbx > 0 ? (uint32_t)G.g.nbx : 1u);
    G.fnby.init(G.g.nby > 0 ? (uint32_t)G.g.nby : 1u);
    G.periodic = h->periodic;
    G.rank = (const RankWord *)h->rank;
    G.tile_word = h->tile_word;
    return G;
}

template <typename R, int MODE, int MOB, bool REG, int TOT>
int launch_one(vg_sim *h, const StepBufs<R> &B, const Coef<R> &C, hipStream_t s) {
    if (use_rank(h) && MODE != MODE_NONE) {
        const bool fast = h->brick == 0 && h->periodic == 0 && h->nx <= 1024 && h->ny <= 1024 && h->nz <= 1024 &&
                          h->nx >= 32;
        if (fast)
            hipLaunchKernelGGL((k_step_rank<R, MODE, MOB, REG, TOT, true>), dim3((unsigned)h->ntiles), dim3(kBlock), 0,
                               s, B, C, make_rgeom(h), h->part);
        else
            hipLaunchKernelGGL((k_step_rank<R, MODE, MOB, REG, TOT, false>), dim3((unsigned)h->ntiles), dim3(kBlock),
                               0, s, B, C, make_rgeom(h), h->part);
        return launch_status("k_step_rank");
    }
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    hipLaunchKernelGGL((k_step<R, MODE, MOB, REG, TOT>), dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, B, C, pc,
                       h->part);
    return launch_status("k_step");
}

template <typename R, int MODE, int MOB, bool REG>
int pick_tot(vg_sim *h, int tot, const StepBufs<R> &B, const Coef<R> &C, hipStream_t s) {
    switch (tot) {
        case TOT_NONE: return launch_one<R, MODE, MOB, REG, TOT_NONE>(h, B, C, s);
        case TOT_IN: return launch_one<R, MODE, MOB, REG, TOT_IN>(h, B, C, s);
        case TOT_MID: return launch_one<R, MODE, MOB, REG, TOT_MID>(h, B, C, s);
        default: return launch_one<R, MODE, MOB, REG, TOT_OUT>(h, B, C, s);
    }
}

template <typename R, int MODE, int MOB>
int pick_reg(vg_sim *h, int tot, const StepBufs<R> &B, const Coef<R> &C, hipStream_t s) {
    if (B.rcode) return pick_tot<R, MODE, MOB, true>(h, tot, B, C, s);
    return pick_tot<R, MODE, MOB, false>(h, tot, B, C, s);
}

template <typename R>
int dispatch_bufs(vg_sim *h, int mode, int tot, double dt, const StepBufs<R> &B, hipStream_t s) {
    const Coef<R> C = make_coef<R>(h, dt);
    const int mob = h->mobile_mode();
    if (mode == MODE_T) return pick_tot<R, MODE_T, 1, false>(h, tot, B, C, s);
    if (mode == MODE_NONE) return launch_one<R, MODE_NONE, 1, false, TOT_IN>(h, B, C, s);
    if (mode == MODE_D) return mob == 2 ? pick_reg<R, MODE_D, 2>(h, tot, B, C, s)
                                        : pick_reg<R, MODE_D, 1>(h, tot, B, C, s);
    return mob == 2 ? pick_reg<R, MODE_DT, 2>(h, tot, B, C, s) : pick_reg<R, MODE_DT, 1>(h, tot, B, C, s);
}

template <typename R>
int dispatch(vg_sim *h, int mode, int tot, double dt, hipStream_t s) {
    StepBufs<R> B;
    B.nbr = h->nbr;
    B.rcode = h->rcode;
    B.n = h->n;
    const int mob = h->mobile_mode();
    R *canon = (R *)h->fields;
    R *alt = (R *)h->alt;
    for (int p = 0; p < VG_NPOOL; p++) {
        const bool mob_p = mob == 2 || p == 1;
        R *here = canon + (int64_t)p * h->n;
        R *there = nullptr;
        if (mob_p) there = (mob == 2) ? alt + (int64_t)p * h->n : alt;
        R *cur = (mob_p && h->cur) ? there : here;
        R *oth = (mob_p && h->cur) ? here : there;
        B.src[p] = cur;
        // a pass that diffuses writes mobile pools to the other buffer
        B.dst[p] = (mob_p && (mode == MODE_D || mode == MODE_DT)) ? oth : cur;
    }
    const int rc = dispatch_bufs<R>(h, mode, tot, dt, B, s);
    if (rc) return rc;
    if (mode == MODE_D || mode == MODE_DT) h->cur ^= 1;
    return VG_OK;
}

}  // namespace

bool use_rank(const vg_sim *h) {
    const bool ok = h->rank != nullptr && h->tile_word != nullptr && h->nseg == 1;
    if (h->kernel == 1) return false;
    return ok;
}

int launch_tile_words(vg_sim *h, hipStream_t s) {
    if (!h->rank || h->ntiles == 0) return VG_OK;
    Geom g;
    int rc = make_geom(h->nx, h->ny, h->nz, h->brick, &g);
    if (rc) return rc;
    hipLaunchKernelGGL(k_tile_words, dim3((unsigned)((h->ntiles + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const RankWord *)h->rank, g.nwords, h->ntiles, h->tile_word);
    return launch_status("k_tile_words");
}

int launch_pass(vg_sim *h, int mode, int tot, double dt, hipStream_t s) {
    if (h->n == 0) return VG_OK;
    if (h->prec == VG_F64) return dispatch<double>(h, mode, tot, dt, s);
    return dispatch<float>(h, mode, tot, dt, s);
}

// A pass between explicit buffers (pool s read from src[s], written to
// dst[s]); used by the adjoint's forward recording.
int launch_pass_bufs(vg_sim *h, int mode, int tot, double dt, const void *const src[VG_NPOOL],
                     void *const dst[VG_NPOOL], hipStream_t s) {
    if (h->n == 0) return VG_OK;
    if (h->prec == VG_F64) {
        StepBufs<double> B;
        B.nbr = h->nbr; B.rcode = h->rcode; B.n = h->n;
        for (int p = 0; p < VG_NPOOL; p++) { B.src[p] = (const double *)src[p]; B.dst[p] = (double *)dst[p]; }
        return dispatch_bufs<double>(h, mode, tot, dt, B, s);
    }
    StepBufs<float> B;
    B.nbr = h->nbr; B.rcode = h->rcode; B.n = h->n;
    for (int p = 0; p < VG_NPOOL; p++) { B.src[p] = (const float *)src[p]; B.dst[p] = (float *)dst[p]; }
    return dispatch_bufs<float>(h, mode, tot, dt, B, s);
}

int launch_totals_finalize(vg_sim *h, double *out_rows, hipStream_t s) {
    if (h->nseg == 0 || h->n == 0) return VG_OK;
    hipLaunchKernelGGL(k_tot_chunks, dim3((unsigned)h->nchunks), dim3(kBlock), 0, s, h->part, h->chunk_first,
                       h->chunk_part);
    int rc = launch_status("k_tot_chunks");
    if (rc) return rc;
    hipLaunchKernelGGL(k_tot_segments, dim3((unsigned)h->nseg), dim3(kBlock), 0, s, h->chunk_part, h->seg_chunk,
                       out_rows);
    return launch_status("k_tot_segments");
}

// Mobile pools that currently live in the alt buffer are copied back to the
// caller's field buffer, so the fields hold the state between calls.
int restore_canonical(vg_sim *h, hipStream_t s) {
    if (!h->cur) return VG_OK;
    const size_t e = h->elem();
    const int mob = h->mobile_mode();
    int rc;
    if (mob == 2) {
        rc = hip_status(hipMemcpyAsync(h->fields, h->alt, e * VG_NPOOL * (size_t)h->n, hipMemcpyDeviceToDevice, s),
                        "restore fields");
    } else {
        rc = hip_status(hipMemcpyAsync(h->fields + e * (size_t)h->n, h->alt, e * (size_t)h->n,
                                       hipMemcpyDeviceToDevice, s),
                        "restore DOM");
    }
    if (rc) return rc;
    h->cur = 0;
    return VG_OK;
}

}  // namespace vg
