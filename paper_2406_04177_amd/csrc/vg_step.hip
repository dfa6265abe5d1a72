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
//   rank   a 32-bit geometry word per voxel (packed coordinates, and in raster
//          order the -x / +x neighbours, which are i - 1 / i + 1) plus the rank
//          index of the enumeration: a neighbour's compact index is the rank of
//          its position (pore-bitmap word + popcount; the words are cache
//          hits), so a pass moves ~46 B per voxel instead of 64 B.  Single
//          volume, no periodic axis, every dimension <= 1024.
//   offset two 32-bit words per voxel holding the distances i - j (minus side)
//          and j - i (plus side) to its neighbours in the enumeration, packed
//          by axis (48 B per voxel and pass, and the neighbour loads depend on
//          one load only).  Any volume or batch without periodic wrap whose
//          largest distances fit the packing.
//   relative  one 32-bit word per voxel of per-slot codes relative to base
//          distances shared by each group of 64 voxels (one wave): 44.5 B per
//          voxel and pass.  The default where it fits.
//
// The band kernel (k_band2, below) applies two fused passes per launch to
// bands of rows marching along z, keeping the first pass's DOM in LDS, for a
// single raster volume with relative codes.
//
// The paper's step is T then D.  The pass computes K = T o D (diffuse, then
// transform), so n paper steps run as T, K^(n-1), D.  Inside a K pass the
// state between its D and T halves is exactly the paper state after a full
// step, which is where the totals of that step are taken.
#include "vg_internal.h"

#pragma clang fp contract(off)

namespace vg {
namespace {

// Transformation of one voxel, Appendix A Algorithm 2 (sequential): uptake,
// mortality, respiration, SOM and FOM turnover update the masses one after
// the other, each from what the previous left; a process that would take
// more than its source holds takes all of it.  The printed algorithm's slips
// are read as corrected (each turnover against its own pool, the pool moved
// to DOM before it is zeroed, MB zeroed when it all dies).
template <typename R>
__device__ __forceinline__ void transform_seq(const Coef<R> &C, R &m1, R &m2, R &m3, R &m4, R &m5) {
    if (m1 > R(0)) {
        if (m2 > R(0)) {
            const R uptake = C.v_dom * m2 / (C.k_dom + m2) * m1 * C.dt;
            if (uptake < m2) {
                m1 = m1 + uptake;
                m2 = m2 - uptake;
            } else {
                m1 = m1 + m2;
                m2 = R(0);
            }
        }
        const R morta = C.mu * m1 * C.dt;
        const R dead = morta < m1 ? morta : m1;
        m1 = morta < m1 ? m1 - morta : R(0);
        if (C.route == 0) {
            m2 = m2 + C.beta * dead;
            m3 = m3 + C.omb * dead;
        } else {
            m4 = m4 + dead;
        }
        const R resp = C.rho * m1 * C.dt;
        if (resp < m1) {
            m1 = m1 - resp;
            m5 = m5 + resp;
        } else {
            m5 = m5 + m1;
            m1 = R(0);
        }
    }
    if (m3 > R(0)) {
        const R turn = C.v_som * m3 * C.dt;
        if (turn < m3) {
            m3 = m3 - turn;
            m2 = m2 + turn;
        } else {
            m2 = m2 + m3;
            m3 = R(0);
        }
    }
    if (m4 > R(0)) {
        const R turn = C.v_p4 * m4 * C.dt;
        if (turn < m4) {
            m4 = m4 - turn;
            m2 = m2 + turn;
        } else {
            m2 = m2 + m4;
            m4 = R(0);
        }
    }
}

// Transformation of one voxel, Appendix A Algorithm 1: fluxes from the
// pre-step masses, each clamped to what its source pool holds, then applied.
template <typename R>
__device__ __forceinline__ void transform_flux(const Coef<R> &C, R &m1, R &m2, R &m3, R &m4, R &m5) {
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

// The algorithm chosen at compile time (the hot pass) or by C.seq.
template <bool SEQ, typename R>
__device__ __forceinline__ void transform_alg(const Coef<R> &C, R &m1, R &m2, R &m3, R &m4, R &m5) {
    if constexpr (SEQ) transform_seq(C, m1, m2, m3, m4, m5);
    else transform_flux(C, m1, m2, m3, m4, m5);
}

template <typename R>
__device__ __forceinline__ void transform(const Coef<R> &C, R &m1, R &m2, R &m3, R &m4, R &m5) {
    if (C.seq) transform_seq(C, m1, m2, m3, m4, m5);
    else transform_flux(C, m1, m2, m3, m4, m5);
}

template <typename R>
struct StepBufs {
    const int32_t *nbr = nullptr;       // [6][n]
    const uint16_t *rcode = nullptr;    // [n] or null
    PackedNbr pk;                       // packed neighbour sources (when built)
    const R *src[VG_NPOOL] = {};
    R *dst[VG_NPOOL] = {};
    // when set (a recording pass of the adjoint that keeps the diffused
    // DOM): a fused pass also writes each voxel's DOM after the diffusion
    // half, before the transformation, here
    R *xdom = nullptr;
    int64_t n = 0;
};

// The graph-side members of a pass's buffers, all taken from the handle (the
// pool pointers are the caller's).
template <typename R>
StepBufs<R> graph_bufs(const vg_sim *h) {
    StepBufs<R> B;
    B.nbr = h->nbr;
    B.rcode = h->rcode;
    B.pk = packed_of(h);
    B.n = h->n;
    return B;
}


// Loads and stores of data used once per pass (the neighbour table, the
// immobile pools); plain accesses (nontemporal ones measured no faster).
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) {
    return *p;
}
template <typename T>
__device__ __forceinline__ void st_once(T *p, T v) {
    *p = v;
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
    if (MODE == MODE_DT && MOB == 1 && B.xdom) {
#pragma unroll
        for (int v = 0; v < kVPT; v++)
            if (act[v]) B.xdom[ic[v]] = x[v][1];
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

// Per-piece sums of the thread's accumulators (a piece is the part of a tile
// inside one segment), written to part[piece][pool] in a fixed order; `lds`
// holds kRows * 5 doubles.
__device__ __forceinline__ void tile_totals(const Pieces &pc, int64_t tile, const double (&acc)[kVPT][VG_NPOOL],
                                            double *__restrict__ part, double *lds) {
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
        tile_sum_to<VG_NPOOL>(v5, lds, part + (int64_t)p * VG_NPOOL);
    }
}

template <typename R, int MODE, int MOB, bool REG, int TOT>
__global__ __launch_bounds__(kBlock) void k_step(StepBufs<R> B, Coef<R> C, Pieces pc, double *__restrict__ part) {
    __shared__ double lds[kRows * VG_NPOOL];
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
    if (TOT != TOT_NONE) tile_totals(pc, tile, acc, part, lds);
}

// Packed-offset variant of the diffusing passes (D and DT).  Neighbour j of
// voxel i is i - d or i + d with d unpacked from the voxel's two offset words;
// an absent neighbour has d = 0 and so reads the voxel itself, whose
// difference x_i - x_i is exactly +0 (the absent slot's zero) for finite
// values, so no selects are needed.  All indices are 32-bit.
template <typename R, int MODE, int MOB, bool REG, int TOT, bool RELC, bool SEQ, int V = kVPT>
__global__ __launch_bounds__(kBlock) void k_step_off(StepBufs<R> B, Coef<R> C, Pieces pc, double *__restrict__ part) {
    static_assert(MODE == MODE_D || MODE == MODE_DT, "diffusing passes only");
    __shared__ double lds[kRows * VG_NPOOL];
    __shared__ R cl[VG_NREG];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t n = (uint32_t)B.n;
    if (REG) {
        if (threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];
        __syncthreads();
    }
    uint32_t ic[V];
    bool act[V];
#pragma unroll
    for (int v = 0; v < V; v++) {
        const uint32_t i = (uint32_t)tile * (uint32_t)(kBlock * V) + (uint32_t)(v * kBlock) + threadIdx.x;
        act[v] = i < n;
        ic[v] = act[v] ? i : n - 1;
    }
    // the neighbour words first (the gathers depend on them), then the pools
    PackedWords pw[V];
#pragma unroll
    for (int v = 0; v < V; v++) pw[v] = packed_words<RELC>(B.pk, ic[v]);
    R x[V][VG_NPOOL];
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++)
            x[v][s] = reads<MODE, MOB, TOT>(s) ? (mobile<MOB>(s) ? at(B.src[s], ic[v]) : ld_once(&at(B.src[s], ic[v])))
                                               : R(0);
    uint32_t j[V][6];
#pragma unroll
    for (int v = 0; v < V; v++) packed_decode<RELC>(B.pk, ic[v], pw[v], j[v]);   // lanes past n hold n - 1
    R w[V][6];
#pragma unroll
    for (int v = 0; v < V; v++) {
        if (REG) {
            const uint32_t code = at(B.rcode, ic[v]);
            const uint32_t own = code & 7u;
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const uint32_t other = own ^ (((code >> (3 + k)) & 1u) << (k >> 1));
                w[v][k] = R(0.5) * (cl[own] + cl[other]);
            }
        }
    }
    double acc[V][VG_NPOOL];
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) acc[v][s] = (TOT == TOT_IN && act[v]) ? (double)x[v][s] : 0.0;
    // Scheme 1: every gather of the thread first, then the sums
    constexpr int NM = MOB == 2 ? VG_NPOOL : 1;
    R g[V][NM][6];
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int m = 0; m < NM; m++)
#pragma unroll
            for (int k = 0; k < 6; k++) g[v][m][k] = at(B.src[NM == 1 ? 1 : m], j[v][k]);
#pragma unroll
    for (int v = 0; v < V; v++)
#pragma unroll
        for (int m = 0; m < NM; m++) {
            const int s = NM == 1 ? 1 : m;
            const R xi = x[v][s];
            R d[6];
#pragma unroll
            for (int k = 0; k < 6; k++) d[k] = REG ? w[v][k] * (g[v][m][k] - xi) : g[v][m][k] - xi;
            const R sum = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]);
            x[v][s] = xi + C.a[s] * sum;
        }
    if (MODE == MODE_DT && MOB == 1 && B.xdom) {
#pragma unroll
        for (int v = 0; v < V; v++)
            if (act[v]) at(B.xdom, ic[v]) = x[v][1];
    }
#pragma unroll
    for (int v = 0; v < V; v++) {
        if (TOT == TOT_MID && act[v]) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[v][s] = (double)x[v][s];
        }
        if (MODE == MODE_DT) transform_alg<SEQ>(C, x[v][0], x[v][1], x[v][2], x[v][3], x[v][4]);
        if (TOT == TOT_OUT && act[v]) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[v][s] = (double)x[v][s];
        }
    }
#pragma unroll
    for (int v = 0; v < V; v++) {
        if (!act[v]) continue;
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            if (mobile<MOB>(s)) at(B.dst[s], ic[v]) = x[v][s];
            else if (MODE != MODE_D) st_once(&at(B.dst[s], ic[v]), x[v][s]);
        }
    }
    if constexpr (TOT != TOT_NONE) {
        // totals per reduction tile of kTile voxels: the thread's voxel v
        // lies in tile tile * V + v (uniform over the block)
        static_assert(kVPT == 1, "one voxel per thread and reduction tile");
#pragma unroll
        for (int v = 0; v < V; v++) {
            const int64_t tv = tile * V + v;
            if (tv * kTile < (int64_t)n) tile_totals(pc, tv, reinterpret_cast<const double(&)[1][VG_NPOOL]>(acc[v]), part, lds);
        }
    }
}

// Compensated float32 fields (VG_F32C): every pool is a float hi and an
// int16 compensation word lo (6 B per value, a 39-bit significand, see
// comp_get / comp_put).  The pass decodes to FP64, diffuses and transforms in
// FP64 with the operations of the FP64 pass in the same order, and rounds
// each value once on the way out.  Neighbours come from the table or a packed
// source, chosen at run time (uniform branch); region weights and the
// algorithm likewise.
struct CompBufs {
    const int32_t *nbr = nullptr;       // [6][n]
    const uint16_t *rcode = nullptr;    // [n] or null
    PackedNbr pk;
    int ns = 0;                         // 0 table, 1 relative codes, 2 packed offsets
    const float *src[VG_NPOOL] = {};
    const int16_t *slo[VG_NPOOL] = {};
    float *dst[VG_NPOOL] = {};
    int16_t *dlo[VG_NPOOL] = {};
    int64_t n = 0;
};

__device__ __forceinline__ double comp_at(const float *hi, const int16_t *lo, uint32_t i) {
    return comp_get(at(hi, i), at(lo, i));
}

template <int MODE, int MOB, int TOT>
__global__ __launch_bounds__(kBlock) void k_step_c(CompBufs B, Coef<double> C, Pieces pc,
                                                   double *__restrict__ part) {
    __shared__ double lds[kRows * VG_NPOOL];
    __shared__ double cl[VG_NREG];
    constexpr bool do_d = MODE == MODE_D || MODE == MODE_DT;
    constexpr bool do_t = MODE == MODE_T || MODE == MODE_DT;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t n = (uint32_t)B.n;
    const bool reg = B.rcode != nullptr;
    if (reg) {   // uniform over the block
        if (threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];
        __syncthreads();
    }
    const uint32_t i0 = (uint32_t)tile * (uint32_t)kBlock + threadIdx.x;
    const bool act = i0 < n;
    const uint32_t i = act ? i0 : n - 1;
    // neighbours: an absent one is the voxel itself (its difference is +0)
    uint32_t j[6];
    bool pres[6];
    if (do_d) {
        if (B.ns == 0) {
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int32_t jk = B.nbr[(int64_t)k * B.n + i];
                pres[k] = jk >= 0;
                j[k] = pres[k] ? (uint32_t)jk : i;
            }
        } else {
            const bool relc = B.ns == 1;
            const PackedWords W = relc ? packed_words<true>(B.pk, i) : packed_words<false>(B.pk, i);
            if (relc) packed_decode<true>(B.pk, i, W, j);
            else packed_decode<false>(B.pk, i, W, j);
#pragma unroll
            for (int k = 0; k < 6; k++) pres[k] = j[k] != i;   // no periodic wrap in packed sources
        }
    }
    double x[VG_NPOOL];
#pragma unroll
    for (int s = 0; s < VG_NPOOL; s++)
        x[s] = reads<MODE, MOB, TOT>(s) ? comp_at(B.src[s], B.slo[s], i) : 0.0;
    double acc[1][VG_NPOOL];
#pragma unroll
    for (int s = 0; s < VG_NPOOL; s++) acc[0][s] = (TOT == TOT_IN && act) ? x[s] : 0.0;
    if (do_d) {
        double w[6] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
        if (reg) {
            const uint32_t code = at(B.rcode, i);
            const uint32_t own = code & 7u;
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const uint32_t other = own ^ (((code >> (3 + k)) & 1u) << (k >> 1));
                w[k] = 0.5 * (cl[own] + cl[other]);
            }
        }
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            if (!mobile<MOB>(s)) continue;
            const double xi = x[s];
            double v[6];
#pragma unroll
            for (int k = 0; k < 6; k++) v[k] = comp_at(B.src[s], B.slo[s], j[k]);
            double d[6];
#pragma unroll
            for (int k = 0; k < 6; k++) d[k] = pres[k] ? (reg ? w[k] * (v[k] - xi) : v[k] - xi) : 0.0;
            const double sum = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]);
            x[s] = xi + C.a[s] * sum;
        }
    }
    if (TOT == TOT_MID && act) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) acc[0][s] = x[s];
    }
    if (do_t) transform(C, x[0], x[1], x[2], x[3], x[4]);
    if (TOT == TOT_OUT && act) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) acc[0][s] = x[s];
    }
    if (MODE != MODE_NONE && act) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            if (mobile<MOB>(s) || MODE != MODE_D) {
                float hi;
                int16_t lo;
                comp_put(x[s], hi, lo);
                at(B.dst[s], i) = hi;
                at(B.dlo[s], i) = lo;
            }
        }
    }
    if constexpr (TOT != TOT_NONE) tile_totals(pc, tile, acc, part, lds);
}

// Rank-index variant (single volume: one piece per tile).  Each voxel has a
// 32-bit geometry word (x | y << 10 | z << 20, and in raster order whether
// its -x / +x neighbours are pore in bits 30 / 31: their compact indices are
// then i - 1 / i + 1).  The other neighbours' compact indices are ranks of
// their positions: one pore-bitmap word (8 B, a cache hit) and a popcount.
// Per voxel and pass this reads 4 B of geometry instead of 24 B of table.
// Neighbours of one thread's voxels from their geometry words (rank index).
template <typename R, bool REG, bool RASTER>
__device__ __forceinline__ void geo_neighbours(const RGeom &G, const R *cl, const int64_t (&ic)[kVPT],
                                               const uint32_t (&gw)[kVPT], int32_t (&j)[kVPT][6],
                                               R (&w)[kVPT][6]) {
    constexpr int NW = RASTER ? 4 : 6;        // neighbours found through the bitmap
    const uint32_t nx = G.fnx.d, plane = G.fnx.d * G.fny.d;
    uint32_t pq[kVPT][NW];
    bool ok[kVPT][NW];
#pragma unroll
    for (int v = 0; v < kVPT; v++) {
        const uint32_t c = gw[v];
        const int xx = (int)(c & 1023u), yy = (int)((c >> 10) & 1023u), zz = (int)((c >> 20) & 1023u);
        if (RASTER) {
            const uint32_t p = (uint32_t)xx + nx * ((uint32_t)yy + G.fny.d * (uint32_t)zz);
            j[v][0] = ((c >> 30) & 1u) ? (int32_t)ic[v] - 1 : -1;
            j[v][1] = (c >> 31) ? (int32_t)ic[v] + 1 : -1;
            ok[v][0] = yy > 0;
            ok[v][1] = yy + 1 < G.g.ny;
            ok[v][2] = zz > 0;
            ok[v][3] = zz + 1 < G.g.nz;
            pq[v][0] = ok[v][0] ? p - nx : p;
            pq[v][1] = ok[v][1] ? p + nx : p;
            pq[v][2] = ok[v][2] ? p - plane : p;
            pq[v][3] = ok[v][3] ? p + plane : p;
        } else {
            const int xyz[3] = {xx, yy, zz};
            const int dims[3] = {G.g.nx, G.g.ny, G.g.nz};
            const uint32_t p = rg_pos(G, xx, yy, zz);
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int axis = k >> 1;
                int q[3] = {xyz[0], xyz[1], xyz[2]};
                q[axis] += (k & 1) ? 1 : -1;
                ok[v][k % NW] = q[axis] >= 0 && q[axis] < dims[axis];
                pq[v][k % NW] = ok[v][k % NW] ? rg_pos(G, q[0], q[1], q[2]) : p;
            }
        }
        if (REG) {
            const int hx = G.g.nx / 2, hy = G.g.ny / 2, hz = G.g.nz / 2;
            const int oct = 4 * (zz >= hz) + 2 * (yy >= hy) + (xx >= hx);
            const int nb[6] = {oct ^ ((xx - 1 >= hx) != (xx >= hx)), oct ^ ((xx + 1 >= hx) != (xx >= hx)),
                               oct ^ (2 * ((yy - 1 >= hy) != (yy >= hy))), oct ^ (2 * ((yy + 1 >= hy) != (yy >= hy))),
                               oct ^ (4 * ((zz - 1 >= hz) != (zz >= hz))), oct ^ (4 * ((zz + 1 >= hz) != (zz >= hz)))};
#pragma unroll
            for (int k = 0; k < 6; k++) w[v][k] = R(0.5) * (cl[oct] + cl[nb[k]]);
        }
    }
    // all bitmap words of the thread are loaded before any is used
    uint32_t wb[kVPT][NW], wbefore[kVPT][NW];
#pragma unroll
    for (int v = 0; v < kVPT; v++)
#pragma unroll
        for (int k = 0; k < NW; k++) {
            const RankWord t = G.rank[pq[v][k] >> 5];
            wb[v][k] = t.bits;
            wbefore[v][k] = t.before;
        }
#pragma unroll
    for (int v = 0; v < kVPT; v++)
#pragma unroll
        for (int k = 0; k < NW; k++) {
            const uint32_t bit = pq[v][k] & 31u;
            const bool pore = ok[v][k] && ((wb[v][k] >> bit) & 1u);
            j[v][k + 6 - NW] = pore ? (int32_t)(wbefore[v][k] + (uint32_t)__popc(wb[v][k] & ((1u << bit) - 1u))) : -1;
        }
}

// Rank-index variant (single volume, one tile per block).  Each voxel has a
// 32-bit geometry word (x | y << 10 | z << 20, and in raster order whether its
// -x / +x neighbours are pore in bits 30 / 31: their compact indices are then
// i - 1 / i + 1).  The other neighbours' compact indices are ranks of their
// positions: one pore-bitmap word (8 B, a cache hit) and a popcount.  Per
// voxel and pass this reads 4 B of geometry instead of 24 B of table.
// (A persistent, software-pipelined form of this kernel measured slower.)
template <typename R, int MODE, int MOB, bool REG, int TOT, bool RASTER>
__global__ __launch_bounds__(kBlock) void k_step_geo(StepBufs<R> B, Coef<R> C, RGeom G,
                                                     const uint32_t *__restrict__ geo, double *__restrict__ part) {
    __shared__ double lds[kRows * VG_NPOOL];
    __shared__ R cl[VG_NREG];
    constexpr bool do_d = MODE == MODE_D || MODE == MODE_DT;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t n = B.n;
    if (REG) {
        if (threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];
        __syncthreads();
    }
    int64_t ic[kVPT];
    bool act[kVPT];
#pragma unroll
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = tile * kTile + v * kBlock + threadIdx.x;
        act[v] = i < n;
        ic[v] = act[v] ? i : n - 1;
    }
    uint32_t gw[kVPT];
    if (do_d) {
#pragma unroll
        for (int v = 0; v < kVPT; v++) gw[v] = ld_once(&geo[ic[v]]);
    }
    R x[kVPT][VG_NPOOL];
    load_own<R, MODE, MOB, TOT>(B, ic, x);
    int32_t j[kVPT][6];
    R w[kVPT][6];
    if (do_d) geo_neighbours<R, REG, RASTER>(G, cl, ic, gw, j, w);
    double acc[kVPT][VG_NPOOL];
    finish<R, MODE, MOB, REG, TOT>(B, C, ic, act, j, w, x, acc);
    if (TOT != TOT_NONE) {
        double a5[VG_NPOOL] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < kVPT; v++)
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) a5[s] += acc[v][s];
        tile_sum_to<VG_NPOOL>(a5, lds, part + tile * VG_NPOOL);
    }
}

// Geometry words of the rank-index kernel, from the compacted list.
__global__ __launch_bounds__(kBlock) void k_geometry(const int32_t *__restrict__ vox, int64_t n, RGeom G,
                                                     uint32_t *__restrict__ geo) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = (uint32_t)vox[i];
    const uint32_t q1 = G.fnx.div(v);
    const uint32_t z = G.fny.div(q1);
    const uint32_t x = v - q1 * G.fnx.d, y = q1 - z * G.fny.d;
    uint32_t c = x | (y << 10) | (z << 20);
    if (G.g.b <= 0) {
        // raster: the -x / +x neighbours, when pore, are compact voxels i -/+ 1
        if (x > 0) {
            const RankWord wd = G.rank[(v - 1) >> 5];
            if ((wd.bits >> ((v - 1) & 31u)) & 1u) c |= 1u << 30;
        }
        if (x + 1 < G.fnx.d) {
            const RankWord wd = G.rank[(v + 1) >> 5];
            if ((wd.bits >> ((v + 1) & 31u)) & 1u) c |= 1u << 31;
        }
    }
    geo[i] = c;
}

// Packed offsets, pass 2: the two words of every voxel.
__global__ __launch_bounds__(kBlock) void k_offsets(const int32_t *__restrict__ nbr, int64_t n, DLayout L,
                                                    uint32_t *__restrict__ off_m, uint32_t *__restrict__ off_p) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t shift[3] = {L.sx, L.bz, 0};
    uint32_t wm = 0, wp = 0;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int32_t j = nbr[(int64_t)k * n + i];
        if (j < 0) continue;
        const uint32_t d = (k & 1) ? (uint32_t)((int64_t)j - i) : (uint32_t)(i - (int64_t)j);
        if (k & 1) wp |= d << shift[k >> 1];
        else wm |= d << shift[k >> 1];
    }
    off_m[i] = wm;
    off_p[i] = wp;
}

// Neighbour distances, one pass over the table (both packings): per group of
// 64 voxels (one wave) and slot the smallest distance, base[g][k]; over the
// graph the largest distance per axis (stat[0..2]), a flag when a minus-side
// neighbour does not precede the voxel or a plus-side one does not follow it
// (stat[3], as across a periodic wrap) and the largest spread + 1 of a slot's
// distances within a group, per axis (stat[4..6]).  A bounded grid strides
// over the voxels and each block adds its maxima with one atomic per value.
__global__ __launch_bounds__(kBlock) void k_neighbour_stat(const int32_t *__restrict__ nbr, int64_t n,
                                                           uint32_t *__restrict__ base, uint32_t *__restrict__ stat) {
    static_assert(kGroup == 64, "a group is one wave");
    __shared__ uint32_t red[kWaves][7];
    uint32_t acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < n; i0 += (int64_t)gridDim.x * kBlock) {
        const int64_t i = i0 + threadIdx.x;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const int32_t j = i < n ? nbr[(int64_t)k * n + i] : -1;
            const int64_t d64 = (k & 1) ? (int64_t)j - i : i - (int64_t)j;
            if (j >= 0 && d64 <= 0) acc[3] = 1;
            const bool pres = j >= 0 && d64 > 0;
            const uint32_t d = pres ? (uint32_t)d64 : 0u;
            acc[k >> 1] = max(acc[k >> 1], d);
            uint32_t lo = pres ? d : 0xffffffffu, hi = d;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
                hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
            }
            if ((threadIdx.x & 63) == 0 && i < n) base[(i / kGroup) * 8 + k] = lo == 0xffffffffu ? 0u : lo;
            if (lo != 0xffffffffu) acc[4 + (k >> 1)] = max(acc[4 + (k >> 1)], hi - lo + 1u);
        }
    }
#pragma unroll
    for (int q = 0; q < 7; q++)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[q] = max(acc[q], (uint32_t)__shfl_xor((int)acc[q], o, 64));
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 7; q++) red[threadIdx.x >> 6][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        uint32_t v = red[0][threadIdx.x];
        for (int w = 1; w < kWaves; w++) v = max(v, red[w][threadIdx.x]);
        if (v) atomicMax(&stat[threadIdx.x], v);
    }
}

// Relative codes, pass 2: the code word of every voxel.
__global__ __launch_bounds__(kBlock) void k_rel_pack(const int32_t *__restrict__ nbr, int64_t n,
                                                     const uint32_t *__restrict__ base, RLayout L,
                                                     uint32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t *bp = base + (i / kGroup) * 8;
    uint32_t w = 0;
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int32_t j = nbr[(int64_t)k * n + i];
        if (j < 0) continue;
        const uint32_t d = (uint32_t)((k & 1) ? (int64_t)j - i : i - (int64_t)j);
        w |= (d - bp[k] + 1u) << L.sh[k];
    }
    out[i] = w;
}

// Totals, stage 1: chunks of up to kChunk pieces of one segment (blockIdx.y:
// the logged pass; part and chunk_part advance by their row strides).
__global__ __launch_bounds__(kBlock) void k_tot_chunks(const double *__restrict__ part,
                                                       const int32_t *__restrict__ chunk_first,
                                                       double *__restrict__ chunk_part, int64_t part_stride,
                                                       int64_t chunk_stride) {
    __shared__ double lds[kWaves * VG_NPOOL];
    const int c = blockIdx.x;
    part += blockIdx.y * part_stride;
    chunk_part += blockIdx.y * chunk_stride;
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
                                                         double *__restrict__ out, int64_t chunk_stride,
                                                         int64_t out_stride) {
    __shared__ double lds[kWaves * VG_NPOOL];
    const int g = blockIdx.x;
    chunk_part += blockIdx.y * chunk_stride;
    out += blockIdx.y * out_stride;
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

// Totals in one stage, for segments of at most kDirectPieces pieces: one
// block per segment sums its pieces (thread t: pieces t, t + 256, ... in
// order, then the block in a fixed order), then the five pool totals into
// total carbon.
constexpr int32_t kDirectPieces = 4096;

__global__ __launch_bounds__(kBlock) void k_tot_direct(const double *__restrict__ part,
                                                       const int32_t *__restrict__ seg_first,
                                                       double *__restrict__ out, int64_t part_stride,
                                                       int64_t out_stride) {
    __shared__ double lds[kWaves * VG_NPOOL];
    const int g = blockIdx.x;
    part += blockIdx.y * part_stride;
    out += blockIdx.y * out_stride;
    double v[VG_NPOOL] = {0, 0, 0, 0, 0};
    for (int32_t p = seg_first[g] + (int32_t)threadIdx.x; p < seg_first[g + 1]; p += kBlock) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) v[s] += part[(int64_t)p * VG_NPOOL + s];
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
    return G;
}

template <typename R, int MODE, int MOB, bool REG, int TOT>
int launch_one(vg_sim *h, const StepBufs<R> &B, const Coef<R> &C, hipStream_t s) {
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    if constexpr (MODE == MODE_D || MODE == MODE_DT) {
        // the algorithm is a template argument of the packed-source pass
        // (Algorithm 2 instances only where a transformation runs)
        const bool seq = MODE == MODE_DT && C.seq;
        if constexpr (MODE == MODE_D) {
            // diffusion-only passes move 12.5 B per voxel (28.5 with totals):
            // two voxels per thread keep more loads in flight (measured 6.5 %
            // faster sub-cycled runs; the fused pass is faster with one)
            constexpr int V2 = 2;
            const unsigned grid = (unsigned)((h->n + kBlock * V2 - 1) / (kBlock * V2));
            if (use_relative(h)) {
                hipLaunchKernelGGL((k_step_off<R, MODE, MOB, REG, TOT, true, false, V2>), dim3(grid), dim3(kBlock),
                                   0, s, B, C, pc, part_of(h));
                return launch_status("k_step_off relative");
            }
            if (use_offsets(h)) {
                hipLaunchKernelGGL((k_step_off<R, MODE, MOB, REG, TOT, false, false, V2>), dim3(grid), dim3(kBlock),
                                   0, s, B, C, pc, part_of(h));
                return launch_status("k_step_off");
            }
        }
        if (use_relative(h)) {
            if (seq)
                hipLaunchKernelGGL((k_step_off<R, MODE, MOB, REG, TOT, true, MODE == MODE_DT>),
                                   dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, B, C, pc, part_of(h));
            else
                hipLaunchKernelGGL((k_step_off<R, MODE, MOB, REG, TOT, true, false>), dim3((unsigned)h->ntiles),
                                   dim3(kBlock), 0, s, B, C, pc, part_of(h));
            return launch_status("k_step_off relative");
        }
        if (use_offsets(h)) {
            if (seq)
                hipLaunchKernelGGL((k_step_off<R, MODE, MOB, REG, TOT, false, MODE == MODE_DT>),
                                   dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, B, C, pc, part_of(h));
            else
                hipLaunchKernelGGL((k_step_off<R, MODE, MOB, REG, TOT, false, false>), dim3((unsigned)h->ntiles),
                                   dim3(kBlock), 0, s, B, C, pc, part_of(h));
            return launch_status("k_step_off");
        }
    }
    if (use_rank(h) && MODE != MODE_NONE) {
        if (h->brick == 0)
            hipLaunchKernelGGL((k_step_geo<R, MODE, MOB, REG, TOT, true>), dim3((unsigned)h->ntiles), dim3(kBlock), 0,
                               s, B, C, make_rgeom(h), h->geo, part_of(h));
        else
            hipLaunchKernelGGL((k_step_geo<R, MODE, MOB, REG, TOT, false>), dim3((unsigned)h->ntiles), dim3(kBlock), 0,
                               s, B, C, make_rgeom(h), h->geo, part_of(h));
        return launch_status("k_step_geo");
    }
    hipLaunchKernelGGL((k_step<R, MODE, MOB, REG, TOT>), dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, B,
                       C, pc, part_of(h));
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
int dispatch_bufs(vg_sim *h, int mode, int tot, double dt_t, double dt_d, const StepBufs<R> &B, hipStream_t s) {
    const Coef<R> C = make_coef2<R>(h, dt_t, dt_d);
    const int mob = h->mobile_mode();
    if (mode == MODE_T) return pick_tot<R, MODE_T, 1, false>(h, tot, B, C, s);
    if (mode == MODE_NONE) return launch_one<R, MODE_NONE, 1, false, TOT_IN>(h, B, C, s);
    if (mode == MODE_D) return mob == 2 ? pick_reg<R, MODE_D, 2>(h, tot, B, C, s)
                                        : pick_reg<R, MODE_D, 1>(h, tot, B, C, s);
    return mob == 2 ? pick_reg<R, MODE_DT, 2>(h, tot, B, C, s) : pick_reg<R, MODE_DT, 1>(h, tot, B, C, s);
}

// ---------------------------------------------------------------- band kernel
// Two fused passes (x <- T(D(x)), twice) in one launch, for a single volume
// in raster order with relative neighbour codes, only DOM diffusing, unit
// weights and Algorithm 1.  Block (band, chunk) owns the rows
// [y0, y0 + H) of the planes [z0, z0 + Z) and marches along z.  At plane p
// it applies the first pass to the rows [y0 - 1, y0 + H] (the band and one
// neighbour row on each side: one contiguous range of the compact list) and
// keeps in LDS the DOM of those rows after the first pass (three planes) and
// after its diffusion (two planes).  Then it applies the second pass to the
// band rows of plane p - 1: every neighbour's first-pass DOM is in LDS (same
// plane: band and neighbour rows; planes p - 2 and p: band rows); the other
// first-pass pools are recomputed from the input pools and the diffused DOM.
// The output is written once per pass pair.  Inputs and outputs are separate
// field sets, since neighbouring blocks read the inputs next to their rows
// and planes.  Same operations in the same order as two single passes, so
// the result is bit-identical.
struct BandGeom {
    int ny, nz, H, Z, nbands, cap;   // cap: the widest range of a plane's band and neighbour rows
};

// rs[r] = compact index of the first pore voxel at or after the start of
// row r = z * ny + y (vox ascending: the raster-order compact list).
__global__ __launch_bounds__(kBlock) void k_band_rows(const int32_t *__restrict__ vox, int64_t n, int nx,
                                                      int64_t nrows, int32_t *__restrict__ rs) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r > nrows) return;
    const int64_t target = r * nx;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)vox[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    rs[r] = (int32_t)lo;
}

// LDS of a block: [3][cap] DOM after the first pass, [2][cap] DOM after the
// first pass's diffusion.
template <typename R>
size_t band_lds_bytes(int cap) {
    return (size_t)5 * cap * sizeof(R);
}

constexpr int kBandU = 4;   // slots per thread handled together: voxels base + u * kBlock + lane

// First pass on U slots of plane p's range [es, ee); all loads of the slots
// are issued before their use.
template <typename R, int U>
__device__ __forceinline__ void band_first(const StepBufs<R> &B, const Coef<R> &C, uint32_t base, uint32_t es,
                                           uint32_t ee, R *d1, R *dm) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t e[U], i[U], w[U];
    R m[4][U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        e[u] = base + (uint32_t)(u * kBlock) + lane;
        i[u] = e[u] < es ? es : (e[u] < ee ? e[u] : ee - 1u);
        w[u] = packed_words<true>(B.pk, i[u]).a;
    }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int s = 0; s < 4; s++) m[s][u] = at(B.src[s], i[u]);   // CO2 does not enter the DOM
    R g[U][6];
#pragma unroll
    for (int u = 0; u < U; u++) {
        uint32_t j[6];
        packed_decode<true>(B.pk, i[u], PackedWords{w[u], 0u}, j);
#pragma unroll
        for (int k = 0; k < 6; k++) g[u][k] = at(B.src[1], j[k]);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        R x1 = m[0][u], x2 = m[1][u], x3 = m[2][u], x4 = m[3][u], x5 = R(0);
        R d[6];
#pragma unroll
        for (int k = 0; k < 6; k++) d[k] = g[u][k] - x2;
        x2 = x2 + C.a[1] * (((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]));
        const bool act = e[u] >= es && e[u] < ee;
        if (act) dm[e[u] - es] = x2;
        transform_alg<false>(C, x1, x2, x3, x4, x5);
        if (act) d1[e[u] - es] = x2;
    }
}

// Second pass on U slots of the band range [bs, be) of plane q: the pools
// are read again and the first pass's transformation recomputed from its
// diffused DOM; the neighbours' first-pass DOM comes from LDS.  In two
// parts, so that the loads can be issued before the first pass of the same
// marching step and their latency overlaps it.
template <typename R, int U>
struct BandSecond {
    uint32_t e[U], i[U], w[U];
    R m1[U], m3[U], m4[U], m5[U];
};

template <typename R, int U>
__device__ __forceinline__ void band_second_load(const StepBufs<R> &B, uint32_t base, uint32_t bs, uint32_t be,
                                                 BandSecond<R, U> &L) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (int u = 0; u < U; u++) {
        L.e[u] = base + (uint32_t)(u * kBlock) + lane;
        L.i[u] = L.e[u] < bs ? bs : (L.e[u] < be ? L.e[u] : be - 1u);
        L.w[u] = packed_words<true>(B.pk, L.i[u]).a;
        L.m1[u] = at(B.src[0], L.i[u]);
        L.m3[u] = at(B.src[2], L.i[u]);
        L.m4[u] = at(B.src[3], L.i[u]);
        L.m5[u] = at(B.src[4], L.i[u]);
    }
}

template <typename R, int U>
__device__ __forceinline__ void band_second_finish(const StepBufs<R> &B, const Coef<R> &C, uint32_t base, uint32_t bs,
                                                   uint32_t be, uint32_t es, uint32_t esm, uint32_t esp, const R *d1m,
                                                   const R *d1c, const R *d1p, const R *dm, const BandSecond<R, U> &L) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        if (base + (uint32_t)(u * kBlock) >= be) break;   // uniform over the wave
        const uint32_t i = L.i[u];
        R x1 = L.m1[u], x2 = dm[i - es], x3 = L.m3[u], x4 = L.m4[u], x5 = L.m5[u];
        transform_alg<false>(C, x1, x2, x3, x4, x5);   // the first pass's output
        uint32_t j[6];
        packed_decode<true>(B.pk, i, PackedWords{L.w[u], 0u}, j);
        R g[6];
#pragma unroll
        for (int k = 0; k < 4; k++) g[k] = d1c[j[k] - es];   // same plane (absent: i itself)
        g[4] = j[4] == i ? x2 : d1m[j[4] - esm];
        g[5] = j[5] == i ? x2 : d1p[j[5] - esp];
        R d[6];
#pragma unroll
        for (int k = 0; k < 6; k++) d[k] = g[k] - x2;
        x2 = x2 + C.a[1] * (((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]));
        transform_alg<false>(C, x1, x2, x3, x4, x5);
        if (L.e[u] >= bs && L.e[u] < be) {
            at(B.dst[0], i) = x1;
            at(B.dst[1], i) = x2;
            at(B.dst[2], i) = x3;
            at(B.dst[3], i) = x4;
            at(B.dst[4], i) = x5;
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_band2(StepBufs<R> B, Coef<R> C, BandGeom G,
                                                  const int32_t *__restrict__ rs) {
    extern __shared__ __align__(16) unsigned char band_lds[];
    R *dom1 = reinterpret_cast<R *>(band_lds);
    R *dmid = dom1 + 3 * G.cap;
    const int band = (int)(blockIdx.x % (unsigned)G.nbands), chunk = (int)(blockIdx.x / (unsigned)G.nbands);
    const int y0 = band * G.H, y1 = min(y0 + G.H, G.ny);
    const int ey0 = max(y0 - 1, 0), ey1 = min(y1 + 1, G.ny);
    const int z0 = chunk * G.Z, z1 = min(z0 + G.Z, G.nz);
    const uint32_t wave = threadIdx.x >> 6;
    constexpr uint32_t kStep = (uint32_t)(kBandU * kBlock);
    for (int p = z0 - 1; p <= z1; p++) {
        // the second pass of this step works on plane q = p - 1, band rows:
        // its first slots' pools and codes are loaded before the first pass
        const int q = p - 1;
        const int64_t rq = (int64_t)q * G.ny;
        const bool has_q = q >= z0 && q < z1;
        const uint32_t qbs = has_q ? (uint32_t)rs[rq + y0] : 0u, qbe = has_q ? (uint32_t)rs[rq + y1] : 0u;
        const uint32_t qbase = (qbs & ~63u) + wave * 64u;
        BandSecond<R, kBandU> L2;
        if (qbs < qbe && qbase < qbe) band_second_load<R, kBandU>(B, qbase, qbs, qbe, L2);
        // first pass on plane p, rows ey0 .. ey1 - 1 (waves start on 64-voxel
        // groups: the relative codes' bases are per group)
        const bool has_p = p >= 0 && p < G.nz;
        const int64_t rp = (int64_t)p * G.ny;
        const uint32_t es = has_p ? (uint32_t)rs[rp + ey0] : 0u, ee = has_p ? (uint32_t)rs[rp + ey1] : 0u;
        if (es < ee) {   // plane p exists and its rows hold voxels
            R *d1 = dom1 + ((p + 3) % 3) * G.cap, *dm = dmid + ((p + 2) % 2) * G.cap;
            for (uint32_t base = (es & ~63u) + wave * 64u; base < ee; base += kStep)
                band_first<R, kBandU>(B, C, base, es, ee, d1, dm);
        }
        lds_barrier();
        // second pass on plane q, band rows
        if (qbs < qbe) {   // plane q is the block's and its band rows hold voxels
            const uint32_t qes = (uint32_t)rs[rq + ey0];
            const uint32_t esm = q > 0 ? (uint32_t)rs[rq - G.ny + ey0] : 0u;
            const uint32_t esp = q + 1 < G.nz ? (uint32_t)rs[rq + G.ny + ey0] : 0u;
            const R *d1m = dom1 + ((q + 2) % 3) * G.cap, *d1c = dom1 + ((q + 3) % 3) * G.cap,
                    *d1p = dom1 + ((q + 4) % 3) * G.cap, *dmq = dmid + ((q + 2) % 2) * G.cap;
            if (qbase < qbe) band_second_finish<R, kBandU>(B, C, qbase, qbs, qbe, qes, esm, esp, d1m, d1c, d1p, dmq, L2);
            for (uint32_t base = qbase + kStep; base < qbe; base += kStep) {
                BandSecond<R, kBandU> L;
                band_second_load<R, kBandU>(B, base, qbs, qbe, L);
                band_second_finish<R, kBandU>(B, C, base, qbs, qbe, qes, esm, esp, d1m, d1c, d1p, dmq, L);
            }
        }
        lds_barrier();
    }
}

template <int MODE, int MOB, int TOT>
int launch_c(vg_sim *h, const CompBufs &B, const Coef<double> &C, hipStream_t s) {
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    hipLaunchKernelGGL((k_step_c<MODE, MOB, TOT>), dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, B, C, pc, part_of(h));
    return launch_status("k_step_c");
}

template <int MODE, int MOB>
int pick_tot_c(vg_sim *h, int tot, const CompBufs &B, const Coef<double> &C, hipStream_t s) {
    switch (tot) {
        case TOT_NONE: return launch_c<MODE, MOB, TOT_NONE>(h, B, C, s);
        case TOT_IN: return launch_c<MODE, MOB, TOT_IN>(h, B, C, s);
        case TOT_MID: return launch_c<MODE, MOB, TOT_MID>(h, B, C, s);
        default: return launch_c<MODE, MOB, TOT_OUT>(h, B, C, s);
    }
}

// A pass on compensated fields: the same buffer rotation as dispatch<R>, for
// the float parts and the compensation words alike.
int dispatch_c(vg_sim *h, int mode, int tot, double dt_t, double dt_d, hipStream_t s) {
    CompBufs B;
    B.nbr = h->nbr;
    B.rcode = h->rcode;
    B.pk = packed_of(h);
    B.ns = use_relative(h) ? 1 : (use_offsets(h) ? 2 : 0);
    B.n = h->n;
    const int mob = h->mobile_mode();
    for (int p = 0; p < VG_NPOOL; p++) {
        const bool mob_p = mob == 2 || p == 1;
        const int64_t off = (int64_t)p * h->n;
        float *here = (float *)h->fields + off;
        int16_t *here_lo = h->lo + off;
        float *there = nullptr;
        int16_t *there_lo = nullptr;
        if (mob_p) {
            there = (float *)h->alt + (mob == 2 ? off : 0);
            there_lo = h->lo_alt + (mob == 2 ? off : 0);
        }
        const bool flip = mob_p && h->cur;
        float *cur = flip ? there : here, *oth = flip ? here : there;
        int16_t *cur_lo = flip ? there_lo : here_lo, *oth_lo = flip ? here_lo : there_lo;
        const bool moves = mob_p && (mode == MODE_D || mode == MODE_DT);
        B.src[p] = cur;
        B.slo[p] = cur_lo;
        B.dst[p] = moves ? oth : cur;
        B.dlo[p] = moves ? oth_lo : cur_lo;
    }
    const Coef<double> C = make_coef2<double>(h, dt_t, dt_d);
    int rc;
    if (mode == MODE_T) rc = pick_tot_c<MODE_T, 1>(h, tot, B, C, s);
    else if (mode == MODE_NONE) rc = launch_c<MODE_NONE, 1, TOT_IN>(h, B, C, s);
    else if (mode == MODE_D) rc = mob == 2 ? pick_tot_c<MODE_D, 2>(h, tot, B, C, s) : pick_tot_c<MODE_D, 1>(h, tot, B, C, s);
    else rc = mob == 2 ? pick_tot_c<MODE_DT, 2>(h, tot, B, C, s) : pick_tot_c<MODE_DT, 1>(h, tot, B, C, s);
    if (rc) return rc;
    if (mode == MODE_D || mode == MODE_DT) h->cur ^= 1;
    return VG_OK;
}

// State conversions: x [5][n] of type X into the bound fields, or back.
template <typename X, typename F>
__global__ __launch_bounds__(kBlock) void k_load_state(const X *__restrict__ x, int64_t m, F f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) f.put(i, (double)x[i]);
}

template <typename X, typename F>
__global__ __launch_bounds__(kBlock) void k_store_state(X *__restrict__ x, int64_t m, F f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) x[i] = (X)f.get(i);
}

// float parts of compensated fields as float (the exact values, no rounding)
__global__ __launch_bounds__(kBlock) void k_store_hi(float *__restrict__ x, int64_t m, const float *__restrict__ hi) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) x[i] = hi[i];
}

template <typename R>
int dispatch(vg_sim *h, int mode, int tot, double dt_t, double dt_d, hipStream_t s) {
    StepBufs<R> B = graph_bufs<R>(h);
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
    const int rc = dispatch_bufs<R>(h, mode, tot, dt_t, dt_d, B, s);
    if (rc) return rc;
    if (mode == MODE_D || mode == MODE_DT) h->cur ^= 1;
    return VG_OK;
}

}  // namespace

// Neighbour source: an explicit choice, else packed offsets when they fit,
// else the rank index when there is one, else the table.
PackedNbr packed_of(const vg_sim *h) {
    PackedNbr P;
    P.rel_w = h->rel_w;
    P.rel_base = h->rel_base;
    P.rl = h->rel_layout;
    P.off_m = h->off_m;
    P.off_p = h->off_p;
    P.dl = h->off_layout;
    return P;
}

bool use_relative(const vg_sim *h) {
    return h->rel_ok &&
           (h->kernel == VG_KERNEL_AUTO || h->kernel == VG_KERNEL_RELATIVE || h->kernel == VG_KERNEL_BAND);
}

bool band_geometry(const vg_sim *h) {
    return (h->features & VG_FEAT_BAND) && h->nseg == 1 && h->vox != nullptr && h->brick == 0 &&
           h->periodic == 0 && h->n > 0 && h->prec != VG_F32C;
}

// AUTO takes the band kernel for FP32 fields when its chunks are long enough
// (in FP64 its LDS budget allows only narrow bands: slower than single
// passes).
bool use_band(const vg_sim *h) {
    return h->band_ok && h->rel_ok && h->prec != VG_F32C &&
           (h->kernel == VG_KERNEL_BAND || (h->kernel == VG_KERNEL_AUTO && h->prec == VG_F32 && h->band_auto)) &&
           !h->mobile_all && h->rcode == nullptr && h->params.sequential == 0;
}

// Row index, band height and chunk length.  The band height is the largest
// of 8, 6, 4, 2 rows whose widest range of a plane's band and neighbour rows
// fits a block's LDS budget (40 KiB); the chunks are sized so that every
// block is resident at once.  Measured on the 512^3 FP32 step (a pass pair
// in one launch vs two single passes): 8 rows 5.7 % faster, 6 rows equal,
// 4 rows 23 % slower, 12 rows 3.5 % faster, 10 and 16 rows no faster.
int build_band(vg_sim *h, hipStream_t s) {
    h->band_ok = false;
    h->band_auto = false;
    if (!band_geometry(h) || !h->rel_ok) return VG_OK;
    const int64_t nrows = (int64_t)h->nz * h->ny;
    hipLaunchKernelGGL(k_band_rows, dim3((unsigned)((nrows + 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, h->vox,
                       h->n, h->nx, nrows, h->band_rs);
    int rc = launch_status("k_band_rows");
    if (rc) return rc;
    std::vector<int32_t> rs((size_t)nrows + 1);
    if ((rc = hip_status(hipMemcpyAsync(rs.data(), h->band_rs, sizeof(int32_t) * rs.size(), hipMemcpyDeviceToHost, s),
                         "band rows"))) return rc;
    if ((rc = hip_status(hipStreamSynchronize(s), "band rows"))) return rc;
    if (rs[(size_t)nrows] != h->n) { set_error("row index does not cover the compact list"); return VG_EINVAL; }
    const size_t lds_max = 40 * 1024;
    for (int H : {8, 6, 4, 2}) {
        int64_t cap = 1;
        for (int z = 0; z < h->nz; z++)
            for (int y0 = 0; y0 < h->ny; y0 += H) {
                const size_t r = (size_t)z * h->ny;
                const int y1 = y0 + H < h->ny ? y0 + H : h->ny;
                const int ey0 = y0 > 0 ? y0 - 1 : 0, ey1 = y1 + 1 < h->ny ? y1 + 1 : h->ny;
                const int64_t c = (int64_t)rs[r + ey1] - rs[r + ey0];
                if (c > cap) cap = c;
            }
        const size_t lds = h->prec == VG_F64 ? band_lds_bytes<double>((int)cap) : band_lds_bytes<float>((int)cap);
        if (lds > lds_max) continue;
        h->band_h = H;
        h->band_cap = (int)cap;
        h->band_nbands = (h->ny + H - 1) / H;
        // blocks resident at once (registers and this LDS size) on the device
        int per = 0, cus = 0, dev = 0;
        const void *kern = h->prec == VG_F64 ? (const void *)k_band2<double> : (const void *)k_band2<float>;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kBlock, lds) != hipSuccess || per < 1) {
            (void)hipGetLastError();
            per = 4;
            cus = 256;
        }
        const int resident = per * cus;
        int chunks = (int)((resident + h->band_nbands / 2) / h->band_nbands);
        if (chunks > (h->nz + 3) / 4) chunks = (h->nz + 3) / 4;
        if (chunks < 1) chunks = 1;

        h->band_z = (h->nz + chunks - 1) / chunks;
        h->band_nchunks = (h->nz + h->band_z - 1) / h->band_z;
        h->band_ok = true;
        // AUTO leaves chunks of fewer than 20 planes to single passes: their
        // two extra planes and the march's start cost more than the pass
        // pair saves (256^3: 7-plane chunks, 47 % slower)
        h->band_auto = h->band_z >= 20;
        return VG_OK;
    }
    return VG_OK;
}

namespace {
template <typename R>
int band_quad(vg_sim *h, double dt, hipStream_t s) {
    const Coef<R> C = make_coef2<R>(h, dt, dt);
    BandGeom G{h->ny, h->nz, h->band_h, h->band_z, h->band_nbands, h->band_cap};
    StepBufs<R> A = graph_bufs<R>(h), Bk = graph_bufs<R>(h);
    R *canon = (R *)h->fields;
    R *mid = (R *)h->band_alt;
    for (int p = 0; p < VG_NPOOL; p++) {
        R *cur = (p == 1 && h->cur) ? (R *)h->alt : canon + (int64_t)p * h->n;
        A.src[p] = cur;
        A.dst[p] = mid + (int64_t)p * h->n;
        Bk.src[p] = mid + (int64_t)p * h->n;
        Bk.dst[p] = cur;
    }
    const unsigned grid = (unsigned)(h->band_nbands * h->band_nchunks);
    const size_t lds = band_lds_bytes<R>(h->band_cap);
    hipLaunchKernelGGL(k_band2<R>, dim3(grid), dim3(kBlock), lds, s, A, C, G, h->band_rs);
    int rc = launch_status("k_band2");
    if (rc) return rc;
    hipLaunchKernelGGL(k_band2<R>, dim3(grid), dim3(kBlock), lds, s, Bk, C, G, h->band_rs);
    return launch_status("k_band2");
}
}  // namespace

// Four fused passes as two band launches (into the intermediate field set
// and back), so every pool ends where it started.
int launch_band_quad(vg_sim *h, double dt, hipStream_t s) {
    if (h->prec == VG_F64) return band_quad<double>(h, dt, s);
    return band_quad<float>(h, dt, s);
}

bool use_offsets(const vg_sim *h) {
    if (h->kernel == VG_KERNEL_OFFSET) return h->off_ok;
    return h->off_ok && h->kernel == VG_KERNEL_AUTO && !h->rel_ok;
}

bool use_rank(const vg_sim *h) {
    const bool ok = h->rank != nullptr && h->geo != nullptr && h->nseg == 1 && h->prec != VG_F32C;
    if (h->kernel == VG_KERNEL_RANK) return ok;
    return ok && h->kernel == VG_KERNEL_AUTO && !h->off_ok && !h->rel_ok;
}

static uint32_t bit_width(uint32_t v) {
    uint32_t b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

// Measures the neighbour distances and, when they fit, writes the packed
// offsets.  Synchronises the stream (the layout is chosen on the host).
int build_offsets(vg_sim *h, hipStream_t s) {
    h->off_ok = false;
    h->rel_ok = false;
    if (h->n == 0 || !h->off_m || !h->rel_w || !h->nbr) return VG_OK;
    int rc;
    if ((rc = hip_status(hipMemsetAsync(h->off_stat, 0, 8 * sizeof(uint32_t), s), "clear offset statistics")))
        return rc;
    const unsigned blocks = (unsigned)((h->n + kBlock - 1) / kBlock);
    const unsigned stat_blocks = blocks < 2048u ? blocks : 2048u;
    hipLaunchKernelGGL(k_neighbour_stat, dim3(stat_blocks), dim3(kBlock), 0, s, h->nbr, h->n, h->rel_base,
                       h->off_stat);
    if ((rc = launch_status("k_neighbour_stat"))) return rc;
    uint32_t st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if ((rc = hip_status(hipMemcpyAsync(st, h->off_stat, sizeof(st), hipMemcpyDeviceToHost, s), "read offsets")))
        return rc;
    if ((rc = hip_status(hipStreamSynchronize(s), "synchronise"))) return rc;
    const uint32_t bx = bit_width(st[0]), by = bit_width(st[1]), bz = bit_width(st[2]);
    // periodic wrap or byte offsets beyond 32 bits: neither packing
    if (st[3] || (uint64_t)h->n * h->elem() >= ((uint64_t)1 << 32)) return VG_OK;
    auto mask = [](uint32_t b) { return b >= 32 ? 0xffffffffu : (1u << b) - 1u; };
    // relative codes: widths from the largest spread + 1 per axis
    const uint32_t cx = bit_width(st[4]), cy = bit_width(st[5]), cz = bit_width(st[6]);
    if (2 * (cx + cy + cz) <= 32) {
        RLayout R;
        const uint32_t width[6] = {cx, cx, cy, cy, cz, cz};
        const uint32_t order[6] = {4, 5, 2, 3, 0, 1};      // z-, z+, y-, y+, x-, x+ from bit 0 up
        uint32_t at_bit = 0;
        for (int q = 0; q < 6; q++) {
            const uint32_t k = order[q];
            R.sh[k] = at_bit & 31u;                         // a zero-width field's shift is never used
            R.mk[k] = mask(width[k]);
            at_bit += width[k];
        }
        hipLaunchKernelGGL(k_rel_pack, dim3(blocks), dim3(kBlock), 0, s, h->nbr, h->n, h->rel_base, R, h->rel_w);
        if ((rc = launch_status("k_rel_pack"))) return rc;
        h->rel_layout = R;
        h->rel_ok = true;
    }
    // neighbours too far apart: no packed offsets
    if (bx + by + bz > 32) return VG_OK;
    DLayout L;
    L.bz = bz & 31u;                     // an empty field's shift is never used
    L.by = by;
    L.sx = (bz + by) & 31u;
    L.mz = mask(bz);
    L.my = mask(by);
    L.mx = mask(bx);
    hipLaunchKernelGGL(k_offsets, dim3(blocks), dim3(kBlock), 0, s, h->nbr, h->n, L, h->off_m, h->off_p);
    if ((rc = launch_status("k_offsets"))) return rc;
    h->off_layout = L;
    h->off_ok = true;
    return VG_OK;
}

int launch_geometry(vg_sim *h, hipStream_t s) {
    if (!h->rank || h->n == 0) return VG_OK;
    hipLaunchKernelGGL(k_geometry, dim3((unsigned)((h->n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, h->vox, h->n,
                       make_rgeom(h), h->geo);
    return launch_status("k_geometry");
}

int launch_pass2(vg_sim *h, int mode, int tot, double dt_t, double dt_d, hipStream_t s) {
    if (h->n == 0) return VG_OK;
    if (h->prec == VG_F32C) return dispatch_c(h, mode, tot, dt_t, dt_d, s);
    if (h->prec == VG_F64) return dispatch<double>(h, mode, tot, dt_t, dt_d, s);
    return dispatch<float>(h, mode, tot, dt_t, dt_d, s);
}

int launch_pass(vg_sim *h, int mode, int tot, double dt, hipStream_t s) {
    return launch_pass2(h, mode, tot, dt, dt, s);
}

// A pass between explicit buffers (pool s read from src[s], written to
// dst[s]); used by the adjoint's forward recording.  xdom: see StepBufs
// (fused passes, only DOM diffusing; a row the pass does not read).
int launch_pass_bufs(vg_sim *h, int mode, int tot, double dt, const void *const src[VG_NPOOL],
                     void *const dst[VG_NPOOL], hipStream_t s, void *xdom) {
    if (h->n == 0) return VG_OK;
    if (h->prec == VG_F64) {
        StepBufs<double> B = graph_bufs<double>(h);
        for (int p = 0; p < VG_NPOOL; p++) { B.src[p] = (const double *)src[p]; B.dst[p] = (double *)dst[p]; }
        B.xdom = (double *)xdom;
        return dispatch_bufs<double>(h, mode, tot, dt, dt, B, s);
    }
    StepBufs<float> B = graph_bufs<float>(h);
    for (int p = 0; p < VG_NPOOL; p++) { B.src[p] = (const float *)src[p]; B.dst[p] = (float *)dst[p]; }
    B.xdom = (float *)xdom;
    return dispatch_bufs<float>(h, mode, tot, dt, dt, B, s);
}

int launch_totals_finalize(vg_sim *h, double *out_rows, int rows, hipStream_t s) {
    if (h->nseg == 0 || h->n == 0 || rows <= 0) return VG_OK;
    const int64_t part_stride = (int64_t)VG_NPOOL * h->npieces, out_stride = (int64_t)h->nseg * 6;
    const int64_t chunk_stride = (int64_t)VG_NPOOL * h->nchunks;
    if (h->max_seg_pieces <= kDirectPieces) {
        hipLaunchKernelGGL(k_tot_direct, dim3((unsigned)h->nseg, (unsigned)rows), dim3(kBlock), 0, s, h->part,
                           h->seg_first, out_rows, part_stride, out_stride);
        return launch_status("k_tot_direct");
    }
    hipLaunchKernelGGL(k_tot_chunks, dim3((unsigned)h->nchunks, (unsigned)rows), dim3(kBlock), 0, s, h->part,
                       h->chunk_first, h->chunk_part, part_stride, chunk_stride);
    int rc = launch_status("k_tot_chunks");
    if (rc) return rc;
    hipLaunchKernelGGL(k_tot_segments, dim3((unsigned)h->nseg, (unsigned)rows), dim3(kBlock), 0, s, h->chunk_part,
                       h->seg_chunk, out_rows, chunk_stride, out_stride);
    return launch_status("k_tot_segments");
}

int launch_load_state(vg_sim *h, const void *x, int xprec, hipStream_t s) {
    const int64_t m = (int64_t)VG_NPOOL * h->n;
    if (m == 0) return VG_OK;
    const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
    if (h->prec == VG_F32C) {
        const CompAcc f{(float *)h->fields, h->lo};
        if (xprec == VG_F64) hipLaunchKernelGGL((k_load_state<double, CompAcc>), grid, dim3(kBlock), 0, s, (const double *)x, m, f);
        else hipLaunchKernelGGL((k_load_state<float, CompAcc>), grid, dim3(kBlock), 0, s, (const float *)x, m, f);
    } else if (h->prec == VG_F64) {
        const PlainAcc<double> f{(double *)h->fields};
        if (xprec == VG_F64) hipLaunchKernelGGL((k_load_state<double, PlainAcc<double>>), grid, dim3(kBlock), 0, s, (const double *)x, m, f);
        else hipLaunchKernelGGL((k_load_state<float, PlainAcc<double>>), grid, dim3(kBlock), 0, s, (const float *)x, m, f);
    } else {
        const PlainAcc<float> f{(float *)h->fields};
        if (xprec == VG_F64) hipLaunchKernelGGL((k_load_state<double, PlainAcc<float>>), grid, dim3(kBlock), 0, s, (const double *)x, m, f);
        else hipLaunchKernelGGL((k_load_state<float, PlainAcc<float>>), grid, dim3(kBlock), 0, s, (const float *)x, m, f);
    }
    return launch_status("k_load_state");
}

int launch_store_state(vg_sim *h, void *x, int xprec, hipStream_t s) {
    const int64_t m = (int64_t)VG_NPOOL * h->n;
    if (m == 0) return VG_OK;
    const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
    if (h->prec == VG_F32C) {
        const CompAcc f{(float *)h->fields, h->lo};
        if (xprec == VG_F64) hipLaunchKernelGGL((k_store_state<double, CompAcc>), grid, dim3(kBlock), 0, s, (double *)x, m, f);
        else hipLaunchKernelGGL(k_store_hi, grid, dim3(kBlock), 0, s, (float *)x, m, (const float *)h->fields);
    } else if (h->prec == VG_F64) {
        const PlainAcc<double> f{(double *)h->fields};
        if (xprec == VG_F64) hipLaunchKernelGGL((k_store_state<double, PlainAcc<double>>), grid, dim3(kBlock), 0, s, (double *)x, m, f);
        else hipLaunchKernelGGL((k_store_state<float, PlainAcc<double>>), grid, dim3(kBlock), 0, s, (float *)x, m, f);
    } else {
        const PlainAcc<float> f{(float *)h->fields};
        if (xprec == VG_F64) hipLaunchKernelGGL((k_store_state<double, PlainAcc<float>>), grid, dim3(kBlock), 0, s, (double *)x, m, f);
        else hipLaunchKernelGGL((k_store_state<float, PlainAcc<float>>), grid, dim3(kBlock), 0, s, (float *)x, m, f);
    }
    return launch_status("k_store_state");
}

// Mobile pools that currently live in the alt buffer are copied back to the
// caller's field buffer, so the fields hold the state between calls.
int restore_canonical(vg_sim *h, hipStream_t s) {
    if (!h->cur) return VG_OK;
    const size_t e = h->elem();
    const int mob = h->mobile_mode();
    int rc;
    if (h->prec == VG_F32C) {
        const size_t cnt = (mob == 2 ? VG_NPOOL : 1) * (size_t)h->n;
        const size_t at0 = mob == 2 ? 0 : (size_t)h->n;
        if ((rc = hip_status(hipMemcpyAsync(h->lo + at0, h->lo_alt, sizeof(int16_t) * cnt, hipMemcpyDeviceToDevice, s),
                             "restore compensation words")))
            return rc;
    }
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
