// Discrete adjoint of the explicit time loop in the paper's order
// (x^(k+1) = D(T(x^k)): transformation of Appendix A Algorithm 1, then
// Scheme 1 diffusion).  Reverse-mode derivative of exactly the arithmetic of
// the forward kernels, for a loss on the per-volume pool totals.
//
// Forward recording stores, per step of a checkpoint segment, the state the
// reverse pass needs: x^k0 for the first step and z^(k-1) = T(x^(k-1)) for the
// others (the fused forward pass produces z; x^k = D(z^(k-1)) is recomputed
// in the adjoint kernel with the forward's own arithmetic, so the stored
// bytes per step equal one field set).
//
// One reverse step is one fused pass per voxel:
//   x   = D(z)_i (or the stored x) and u = T(x) locally,
//   ubar = Q_w lambda (Q_w symmetric, so its transpose is the same gather),
//   dL/da_s += u_s,i * sum_j w_ij (lambda_j - lambda_i),
//   dL/dc_r += a_s u_s,i (lambda_j - lambda_i) (1/2 to each endpoint region),
//   lambda^k = J_T(x)^T ubar + seed,
// with FP64 per-thread accumulators reduced per block in a fixed order.
//
// CO2 neither diffuses (when only DOM does) nor feeds another pool, so its
// adjoint is the same at every voxel of a volume whenever it starts so (the
// seeds of the totals are per volume): then the sweep carries it as one
// value per volume (CO2U) and reads and writes 8 bytes less per voxel and
// step; the per-voxel array is filled once at the end.
#include <vector>

#include "vg_internal.h"

#pragma clang fp contract(off)

namespace vg {
namespace {

constexpr int kG = VG_NGRAD;

// The clamps of both directions are written as selects between values that
// are all computed (no branches): the selected values are the ones the
// branches would produce, so the results are the same, and a wave does not
// split on the voxels' clamp cases.
template <typename R>
__device__ __forceinline__ void transform_fwd(const Coef<R> &C, R &m1, R &m2, R &m3, R &m4, R &m5) {
    R uptake = C.v_dom * m2 / (C.k_dom + m2) * m1 * C.dt;
    uptake = uptake > m2 ? m2 : uptake;
    const R resp0 = C.rho * m1 * C.dt, morta0 = C.mu * m1 * C.dt;
    const bool over = resp0 + morta0 > m1;   // respiration and mortality would take more than there is
    const bool all = over && morta0 > m1;    // mortality alone would
    const R morta = all ? m1 : morta0;
    const R resp = all ? R(0) : (over ? m1 - morta0 : resp0);
    R turn_p4 = C.v_p4 * m4 * C.dt;
    turn_p4 = turn_p4 > m4 ? m4 : turn_p4;
    R turn_som = C.v_som * m3 * C.dt;
    turn_som = turn_som > m3 ? m3 : turn_som;
    const R n1 = m1 + (uptake - morta - resp);
    R n2, n3, n4;
    if (C.route == 0) {
        n2 = m2 + (C.beta * morta - uptake + turn_p4 + turn_som);
        n3 = m3 + (C.omb * morta - turn_som);
        n4 = m4 - turn_p4;
    } else {
        n2 = m2 + (R(0) - uptake + turn_p4 + turn_som);
        n3 = m3 + (R(0) - turn_som);
        n4 = m4 + (morta - turn_p4);
    }
    m1 = n1; m2 = n2; m3 = n3; m4 = n4; m5 = m5 + resp;
}

// Reverse of the transformation at pre-step masses x (clamp cases re-taken
// from x).  In: ybar = adjoint of T's outputs.  Out: adjoint of its inputs.
// The rate derivatives accumulate into g[0..6] = v_DOM, K_DOM, rho, mu, beta,
// v_SOM, v_P4 (FP64 sums of the voxel's terms, each formed in the field
// type; a clamped case adds +0).
template <typename R>
__device__ __forceinline__ void transform_rev(const Coef<R> &C, const R (&x)[VG_NPOOL], R (&bar)[VG_NPOOL],
                                              double *g) {
    const R m1 = x[0], m2 = x[1], m3 = x[2], m4 = x[3];
    const R dt = C.dt;
    const R den = C.k_dom + m2;
    const R up_raw = C.v_dom * m2 / den * m1 * dt;
    const bool up_clamp = up_raw > m2;
    const R resp0 = C.rho * m1 * dt, morta0 = C.mu * m1 * dt;
    // 0 free, 1 all biomass dies, 2 respiration takes the rest
    const bool over = resp0 + morta0 > m1;
    const bool rm1 = over && morta0 > m1, rm2 = over && !rm1;
    const R morta = rm1 ? m1 : morta0;
    const bool p4_clamp = C.v_p4 * m4 * dt > m4;
    const bool som_clamp = C.v_som * m3 * dt > m3;

    const R y1 = bar[0], y2 = bar[1], y3 = bar[2], y4 = bar[3], y5 = bar[4];
    R b1 = y1, b2 = y2, b3 = y3, b4 = y4;
    const R b5 = y5;
    const R upb = y1 - y2;
    R mortb;
    if (C.route == 0) {
        mortb = -y1 + C.beta * y2 + C.omb * y3;
        g[4] += (double)(morta * (y2 - y3));
    } else {
        mortb = -y1 + y4;
    }
    const R respb = -y1 + y5;
    const R p4b = y2 - y4;
    const R somb = y2 - y3;
    // uptake: one division; d(uptake)/d(m2) = v m1 dt K / den^2 and
    // d(uptake)/dK = -v m1 dt m2 / den^2 from 1/den
    {
        const R inv = R(1) / den;
        const R gm = m2 * inv;
        const R vmd = C.v_dom * m1 * dt * inv;
        const R t1 = upb * C.v_dom * gm * dt;
        const R t2 = upb * vmd * (C.k_dom * inv);
        b1 += up_clamp ? R(0) : t1;
        b2 += up_clamp ? upb : t2;
        g[0] += up_clamp ? 0.0 : (double)(upb * (gm * m1 * dt));
        g[1] -= up_clamp ? 0.0 : (double)(upb * (vmd * gm));
    }
    {
        const R mt = mortb - respb;
        const R f0 = respb * C.rho * dt + mortb * C.mu * dt;
        const R f2 = respb + mt * C.mu * dt;
        b1 += rm1 ? mortb : (rm2 ? f2 : f0);
        const bool neither = !over;   // neither respiration nor mortality clamped
        g[2] += neither ? (double)(respb * (m1 * dt)) : 0.0;
        g[3] += rm1 ? 0.0 : (double)((rm2 ? mt : mortb) * (m1 * dt));
    }
    b3 += som_clamp ? somb : somb * C.v_som * dt;
    g[5] += som_clamp ? 0.0 : (double)(somb * (m3 * dt));
    b4 += p4_clamp ? p4b : p4b * C.v_p4 * dt;
    g[6] += p4_clamp ? 0.0 : (double)(p4b * (m4 * dt));
    bar[0] = b1; bar[1] = b2; bar[2] = b3; bar[3] = b4; bar[4] = b5;
}

template <typename R>
struct AdjBufs {
    const int32_t *nbr = nullptr;
    const uint16_t *rcode = nullptr;
    PackedNbr pk;                // packed neighbour sources (when built)
    const R *st = nullptr;       // stored state of this step, pool s at st + s*n
    int co2_row = 4;             // the row of CO2 (a kept-DOM recording has none: never read then)
    const R *lin = nullptr;      // lambda^(k+1)
    R *lout = nullptr;           // lambda^k
    const double *seed = nullptr;   // [nseg][5] for this step
    const R *co2 = nullptr;      // [nseg] CO2 adjoint lambda^(k+1) per volume (CO2U)
    R *co2_next = nullptr;       // [nseg] lambda^k's, written by block 0 (CO2U; the other buffer)
    int nseg = 0;
    int64_t n = 0, ntiles = 0;
};

template <int MOB>
__device__ __forceinline__ constexpr bool mobile(int s) {
    return MOB == 2 || (MOB == 1 && s == 1);
}

// Pools whose adjoint differences a reverse step takes: the diffusing ones,
// and with DALL the others too (for dL/dD_s only); never a uniform CO2
// adjoint (its differences are all zero).
template <int MOB, bool DALL, bool CO2U>
__device__ __forceinline__ constexpr bool adj_differenced(int s) {
    return (DALL || mobile<MOB>(s)) && !(CO2U && s == 4);
}

// Neighbour sources of the adjoint kernel (the forward's): the 6-slot table
// with 64-bit indexing, or a packed source with 32-bit indexing.
enum { NS_TABLE = 0, NS_REL = 1, NS_OFF = 2 };

template <int NS>
struct AdjIndex {
    using T = uint32_t;
};
template <>
struct AdjIndex<NS_TABLE> {
    using T = int64_t;
};

template <typename T>
__device__ __forceinline__ const T &elem(const T *b, uint32_t i) {
    return at(b, i);
}
template <typename T>
__device__ __forceinline__ const T &elem(const T *b, int64_t i) {
    return b[i];
}
template <typename T>
__device__ __forceinline__ T &elem(T *b, uint32_t i) {
    return at(b, i);
}
template <typename T>
__device__ __forceinline__ T &elem(T *b, int64_t i) {
    return b[i];
}

// What a reverse step reads of the voxel itself: its stored state, lambda^(k+1)
// (CO2's only when it is not uniform), its neighbour words (the table's six
// indices, or the packed words) and its region code.
template <typename R, int NS>
struct AdjOwn {
    R x[VG_NPOOL], li[VG_NPOOL];
    int32_t jt[NS == NS_TABLE ? 6 : 1];
    PackedWords W;
    uint32_t code;
};

// A load whose address is the same in every lane, through the constant
// address space: it becomes a scalar load even where the kernel's stores
// keep the compiler from proving that the word is read-only.
template <typename T>
__device__ __forceinline__ T uload(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// Loads o for voxel i (a valid index: the loads are not guarded, so that a
// wave issues the same memory instructions on every path).
template <typename R, int MOB, bool REG, int NS, bool DALL, bool CO2U>
__device__ __forceinline__ void adj_load_own(const AdjBufs<R> &A, const R *const *st, const R *const *lin,
                                             typename AdjIndex<NS>::T i, AdjOwn<R, NS> &o) {
    o.W = PackedWords{0, 0};
    o.code = 0;
    o.x[4] = o.li[4] = R(0);
    if constexpr (NS == NS_TABLE) {
#pragma unroll
        for (int k = 0; k < 6; k++) o.jt[k] = A.nbr[(int64_t)k * A.n + i];
    } else {
        o.jt[0] = -1;
        o.W = packed_words<NS == NS_REL>(A.pk, (uint32_t)i);
    }
#pragma unroll
    for (int s = 0; s < VG_NPOOL - 1; s++) o.x[s] = elem(st[s], i);
    // the CO2 state enters only dL/dD_CO2 (the transformation's derivative
    // does not depend on it): not read when that term is not computed
    if (!(MOB == 1 && (CO2U || !DALL))) o.x[4] = elem(st[4], i);
#pragma unroll
    for (int s = 0; s < VG_NPOOL - 1; s++) o.li[s] = elem(lin[s], i);
    if (!CO2U) o.li[4] = elem(lin[4], i);
    if (REG) o.code = elem(A.rcode, i);
}

// DALL: dL/da_s also for the pools that do not diffuse (their adjoints'
// neighbour differences are gathered only for that term).
template <typename R, int MOB, bool REG, bool FROM_X, int NS, bool DALL, bool CO2U>
__global__ __launch_bounds__(kBlock) void k_adj(AdjBufs<R> A, Coef<R> C, Pieces pc, double *__restrict__ part) {
    static_assert(!CO2U || MOB == 1, "a uniform CO2 adjoint needs CO2 not to diffuse");
    using I = typename AdjIndex<NS>::T;
    __shared__ double lds[kWaves * kG];
    __shared__ R cl[VG_NREG];
    // with region weights each thread keeps its dL/dc_r sums in LDS, region
    // major (conflict-free whatever region each lane adds to): the region of
    // a term depends on the voxel, so registers would need a select per
    // region and term
    __shared__ double creg[REG ? VG_NREG : 1][REG ? kBlock : 1];
    if (threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];
    if (REG) {
#pragma unroll
        for (int r = 0; r < VG_NREG; r++) creg[r][threadIdx.x] = 0.0;
    }
    __syncthreads();
    if (CO2U && blockIdx.x == 0) {
        // the uniform CO2 adjoint after this step: only the seed changes it,
        // with the per-voxel update's rounding, (R)((double)lambda + seed)
        for (int s = threadIdx.x; s < A.nseg; s += kBlock)
            A.co2_next[s] = (R)((double)A.co2[s] + A.seed[(int64_t)s * VG_NPOOL + 4]);
    }
    double g[kG];
#pragma unroll
    for (int q = 0; q < kG; q++) g[q] = 0.0;
    const int64_t n = A.n;
    // pool s of a field set at base + s * n
    const R *st[VG_NPOOL], *lin[VG_NPOOL];
    R *lout[VG_NPOOL];
#pragma unroll
    for (int s = 0; s < VG_NPOOL; s++) {
        st[s] = A.st + (int64_t)(s == 4 ? A.co2_row : s) * n;
        lin[s] = A.lin + (int64_t)s * n;
        lout[s] = A.lout + (int64_t)s * n;
    }

    // the seeds of this step's totals and the uniform CO2 adjoint of voxel
    // i64's volume, taken piece by piece over the pieces that overlap its
    // tile (uniform loads): the last piece that starts at or before the
    // voxel holds it
    auto volume_terms = [&](int64_t t, int64_t i64, double (&sd)[VG_NPOOL], R &lco2) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) sd[s] = 0.0;
        lco2 = R(0);
        const int32_t pf = uload(pc.piece_first + t), pl = uload(pc.piece_first + t + 1);
        for (int32_t p = pf; p < pl; p++) {
            const int32_t sg = uload(pc.piece_seg + p);
            const bool in = p == pf || i64 >= uload(pc.piece_lo + p);
            const double *sp = A.seed + (int64_t)sg * VG_NPOOL;
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) sd[s] = in ? uload(sp + s) : sd[s];
            if (CO2U) lco2 = in ? uload(A.co2 + sg) : lco2;
        }
    };
    // neighbour values of voxel i: the stored state of the diffusing pools
    // (to recompute D) and lambda^(k+1) of the pools whose differences are
    // taken
    auto gather = [&](const AdjOwn<R, NS> &o, I i, R (&zj)[VG_NPOOL][6], R (&lj)[VG_NPOOL][6]) {
        // neighbour indices (an absent neighbour is the voxel itself: every
        // difference of an absent slot is exactly +0)
        I j[6];
        if constexpr (NS == NS_TABLE) {
#pragma unroll
            for (int k = 0; k < 6; k++) j[k] = o.jt[k] >= 0 ? (I)o.jt[k] : i;
        } else {
            uint32_t jp[6];
            packed_decode<NS == NS_REL>(A.pk, (uint32_t)i, o.W, jp);
#pragma unroll
            for (int k = 0; k < 6; k++) j[k] = (I)jp[k];
        }
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            if (!FROM_X && mobile<MOB>(s)) {
#pragma unroll
                for (int k = 0; k < 6; k++) zj[s][k] = elem(st[s], j[k]);
            }
            if (adj_differenced<MOB, DALL, CO2U>(s)) {
#pragma unroll
                for (int k = 0; k < 6; k++) lj[s][k] = elem(lin[s], j[k]);
            }
        }
    };
    // the reverse step at voxel i from its own words and neighbour values
    auto work = [&](const AdjOwn<R, NS> &o, I i, const double (&sd)[VG_NPOOL], R lco2,
                    const R (&zj)[VG_NPOOL][6], const R (&lj)[VG_NPOOL][6]) {
        // forward state of this step and lambda^(k+1) of the voxel
        R x[VG_NPOOL], li[VG_NPOOL];
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            x[s] = o.x[s];
            li[s] = o.li[s];
        }
        if (CO2U) li[4] = lco2;
        R w[6];
        uint32_t code = 0, own = 0;
        if (REG) {
            code = o.code;
            own = code & 7u;
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const uint32_t other = own ^ (((code >> (3 + k)) & 1u) << (k >> 1));
                w[k] = R(0.5) * (cl[own] + cl[other]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 6; k++) w[k] = R(1);
        }
        // x^k = D(z) of the stored z, with the forward's arithmetic
        if (!FROM_X) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) {
                if (!mobile<MOB>(s)) continue;
                const R xi = x[s];
                R d[6];
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const R diff = zj[s][k] - xi;
                    d[k] = REG ? w[k] * diff : diff;
                }
                x[s] = xi + C.a[s] * (((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]));
            }
        }
        R u[VG_NPOOL] = {x[0], x[1], x[2], x[3], x[4]};
        transform_fwd(C, u[0], u[1], u[2], u[3], u[4]);

        // adjoint of the diffusion half: ubar = Q_w lambda; parameter terms
        R bar[VG_NPOOL];
        double own_c = 0.0, cross_c[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            if (!adj_differenced<MOB, DALL, CO2U>(s)) {
                // (a uniform CO2 adjoint has no neighbour differences: its dL/dD term is 0)
                bar[s] = li[s];
                continue;
            }
            R sum = R(0);
            // the voxel's terms of dw/dc (half of each cross-octant edge to
            // each side), summed in the field type
            R creg_own = R(0), creg_x[3] = {R(0), R(0), R(0)};
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const R dl = lj[s][k] - li[s];
                sum += w[k] * dl;
                if (REG && mobile<MOB>(s)) {
                    if ((code >> (3 + k)) & 1u) {
                        creg_own += R(0.5) * dl;
                        creg_x[k >> 1] += R(0.5) * dl;
                    } else {
                        creg_own += dl;
                    }
                }
            }
            bar[s] = mobile<MOB>(s) ? li[s] + C.a[s] * sum : li[s];
            g[s] += (double)(u[s] * sum);   // dL/da_s (each voxel's term in the field type)
            if (REG && mobile<MOB>(s)) {
                const R f = C.a[s] * u[s];
                own_c += (double)(f * creg_own);
                cross_c[0] += (double)(f * creg_x[0]);
                cross_c[1] += (double)(f * creg_x[1]);
                cross_c[2] += (double)(f * creg_x[2]);
            }
        }
        if (REG) {
            // four region slots of this thread (the octant and its three
            // neighbours across the mid-planes); private, in a fixed order
            const unsigned tid = threadIdx.x;
            creg[own][tid] += own_c;
            creg[own ^ 1u][tid] += cross_c[0];
            creg[own ^ 2u][tid] += cross_c[1];
            creg[own ^ 4u][tid] += cross_c[2];
        }
        // adjoint of the transformation half
        transform_rev(C, x, bar, &g[5]);
#pragma unroll
        for (int s = 0; s < VG_NPOOL - 1; s++) elem(lout[s], i) = (R)((double)bar[s] + sd[s]);
        if (!CO2U) elem(lout[4], i) = (R)((double)bar[4] + sd[4]);
    };

    // Full tiles run software-pipelined: a tile's own words (state,
    // lambda^(k+1), neighbour words, region code) are loaded in the previous
    // iteration, right after that iteration's neighbour gathers, so that a
    // tile waits for one dependent round trip (its gathers) instead of two.
    // No memory access in this loop is guarded (every lane of a full tile
    // holds a voxel; the look-ahead past the last full tile reads voxel 0),
    // so every path issues the same memory instructions.  A ragged last tile
    // is the last tile of its block (each block's tiles ascend) and runs
    // after the loop.
    static_assert(kVPT == 1, "one voxel per thread and tile");
    const int64_t nfull = n / kTile;
    auto own_index = [&](int64_t tt) -> I { return (I)(tt < nfull ? tt * kTile + threadIdx.x : 0); };
    int64_t t = xcd_stride_tile(blockIdx.x, gridDim.x, 0, A.ntiles);
    AdjOwn<R, NS> cur;
    if (t < nfull) adj_load_own<R, MOB, REG, NS, DALL, CO2U>(A, st, lin, own_index(t), cur);
    for (int64_t it = 1; t < nfull; it++) {
        const int64_t tn = xcd_stride_tile(blockIdx.x, gridDim.x, it, A.ntiles);
        const int64_t i64 = t * kTile + threadIdx.x;
        const I i = (I)i64;
        double sd[VG_NPOOL];
        R lco2;
        volume_terms(t, i64, sd, lco2);
        R zj[VG_NPOOL][6], lj[VG_NPOOL][6];
        gather(cur, i, zj, lj);
        AdjOwn<R, NS> nxt;
        adj_load_own<R, MOB, REG, NS, DALL, CO2U>(A, st, lin, own_index(tn), nxt);
        work(cur, i, sd, lco2, zj, lj);
        cur = nxt;
        t = tn;
    }
    if (t < A.ntiles) {
        // the ragged last tile
        const int64_t i64 = t * kTile + threadIdx.x;
        double sd[VG_NPOOL];
        R lco2;
        volume_terms(t, i64, sd, lco2);
        if (i64 < n) {
            const I i = (I)i64;
            adj_load_own<R, MOB, REG, NS, DALL, CO2U>(A, st, lin, i, cur);
            R zj[VG_NPOOL][6], lj[VG_NPOOL][6];
            gather(cur, i, zj, lj);
            work(cur, i, sd, lco2, zj, lj);
        }
    }
    if (REG) {
#pragma unroll
        for (int r = 0; r < VG_NREG; r++) g[12 + r] = creg[r][threadIdx.x];
    }
    block_sum<kG>(g, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kG; q++) part[(int64_t)blockIdx.x * kG + q] += g[q];
    }
}

__global__ __launch_bounds__(kBlock) void k_fill(double *__restrict__ p, int64_t cnt, double v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < cnt) p[i] = v;
}

// grad[q] += sum over blocks (fixed order) of part[b][q]; dL/da_s -> dL/dD_s;
// grad[s] = NaN for the pools in `skipped` (bit s).
__global__ __launch_bounds__(kBlock) void k_adj_finalize(const double *__restrict__ part, int nblocks,
                                                         double scale_d, unsigned skipped,
                                                         double *__restrict__ grad) {
    __shared__ double lds[kWaves * kG];
    double v[kG];
#pragma unroll
    for (int q = 0; q < kG; q++) v[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
        for (int q = 0; q < kG; q++) v[q] += part[(int64_t)b * kG + q];
    }
    block_sum<kG>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < kG; q++) {
            if (q < VG_NPOOL && ((skipped >> q) & 1u)) grad[q] = __builtin_nan("");
            else grad[q] += q < VG_NPOOL ? v[q] * scale_d : v[q];
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_seed(R *__restrict__ lam, const double *__restrict__ seed, int zero,
                                                 Pieces pc, int64_t n) {
    const int64_t t = blockIdx.x;
    for (int v = 0; v < kVPT; v++) {
        const int64_t i = t * kTile + v * kBlock + threadIdx.x;
        if (i >= n) return;
        int32_t p = pc.piece_first[t];
        while (p + 1 < pc.piece_first[t + 1] && i >= pc.piece_lo[p + 1]) p++;
        const double *sd = seed + (int64_t)pc.piece_seg[p] * VG_NPOOL;
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            const int64_t e = (int64_t)s * n + i;
            lam[e] = (R)((zero ? 0.0 : (double)lam[e]) + sd[s]);
        }
    }
}

// The volume of voxel i from the reduction pieces of its tile.
__device__ __forceinline__ int32_t seg_of(const Pieces &pc, int64_t i) {
    const int64_t t = i / kTile;
    int32_t p = pc.piece_first[t];
    while (p + 1 < pc.piece_first[t + 1] && i >= pc.piece_lo[p + 1]) p++;
    return pc.piece_seg[p];
}

// flag[g] = 1 where the CO2 adjoint differs from the volume's first voxel's
// (flag cleared before; NaN counts as different).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_co2_check(const R *__restrict__ lam4, int64_t n, Pieces pc,
                                                      const int32_t *__restrict__ seg_first,
                                                      int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t g = seg_of(pc, i);
    const R first = lam4[pc.piece_lo[seg_first[g]]];
    if (!(lam4[i] == first)) atomicOr(&flag[g], 1);
}

// co2[g] = the CO2 adjoint of volume g (its first voxel's; 0 for an empty volume).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_co2_init(const R *__restrict__ lam4, int nseg, Pieces pc,
                                                     const int32_t *__restrict__ seg_first, R *__restrict__ co2) {
    const int g = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (g >= nseg) return;
    const int32_t p = seg_first[g];
    co2[g] = p < pc.npieces && pc.piece_seg[p] == g ? lam4[pc.piece_lo[p]] : R(0);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_co2_expand(R *__restrict__ lam4, int64_t n, Pieces pc,
                                                       const R *__restrict__ co2) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) lam4[i] = co2[seg_of(pc, i)];
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *__restrict__ p, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < cnt) p[i] = 0;
}

template <typename R, int MOB, bool REG, bool FROM_X, int NS, bool DALL, bool CO2U>
int launch_adj_k(vg_sim *h, const AdjBufs<R> &A, const Coef<R> &C, hipStream_t s) {
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    // the partials buffer holds h->adj_blocks slots; fewer blocks leave zeros
    const void *k = (const void *)k_adj<R, MOB, REG, FROM_X, NS, DALL, CO2U>;
    hipLaunchKernelGGL((k_adj<R, MOB, REG, FROM_X, NS, DALL, CO2U>), dim3(resident_blocks(k, h->adj_blocks)),
                       dim3(kBlock), 0, s, A, C, pc, h->adj_part);
    return launch_status("k_adj");
}

template <typename R, int MOB, bool REG, int NS, bool DALL>
int launch_adj_d(vg_sim *h, bool from_x, const AdjBufs<R> &A, const Coef<R> &C, hipStream_t s) {
    if constexpr (MOB == 1) {
        if (A.co2) return from_x ? launch_adj_k<R, MOB, REG, true, NS, DALL, true>(h, A, C, s)
                                 : launch_adj_k<R, MOB, REG, false, NS, DALL, true>(h, A, C, s);
    }
    return from_x ? launch_adj_k<R, MOB, REG, true, NS, DALL, false>(h, A, C, s)
                  : launch_adj_k<R, MOB, REG, false, NS, DALL, false>(h, A, C, s);
}

template <typename R, int MOB, bool REG, int NS>
int launch_adj_ns(vg_sim *h, bool from_x, const AdjBufs<R> &A, const Coef<R> &C, hipStream_t s) {
    // with every pool diffusing there is nothing to skip
    if (MOB == 1 && (h->adj_flags & VG_ADJ_SKIP_STATIC_D))
        return launch_adj_d<R, MOB, REG, NS, false>(h, from_x, A, C, s);
    return launch_adj_d<R, MOB, REG, NS, true>(h, from_x, A, C, s);
}

// the explicit step's neighbour source
template <typename R, int MOB, bool REG>
int launch_adj_step(vg_sim *h, bool from_x, const AdjBufs<R> &A, const Coef<R> &C, hipStream_t s) {
    if (use_relative(h)) return launch_adj_ns<R, MOB, REG, NS_REL>(h, from_x, A, C, s);
    if (use_offsets(h)) return launch_adj_ns<R, MOB, REG, NS_OFF>(h, from_x, A, C, s);
    return launch_adj_ns<R, MOB, REG, NS_TABLE>(h, from_x, A, C, s);
}

}  // namespace

// The recording keeps each step's diffused DOM (VG_ADJ_TAPE_DOM; only DOM
// diffusing).
bool tape_keeps_dom(const vg_sim *h) {
    return (h->adj_flags & VG_ADJ_TAPE_DOM) && !h->mobile_all;
}

int tape_rows(const vg_sim *h) {
    return tape_keeps_dom(h) ? 4 : VG_NPOOL;
}

// A kept-DOM recording holds per state MB, DOM, SOM and P4 (state 0: x^k0's;
// state j >= 1: T(x^(k0+j-1))'s MB, SOM, P4 and x^(k0+j)'s DOM).  The
// transformed DOM and the CO2 of the state a recording pass works on live
// in two ping-pong row pairs of the adjoint's second lambda buffer (idle
// while recording), state j's in pair j & 1; state 0's CO2 is the bound
// fields'.
void tape_pass_bufs(const vg_sim *h, void *states, int64_t j, const void *src[VG_NPOOL], void *dst[VG_NPOOL],
                    void **xdom) {
    const int64_t n = h->n;
    const size_t esz = h->elem();
    char *st = (char *)states;
    const int rows = tape_rows(h);
    auto at_row = [&](int64_t jj, int r) { return (void *)(st + ((size_t)jj * rows + r) * n * esz); };
    for (int p = 0; p < VG_NPOOL; p++) {
        src[p] = p < rows ? at_row(j, p) : nullptr;
        dst[p] = p < rows ? at_row(j + 1, p) : nullptr;
    }
    *xdom = nullptr;
    if (rows == VG_NPOOL) return;
    char *side = (char *)h->lam_alt;
    auto side_row = [&](int64_t jj, int r) { return (void *)(side + ((size_t)(jj & 1) * 2 + r) * n * esz); };
    if (j > 0) {
        src[1] = side_row(j, 0);
        src[4] = side_row(j, 1);
        *xdom = at_row(j, 1);
    } else {
        src[4] = h->fields + 4 * n * esz;
    }
    dst[1] = side_row(j + 1, 0);
    dst[4] = side_row(j + 1, 1);
}

namespace {

template <typename R>
int adjoint_sweep(vg_sim *h, int64_t nsteps, double dt, const void *states, const double *seeds, void *lambda,
                  double *grad, hipStream_t s) {
    const Coef<R> C = make_coef<R>(h, dt);
    const int64_t n = h->n;
    const int64_t cnt = (int64_t)h->adj_blocks * kG;
    int rc;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, h->adj_part, cnt,
                       0.0);
    if ((rc = launch_status("k_fill"))) return rc;
    R *bufs[2] = {(R *)lambda, (R *)h->lam_alt};
    int cur = 0;
    const bool reg = h->rcode != nullptr;
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    const unsigned nb_n = (unsigned)((n + kBlock - 1) / kBlock), nb_g = (unsigned)((h->nseg + kBlock - 1) / kBlock);
    // the uniform CO2 adjoint per volume, in two buffers: reverse step m reads
    // co2b[m & 1] and its block 0 writes the next value into the other
    R *co2b[2] = {(R *)h->adj_co2, (R *)h->adj_co2 + h->nseg};
    R *lam4 = (R *)lambda + 4 * n;
    // a CO2 adjoint uniform over each volume travels as one value per volume
    bool co2u = false;
    if (!h->mobile_all && n > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(nb_g), dim3(kBlock), 0, s, h->adj_flag, (int64_t)h->nseg);
        if ((rc = launch_status("k_fill_i32"))) return rc;
        hipLaunchKernelGGL(k_co2_check<R>, dim3(nb_n), dim3(kBlock), 0, s, lam4, n, pc, h->seg_first, h->adj_flag);
        if ((rc = launch_status("k_co2_check"))) return rc;
        std::vector<int32_t> flag((size_t)h->nseg);
        if ((rc = hip_status(hipMemcpyAsync(flag.data(), h->adj_flag, sizeof(int32_t) * flag.size(),
                                            hipMemcpyDeviceToHost, s), "adjoint CO2 check"))) return rc;
        if ((rc = hip_status(hipStreamSynchronize(s), "adjoint CO2 check"))) return rc;
        co2u = true;
        for (int32_t f : flag) co2u = co2u && f == 0;
        if (co2u) {
            hipLaunchKernelGGL(k_co2_init<R>, dim3(nb_g), dim3(kBlock), 0, s, lam4, h->nseg, pc, h->seg_first, co2b[0]);
            if ((rc = launch_status("k_co2_init"))) return rc;
        }
    }
    // recorded with the diffused DOM kept (see record): every step reads its
    // x^k directly; those states hold no CO2, which only dL/dD_CO2 with a
    // CO2 adjoint that varies within a volume would need
    const bool xd = tape_keeps_dom(h);
    if (xd && !co2u && !(h->adj_flags & VG_ADJ_SKIP_STATIC_D)) {
        set_error("states recorded with VG_ADJ_TAPE_DOM hold no CO2: dL/dD_CO2 needs a CO2 adjoint uniform over "
                  "each volume, or VG_ADJ_SKIP_STATIC_D");
        return VG_EINVAL;
    }
    const int rows = tape_rows(h);
    for (int64_t jstep = nsteps - 1; jstep >= 0; jstep--) {
        AdjBufs<R> A;
        A.nbr = h->nbr;
        A.rcode = h->rcode;
        A.pk = packed_of(h);
        A.st = (const R *)states + jstep * rows * n;
        A.co2_row = rows == VG_NPOOL ? 4 : 3;
        A.lin = bufs[cur];
        A.lout = bufs[cur ^ 1];
        A.seed = seeds + jstep * (int64_t)h->nseg * VG_NPOOL;
        const int m = (int)((nsteps - 1 - jstep) & 1);
        A.co2 = co2u ? co2b[m] : nullptr;
        A.co2_next = co2u ? co2b[m ^ 1] : nullptr;
        A.nseg = h->nseg;
        A.n = n;
        A.ntiles = h->ntiles;
        const bool fx = jstep == 0 || xd;
        if (h->mobile_all) rc = reg ? launch_adj_step<R, 2, true>(h, fx, A, C, s) : launch_adj_step<R, 2, false>(h, fx, A, C, s);
        else rc = reg ? launch_adj_step<R, 1, true>(h, fx, A, C, s) : launch_adj_step<R, 1, false>(h, fx, A, C, s);
        if (rc) return rc;
        cur ^= 1;
    }
    if (cur) {
        // (the CO2 rows are filled below in the uniform case)
        const size_t pools = co2u ? VG_NPOOL - 1 : VG_NPOOL;
        if ((rc = hip_status(hipMemcpyAsync(lambda, h->lam_alt, sizeof(R) * pools * (size_t)n,
                                            hipMemcpyDeviceToDevice, s), "lambda copy"))) return rc;
    }
    if (co2u) {
        hipLaunchKernelGGL(k_co2_expand<R>, dim3(nb_n), dim3(kBlock), 0, s, lam4, n, pc,
                           (const R *)co2b[nsteps & 1]);
        if ((rc = launch_status("k_co2_expand"))) return rc;
    }
    const double scale_d = dt / (h->params.h * h->params.h);
    // pools whose dL/dD_s the sweep skipped: all but DOM, when asked and not every pool diffuses
    const unsigned skipped = (!h->mobile_all && (h->adj_flags & VG_ADJ_SKIP_STATIC_D)) ? 0x1du : 0u;
    hipLaunchKernelGGL(k_adj_finalize, dim3(1), dim3(kBlock), 0, s, h->adj_part, h->adj_blocks, scale_d, skipped,
                       grad);
    return launch_status("k_adj_finalize");
}

template <typename R>
int record(vg_sim *h, int64_t nsteps, double dt, void *states, hipStream_t s) {
    const int64_t n = h->n;
    int rc;
    // states[0] = x^k0 (the bound fields; a kept-DOM recording takes their
    // first four rows)
    if ((rc = hip_status(hipMemcpyAsync(states, h->fields, sizeof(R) * tape_rows(h) * (size_t)n,
                                        hipMemcpyDeviceToDevice, s), "record copy"))) return rc;
    const void *src[VG_NPOOL];
    void *dst[VG_NPOOL];
    void *xdom;
    for (int64_t jstep = 1; jstep < nsteps; jstep++) {
        // states[1] = T(x^k0); states[j] = T(D(states[j-1])) afterwards; a
        // kept-DOM recording writes D(states[j-1])'s DOM into states[j-1]
        tape_pass_bufs(h, states, jstep - 1, src, dst, &xdom);
        if ((rc = launch_pass_bufs(h, jstep == 1 ? MODE_T : MODE_DT, TOT_NONE, dt, src, dst, s, xdom))) return rc;
    }
    if (tape_keeps_dom(h) && nsteps >= 2) {
        // the last state's diffused DOM: a diffusion pass (it writes DOM only)
        tape_pass_bufs(h, states, nsteps - 1, src, dst, &xdom);
        for (int p = 0; p < VG_NPOOL; p++) dst[p] = (void *)src[p];
        dst[1] = xdom;
        if ((rc = launch_pass_bufs(h, MODE_D, TOT_NONE, dt, src, dst, s))) return rc;
    }
    return VG_OK;
}

}  // namespace

int launch_record(vg_sim *h, int64_t nsteps, double dt, void *states, hipStream_t s) {
    if (h->n == 0 || nsteps == 0) return VG_OK;
    if (h->prec == VG_F64) return record<double>(h, nsteps, dt, states, s);
    return record<float>(h, nsteps, dt, states, s);
}

int launch_adjoint(vg_sim *h, int64_t nsteps, double dt, const void *states, const double *seeds, void *lambda,
                   double *grad, hipStream_t s) {
    if (h->n == 0 || nsteps == 0) return VG_OK;
    if (h->prec == VG_F64) return adjoint_sweep<double>(h, nsteps, dt, states, seeds, lambda, grad, s);
    return adjoint_sweep<float>(h, nsteps, dt, states, seeds, lambda, grad, s);
}

int launch_seed(vg_sim *h, const double *seed, void *lambda, int zero, hipStream_t s) {
    if (h->n == 0) return VG_OK;
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    if (h->prec == VG_F64)
        hipLaunchKernelGGL((k_seed<double>), dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, (double *)lambda, seed,
                           zero, pc, h->n);
    else
        hipLaunchKernelGGL((k_seed<float>), dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, (float *)lambda, seed,
                           zero, pc, h->n);
    return launch_status("k_seed");
}

}  // namespace vg
