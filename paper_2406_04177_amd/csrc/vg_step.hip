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

// MOB: 1 = only DOM diffuses, 2 = every pool diffuses (a_s may be 0).
template <int MOB>
__device__ __forceinline__ constexpr bool mobile(int s) {
    return MOB == 2 || (MOB == 1 && s == 1);
}

template <typename R, int MODE, int MOB, bool REG, int TOT>
__global__ __launch_bounds__(kBlock) void k_step(StepBufs<R> B, Coef<R> C, Pieces pc,
                                                 double *__restrict__ part) {
    __shared__ double lds[kWaves * VG_NPOOL];
    __shared__ R cl[VG_NREG];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t i = tile * kTile + threadIdx.x;
    const bool active = i < B.n;
    if (REG) {
        if (threadIdx.x < VG_NREG) cl[threadIdx.x] = C.c[threadIdx.x];
        __syncthreads();
    }

    constexpr bool do_d = MODE == MODE_D || MODE == MODE_DT;
    constexpr bool do_t = MODE == MODE_T || MODE == MODE_DT;
    // pools this pass must read: all of them unless it only diffuses
    // (a D-only pass reads the immobile pools only to total them)
    R x[VG_NPOOL];
    double acc[VG_NPOOL];
#pragma unroll
    for (int s = 0; s < VG_NPOOL; s++) {
        x[s] = R(0);
        acc[s] = 0.0;
    }
    if (active) {
#pragma unroll
        for (int s = 0; s < VG_NPOOL; s++) {
            const bool need = !(MODE == MODE_D) || mobile<MOB>(s) || TOT != TOT_NONE;
            if (need) x[s] = B.src[s][i];
        }
        if (TOT == TOT_IN) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[s] = (double)x[s];
        }
        if (do_d) {
            int32_t j[6];
#pragma unroll
            for (int k = 0; k < 6; k++) j[k] = B.nbr[(int64_t)k * B.n + i];
            R w[6];
            if (REG) {
                const uint32_t code = B.rcode[i];
                const uint32_t own = code & 7u;
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const uint32_t other = own ^ (((code >> (3 + k)) & 1u) << (k >> 1));
                    w[k] = R(0.5) * (cl[own] + cl[other]);
                }
            }
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) {
                if (!mobile<MOB>(s)) continue;
                const R xi = x[s];
                R d[6];
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    R t = R(0);
                    if (j[k] >= 0) {
                        const R diff = B.src[s][j[k]] - xi;
                        t = REG ? w[k] * diff : diff;
                    }
                    d[k] = t;
                }
                const R sum = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]);
                x[s] = xi + C.a[s] * sum;
            }
        }
        if (TOT == TOT_MID) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[s] = (double)x[s];
        }
        if (do_t) transform(C, x[0], x[1], x[2], x[3], x[4]);
        if (TOT == TOT_OUT) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) acc[s] = (double)x[s];
        }
        if (MODE != MODE_NONE) {
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) {
                const bool write = MODE != MODE_D || mobile<MOB>(s);
                if (write) B.dst[s][i] = x[s];
            }
        }
    }
    if (TOT != TOT_NONE) {
        const int32_t p0 = pc.piece_first[tile], p1 = pc.piece_first[tile + 1];
        for (int32_t p = p0; p < p1; p++) {
            const bool in = active && i >= pc.piece_lo[p] && i < pc.piece_lo[p + 1];
            double v[VG_NPOOL];
#pragma unroll
            for (int s = 0; s < VG_NPOOL; s++) v[s] = in ? acc[s] : 0.0;
            block_sum<VG_NPOOL>(v, lds);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int s = 0; s < VG_NPOOL; s++) part[(int64_t)p * VG_NPOOL + s] = v[s];
            }
        }
    }
}

// One block per segment: sum its pieces in a fixed order, then the five pool
// totals into total carbon.
__global__ __launch_bounds__(kBlock) void k_totals_finalize(const double *__restrict__ part,
                                                            const int32_t *__restrict__ seg_first,
                                                            double *__restrict__ out) {
    __shared__ double lds[kWaves * VG_NPOOL];
    const int g = blockIdx.x;
    const int32_t p0 = seg_first[g], p1 = seg_first[g + 1];
    double v[VG_NPOOL] = {0, 0, 0, 0, 0};
    for (int32_t p = p0 + (int32_t)threadIdx.x; p < p1; p += kBlock) {
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

template <typename R, int MODE, int MOB, bool REG, int TOT>
int launch_one(vg_sim *h, const StepBufs<R> &B, const Coef<R> &C, hipStream_t s) {
    Pieces pc{h->piece_first, h->piece_lo, h->piece_seg, h->npieces};
    hipLaunchKernelGGL((k_step<R, MODE, MOB, REG, TOT>), dim3((unsigned)h->ntiles), dim3(kBlock), 0, s, B,
                       C, pc, h->part);
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
    if (mode == MODE_NONE) return pick_tot<R, MODE_NONE, 1, false>(h, TOT_IN, B, C, s);
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
    if (h->nseg == 0) return VG_OK;
    hipLaunchKernelGGL(k_totals_finalize, dim3((unsigned)h->nseg), dim3(kBlock), 0, s, h->part, h->seg_first,
                       out_rows);
    return launch_status("k_totals_finalize");
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
