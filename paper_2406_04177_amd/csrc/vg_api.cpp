// C-ABI of libvgsim: handle, argument validation, workspace layout and the
// orchestration of the kernels of vg_step.hip, vg_cg.hip and vg_adjoint.hip.
// Owns no device memory: every device buffer is bound by the caller.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "vg_internal.h"

namespace vg {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return VG_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return VG_EHIP;
}

int launch_status(const char *what) { return hip_status(hipGetLastError(), what); }

int resident_blocks(const void *kernel, int cap) {
    struct Entry {
        const void *kernel;
        int dev, blocks;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return cap;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (const Entry &e : cache)
            if (e.kernel == kernel && e.dev == dev) return e.blocks < cap ? e.blocks : cap;
    }
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0) != hipSuccess || cus <= 0 ||
        per <= 0) {
        (void)hipGetLastError();
        return cap;
    }
    int g = per * cus;
    if (g >= kNumXcd) g -= g % kNumXcd;
    {
        std::lock_guard<std::mutex> lock(mu);
        cache.push_back({kernel, dev, g});
    }
    return g < cap ? g : cap;
}

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Workspace layout; with base == nullptr it only measures.
size_t layout(vg_sim *h, char *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes ? bytes : 1);
        return p;
    };
    h->piece_first = (int32_t *)take(sizeof(int32_t) * (size_t)(h->ntiles + 1));
    h->piece_lo = (int64_t *)take(sizeof(int64_t) * (size_t)(h->npieces + 1));
    h->piece_seg = (int32_t *)take(sizeof(int32_t) * (size_t)h->npieces);
    h->seg_first = (int32_t *)take(sizeof(int32_t) * (size_t)(h->nseg + 1));
    h->part = (double *)take(sizeof(double) * VG_NPOOL * (size_t)h->npieces * (size_t)h->tot_batch);
    h->tot_tmp = (double *)take(sizeof(double) * 6 * (size_t)h->nseg);
    h->chunk_first = (int32_t *)take(sizeof(int32_t) * (size_t)(h->nchunks + 1));
    h->seg_chunk = (int32_t *)take(sizeof(int32_t) * (size_t)(h->nseg + 1));
    h->chunk_part = (double *)take(sizeof(double) * VG_NPOOL * (size_t)h->nchunks * (size_t)h->tot_batch);
    h->geo = h->rank ? (uint32_t *)take(sizeof(uint32_t) * (size_t)h->n) : nullptr;
    h->off_m = (uint32_t *)take(sizeof(uint32_t) * (size_t)h->n);
    h->off_p = (uint32_t *)take(sizeof(uint32_t) * (size_t)h->n);
    h->off_stat = (uint32_t *)take(sizeof(uint32_t) * 8);
    h->rel_w = (uint32_t *)take(sizeof(uint32_t) * (size_t)h->n);
    h->rel_base = (uint32_t *)take(sizeof(uint32_t) * 8 * (size_t)((h->n + kGroup - 1) / kGroup));
    const size_t nd = sizeof(double) * (size_t)h->n;
    if (h->features & VG_FEAT_CG) {
        h->cg_y = (double *)take(nd);
        h->cg_r = (double *)take(nd);
        h->cg_z = (double *)take(nd);
        h->cg_q = (double *)take(nd);
        h->cg_m = (double *)take(nd);
        h->cg_p[0] = (double *)take(nd);
        h->cg_p[1] = (double *)take(nd);
        h->cg_part = (double *)take(sizeof(double) * 4 * (size_t)h->cg_blocks);
        h->cg_scal = (double *)take(sizeof(double) * 8);
    }
    if (h->features & VG_FEAT_MG) {
        // the hierarchy at the capacities mg_plan reserved (set-up scratch:
        // the occupancy bytes of the largest coarse grid)
        h->mg[0].parent = (int32_t *)take(sizeof(int32_t) * (size_t)h->n);
        h->mg[0].e = (double *)take(sizeof(double) * (size_t)h->n);   // fine residual / prolongated iterate
        size_t mask = 1;
        for (int l = 1; l < h->mg_plan_levels; l++) {
            vg_sim::MgLevel &L = h->mg[l];
            const size_t cap = (size_t)L.cap;
            L.vox = (int32_t *)take(sizeof(int32_t) * cap);
            L.nbr = (int32_t *)take(sizeof(int32_t) * 6 * cap);
            L.w = (float *)take(sizeof(float) * 6 * cap);
            L.mass = (float *)take(sizeof(float) * cap);
            L.invd = (double *)take(sizeof(double) * cap);
            L.r = (double *)take(sizeof(double) * cap);
            L.x = (double *)take(sizeof(double) * cap);
            L.e = (double *)take(sizeof(double) * cap);
            L.parent = (int32_t *)take(sizeof(int32_t) * cap);
            size_t rb = 0;
            vg_rank_bytes(L.nx, L.ny, L.nz, 0, &rb);
            L.rank = (RankWord *)take(rb);
            const size_t cells = (size_t)L.nx * (size_t)L.ny * (size_t)L.nz;
            mask = cells > mask ? cells : mask;
        }
        h->mg_mask = (uint8_t *)take(mask);
    }
    if (h->features & VG_FEAT_ADJ) {
        h->lam_alt = take(h->elem() * VG_NPOOL * (size_t)h->n);
        h->adj_part = (double *)take(sizeof(double) * VG_NGRAD * (size_t)h->adj_blocks);
        h->adj_co2 = take(h->elem() * 2 * (size_t)h->nseg);
        h->adj_flag = (int32_t *)take(sizeof(int32_t) * (size_t)h->nseg);
    }
    if (band_geometry(h)) {
        h->band_rs = (int32_t *)take(sizeof(int32_t) * ((size_t)h->nz * (size_t)h->ny + 1));
        h->band_alt = take(h->elem() * VG_NPOOL * (size_t)h->n);
    }
    if (h->prec == VG_F32C) {
        h->lo = (int16_t *)take(sizeof(int16_t) * VG_NPOOL * (size_t)h->n);
        h->lo_alt = (int16_t *)take(sizeof(int16_t) * (h->mobile_all ? VG_NPOOL : 1) * (size_t)h->n);
    }
    return off;
}

// Pieces: the intersections of the reduction tiles with the segments.
void make_pieces(vg_sim *h) {
    const int64_t n = h->n;
    h->ntiles = (n + kTile - 1) / kTile;
    h->piece_first_h.assign((size_t)h->ntiles + 1, 0);
    h->piece_lo_h.clear();
    h->piece_seg_h.clear();
    int g = 0;
    while (g < h->nseg && h->seg_off[g + 1] <= 0) g++;
    for (int64_t t = 0; t < h->ntiles; t++) {
        h->piece_first_h[t] = (int32_t)h->piece_seg_h.size();
        int64_t lo = t * kTile;
        const int64_t hi = lo + kTile < n ? lo + kTile : n;
        while (lo < hi) {
            while (h->seg_off[g + 1] <= lo) g++;
            h->piece_lo_h.push_back(lo);
            h->piece_seg_h.push_back(g);
            lo = h->seg_off[g + 1] < hi ? h->seg_off[g + 1] : hi;
        }
    }
    h->piece_first_h[h->ntiles] = (int32_t)h->piece_seg_h.size();
    h->npieces = (int32_t)h->piece_seg_h.size();
    h->piece_lo_h.push_back(n);
    h->seg_first_h.assign((size_t)h->nseg + 1, h->npieces);
    for (int gg = h->nseg - 1; gg >= 0; gg--) h->seg_first_h[gg] = h->seg_first_h[gg + 1];
    for (int p = h->npieces - 1; p >= 0; p--) h->seg_first_h[h->piece_seg_h[p]] = p;
    // empty segments take the start of the next non-empty one
    for (int gg = h->nseg - 1; gg >= 0; gg--)
        if (h->seg_off[gg] == h->seg_off[gg + 1]) h->seg_first_h[gg] = h->seg_first_h[gg + 1];
    // totals chunks: runs of up to kChunk pieces inside one segment
    h->chunk_first_h.clear();
    h->seg_chunk_h.assign((size_t)h->nseg + 1, 0);
    for (int gg = 0; gg < h->nseg; gg++) {
        h->seg_chunk_h[gg] = (int32_t)h->chunk_first_h.size();
        for (int32_t p = h->seg_first_h[gg]; p < h->seg_first_h[gg + 1]; p += kChunk) h->chunk_first_h.push_back(p);
    }
    h->nchunks = (int32_t)h->chunk_first_h.size();
    h->max_seg_pieces = 0;
    for (int gg = 0; gg < h->nseg; gg++) {
        const int32_t np = h->seg_first_h[gg + 1] - h->seg_first_h[gg];
        if (np > h->max_seg_pieces) h->max_seg_pieces = np;
    }
    h->seg_chunk_h[h->nseg] = h->nchunks;
    h->chunk_first_h.push_back(h->npieces);
    // logged passes per totals launch: up to 32, within 32 MB of partials
    const int64_t row_bytes = (int64_t)sizeof(double) * VG_NPOOL * (h->npieces > 0 ? h->npieces : 1);
    const int64_t tb = ((int64_t)32 << 20) / row_bytes;
    h->tot_batch = (int)(tb < 1 ? 1 : (tb > 32 ? 32 : tb));
    const int64_t cap = 2048;
    h->cg_blocks = (int)(h->ntiles < cap ? (h->ntiles > 0 ? h->ntiles : 1) : cap);
    h->adj_blocks = h->cg_blocks;
}

int check_params(const vg_sim *h, const vg_params *p) {
    if (!(p->h > 0) || !std::isfinite(p->h)) { set_error("h must be positive"); return VG_EINVAL; }
    if (!(p->k_dom > 0)) { set_error("K_DOM must be positive"); return VG_EINVAL; }
    const double r[6] = {p->v_dom, p->rho, p->mu, p->v_som, p->v_p4, p->beta};
    for (double v : r)
        if (!(v >= 0) || !std::isfinite(v)) { set_error("rates must be finite and >= 0"); return VG_EINVAL; }
    if (p->beta > 1) { set_error("beta must lie in [0, 1]"); return VG_EINVAL; }
    for (int s = 0; s < VG_NPOOL; s++) {
        if (!(p->D[s] >= 0) || !std::isfinite(p->D[s])) { set_error("D must be finite and >= 0"); return VG_EINVAL; }
        if (!h->mobile_all && s != 1 && p->D[s] != 0) {
            set_error("pool %d diffuses but the handle was created with mobile_all = 0", s);
            return VG_EINVAL;
        }
    }
    if (p->step_order != VG_ORDER_TD && p->step_order != VG_ORDER_DT) {
        set_error("step_order must be VG_ORDER_TD or VG_ORDER_DT");
        return VG_EINVAL;
    }
    if (p->sequential != 0 && p->sequential != 1) { set_error("sequential must be 0 or 1"); return VG_EINVAL; }
    return VG_OK;
}

double max_c(const vg_sim *h);

// VG_EUNSTABLE when an explicit diffusion step of dt could make masses negative.
int check_stable(const vg_sim *h, double dt) {
    double dmax = 0;
    for (int s = 0; s < VG_NPOOL; s++) dmax = h->params.D[s] > dmax ? h->params.D[s] : dmax;
    const double worst = dmax * dt / (h->params.h * h->params.h) * 6.0 * max_c(h);
    if (worst > 1.0) {
        set_error("dt = %g gives max_s a_s * sum_j w_ij = %g > 1 (negative masses possible)", dt, worst);
        return VG_EUNSTABLE;
    }
    return VG_OK;
}

double max_c(const vg_sim *h) {
    double m = 1.0;
    if (h->rcode) {
        m = h->c[0];
        for (int r = 1; r < VG_NREG; r++) m = h->c[r] > m ? h->c[r] : m;
    }
    return m;
}

int need_bound(const vg_sim *h) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (!h->bound) { set_error("no state bound (call vg_init_state)"); return VG_ESTATE; }
    return VG_OK;
}

}  // namespace
}  // namespace vg

using namespace vg;

extern "C" const char *vg_strerror(int code) {
    switch (code) {
        case VG_OK: return "ok";
        case VG_EINVAL: return "invalid argument";
        case VG_EUNSTABLE: return "explicit time step above the stability bound";
        case VG_ENOCONV: return "conjugate gradient did not converge";
        case VG_ENONFINITE: return "non-finite mass total";
        case VG_EHIP: return "HIP runtime error";
        case VG_ESTATE: return "call out of sequence";
        default: return "unknown error";
    }
}

extern "C" const char *vg_last_error(void) { return g_err; }

extern "C" int vg_version(void) { return 100; }

extern "C" int vg_create(const vg_desc *d, vg_sim **out) {
    if (!d || !out) { set_error("null pointer argument"); return VG_EINVAL; }
    *out = nullptr;
    if (d->n < 0 || d->n > INT32_MAX || d->nseg < 1 || !d->seg_off || (d->n > 0 && !d->nbr_d)) {
        set_error("bad graph descriptor (n, nseg, seg_off, nbr)");
        return VG_EINVAL;
    }
    if (d->precision != VG_F32 && d->precision != VG_F64 && d->precision != VG_F32C) {
        set_error("precision must be VG_F32, VG_F64 or VG_F32C");
        return VG_EINVAL;
    }
    if (d->precision == VG_F32C && (d->features & VG_FEAT_ADJ)) {
        set_error("the adjoint needs VG_F32 or VG_F64 fields");
        return VG_EINVAL;
    }
    if (d->seg_off[0] != 0 || d->seg_off[d->nseg] != d->n) { set_error("seg_off must run from 0 to n"); return VG_EINVAL; }
    for (int g = 0; g < d->nseg; g++)
        if (d->seg_off[g + 1] < d->seg_off[g]) { set_error("seg_off must be non-decreasing"); return VG_EINVAL; }
    if (d->features & ~(VG_FEAT_CG | VG_FEAT_ADJ | VG_FEAT_BAND | VG_FEAT_MG)) {
        set_error("unknown feature bits");
        return VG_EINVAL;
    }
    vg_sim *h = new (std::nothrow) vg_sim();
    if (!h) { set_error("out of host memory"); return VG_EINVAL; }
    h->n = d->n;
    h->nseg = d->nseg;
    h->prec = d->precision;
    h->mobile_all = d->mobile_all ? 1 : 0;
    h->features = d->features;
    h->seg_off.assign(d->seg_off, d->seg_off + d->nseg + 1);
    h->nbr = d->nbr_d;
    h->rcode = d->rcode_d;
    if (d->rank_d) {
        Geom g;
        int rc = make_geom(d->nx, d->ny, d->nz, d->brick, &g);
        if (rc) { delete h; return rc; }
        if (d->nseg != 1 || g.npos >= ((int64_t)1 << 31) || d->periodic > 7u || !d->vox_d) {
            set_error("a rank index needs a single volume of fewer than 2^31 positions and vox_d");
            delete h;
            return VG_EINVAL;
        }
        // the rank-index kernel covers volumes without periodic axes and with
        // every dimension <= 1024 (10-bit coordinates); others use the table
        if (d->periodic == 0 && d->nx <= 1024 && d->ny <= 1024 && d->nz <= 1024) {
            h->rank = d->rank_d;
            h->vox = d->vox_d;
        }
        h->nx = d->nx; h->ny = d->ny; h->nz = d->nz; h->brick = d->brick; h->periodic = d->periodic;
    }
    vg_params p{};
    p.D[1] = 1e-9;
    p.h = 24e-6;
    p.v_dom = 1e-4; p.k_dom = 0.5; p.rho = 2e-6; p.mu = 5e-7; p.beta = 0.55; p.v_som = 1e-7; p.v_p4 = 1e-7;
    p.mort_to_p4 = 0;
    p.step_order = VG_ORDER_TD;
    h->params = p;
    if (h->features & VG_FEAT_MG) {
        if (!(h->features & VG_FEAT_CG) || !h->rank) {
            set_error("VG_FEAT_MG needs VG_FEAT_CG and a single volume with a rank index, no periodic axis and "
                      "every dimension <= 1024");
            delete h;
            return VG_EINVAL;
        }
        mg_plan(h);
    }
    make_pieces(h);
    *out = h;
    return VG_OK;
}

namespace vg {
namespace {

// Drops the captured runs (their kernels' arguments no longer hold).
void drop_graphs(vg_sim *h) {
    for (auto &g : h->run_graph) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = vg_sim::RunGraph{};
    }
    h->graph_version++;
}

bool graphs_wanted(const vg_sim *h) {
    if (h->launch_flags == VG_LAUNCH_GRAPHS_OFF) return false;
    if (h->launch_flags == VG_LAUNCH_GRAPHS_ON) return true;
    return h->n <= ((int64_t)1 << 19);   // measured: 1.35x at 48^3, 1.02x at 128^3, none from 256^3
}

constexpr int64_t kRunPasses = 16;   // fused passes per captured run (a multiple of 4: band runs)

// Launches (capturing it first if needed) a run of kRunPasses fused passes
// with no totals, starting at the current ping-pong parity.  The run returns
// the parity to where it started (an even number of passes).
int launch_run(vg_sim *h, double dt, bool band, hipStream_t s) {
    vg_sim::RunGraph &g = h->run_graph[h->cur];
    if (!(g.exec && g.version == h->graph_version && g.dt == dt && g.band == (int)band && g.passes == kRunPasses &&
          g.cur == h->cur)) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = vg_sim::RunGraph{};
        int rc;
        if (!h->capture_stream &&
            (rc = hip_status(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking), "capture stream")))
            return rc;
        const int cur0 = h->cur;
        if ((rc = hip_status(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal),
                             "begin capture")))
            return rc;
        int lrc = VG_OK;
        for (int64_t k = 0; k < kRunPasses && lrc == VG_OK; k += band ? 4 : 1)
            lrc = band ? launch_band_quad(h, dt, h->capture_stream)
                       : launch_pass(h, MODE_DT, TOT_NONE, dt, h->capture_stream);
        hipGraph_t graph = nullptr;
        rc = hip_status(hipStreamEndCapture(h->capture_stream, &graph), "end capture");
        h->cur = cur0;   // capturing ran nothing
        if (lrc || rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return lrc ? lrc : rc;
        }
        hipGraphExec_t exec = nullptr;
        rc = hip_status(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate graph");
        (void)hipGraphDestroy(graph);
        if (rc) return rc;
        g.exec = exec;
        g.cur = cur0;
        g.passes = (int)kRunPasses;
        g.dt = dt;
        g.band = band ? 1 : 0;
        g.version = h->graph_version;
    }
    return hip_status(hipGraphLaunch(g.exec, s), "graph launch");
}

}  // namespace
}  // namespace vg

extern "C" int vg_destroy(vg_sim *h) {
    if (!h) return VG_OK;
    vg::drop_graphs(h);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    delete h;
    return VG_OK;
}

extern "C" int vg_set_launch_options(vg_sim *h, unsigned flags) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (flags > VG_LAUNCH_GRAPHS_OFF) { set_error("unknown launch options"); return VG_EINVAL; }
    h->launch_flags = flags;
    return VG_OK;
}

extern "C" int vg_set_kernel(vg_sim *h, int variant) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    const bool comp = h->prec == VG_F32C;   // compensated fields: table or packed sources only
    if (variant < VG_KERNEL_AUTO || variant > VG_KERNEL_BAND || (variant == VG_KERNEL_RANK && (!h->rank || comp)) ||
        (variant == VG_KERNEL_BAND && comp) ||
        (variant == VG_KERNEL_OFFSET && !h->off_ok) || (variant == VG_KERNEL_RELATIVE && !h->rel_ok) ||
        (variant == VG_KERNEL_BAND && !(h->band_ok && h->rel_ok))) {
        set_error("kernel variant %d not available", variant);
        return VG_EINVAL;
    }
    h->kernel = variant;
    drop_graphs(h);
    return VG_OK;
}

extern "C" int vg_set_adjoint_options(vg_sim *h, unsigned flags) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (flags & ~(VG_ADJ_SKIP_STATIC_D | VG_ADJ_TAPE_DOM)) { set_error("unknown adjoint options"); return VG_EINVAL; }
    h->adj_flags = flags;
    return VG_OK;
}

extern "C" int vg_get_kernel(const vg_sim *h, int *variant_in_use) {
    if (!h || !variant_in_use) { set_error("null pointer argument"); return VG_EINVAL; }
    *variant_in_use = vg::use_band(h)       ? VG_KERNEL_BAND
                      : vg::use_relative(h) ? VG_KERNEL_RELATIVE
                      : vg::use_offsets(h) ? VG_KERNEL_OFFSET
                      : vg::use_rank(h)    ? VG_KERNEL_RANK
                                           : VG_KERNEL_TABLE;
    return VG_OK;
}

extern "C" int vg_set_params(vg_sim *h, const vg_params *p) {
    if (!h || !p) { set_error("null pointer argument"); return VG_EINVAL; }
    int rc = check_params(h, p);
    if (rc) return rc;
    h->params = *p;
    drop_graphs(h);
    return VG_OK;
}

extern "C" int vg_set_regions(vg_sim *h, const double *c) {
    if (!h || !c) { set_error("null pointer argument"); return VG_EINVAL; }
    for (int r = 0; r < VG_NREG; r++)
        if (!(c[r] > 0) || !std::isfinite(c[r])) { set_error("region factors must be finite and > 0"); return VG_EINVAL; }
    for (int r = 0; r < VG_NREG; r++) h->c[r] = c[r];
    drop_graphs(h);
    h->mg_wdone = false;   // the coarse weights sum the region-weighted edges
    return VG_OK;
}

extern "C" int vg_alt_elems(const vg_sim *h, int64_t *elems) {
    if (!h || !elems) { set_error("null pointer argument"); return VG_EINVAL; }
    *elems = (h->mobile_all ? VG_NPOOL : 1) * h->n;
    return VG_OK;
}

extern "C" int vg_workspace_bytes(const vg_sim *h, size_t *bytes) {
    if (!h || !bytes) { set_error("null pointer argument"); return VG_EINVAL; }
    vg_sim tmp;
    tmp.n = h->n; tmp.nseg = h->nseg; tmp.prec = h->prec; tmp.features = h->features; tmp.mobile_all = h->mobile_all;
    tmp.ntiles = h->ntiles; tmp.npieces = h->npieces; tmp.cg_blocks = h->cg_blocks; tmp.adj_blocks = h->adj_blocks;
    tmp.nchunks = h->nchunks; tmp.tot_batch = h->tot_batch;
    tmp.rank = h->rank;   // the geometry words are part of the workspace when a rank index is used
    tmp.vox = h->vox; tmp.nx = h->nx; tmp.ny = h->ny; tmp.nz = h->nz; tmp.brick = h->brick; tmp.periodic = h->periodic;
    tmp.mg_plan_levels = h->mg_plan_levels;
    for (int l = 0; l < h->mg_plan_levels; l++) {
        tmp.mg[l].nx = h->mg[l].nx; tmp.mg[l].ny = h->mg[l].ny; tmp.mg[l].nz = h->mg[l].nz;
        tmp.mg[l].cap = h->mg[l].cap;
    }
    *bytes = layout(&tmp, nullptr);
    return VG_OK;
}

extern "C" int vg_init_state(vg_sim *h, void *fields_d, void *alt_d, void *work_d, size_t work_bytes, void *stream) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (h->n > 0 && (!fields_d || !alt_d || !work_d)) { set_error("null buffer"); return VG_EINVAL; }
    size_t need = 0;
    vg_workspace_bytes(h, &need);
    if (work_bytes < need) {
        set_error("workspace too small: %zu < %zu bytes", work_bytes, need);
        return VG_EINVAL;
    }
    drop_graphs(h);
    h->fields = (char *)fields_d;
    h->alt = (char *)alt_d;
    h->work = (char *)work_d;
    layout(h, h->work);
    h->cur = 0;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = hip_status(hipMemcpyAsync(h->piece_first, h->piece_first_h.data(), sizeof(int32_t) * h->piece_first_h.size(),
                                        hipMemcpyHostToDevice, s), "upload tiles"))) return rc;
    if ((rc = hip_status(hipMemcpyAsync(h->piece_lo, h->piece_lo_h.data(), sizeof(int64_t) * h->piece_lo_h.size(),
                                        hipMemcpyHostToDevice, s), "upload pieces"))) return rc;
    if (h->npieces > 0 &&
        (rc = hip_status(hipMemcpyAsync(h->piece_seg, h->piece_seg_h.data(), sizeof(int32_t) * h->piece_seg_h.size(),
                                        hipMemcpyHostToDevice, s), "upload piece segments"))) return rc;
    if ((rc = hip_status(hipMemcpyAsync(h->seg_first, h->seg_first_h.data(), sizeof(int32_t) * h->seg_first_h.size(),
                                        hipMemcpyHostToDevice, s), "upload segments"))) return rc;
    if ((rc = hip_status(hipMemcpyAsync(h->chunk_first, h->chunk_first_h.data(), sizeof(int32_t) * h->chunk_first_h.size(),
                                        hipMemcpyHostToDevice, s), "upload chunks"))) return rc;
    if ((rc = hip_status(hipMemcpyAsync(h->seg_chunk, h->seg_chunk_h.data(), sizeof(int32_t) * h->seg_chunk_h.size(),
                                        hipMemcpyHostToDevice, s), "upload segment chunks"))) return rc;
    if (h->prec == VG_F32C && h->n > 0) {   // the fields hold the initial state exactly
        if ((rc = hip_status(hipMemsetAsync(h->lo, 0, sizeof(int16_t) * VG_NPOOL * (size_t)h->n, s), "clear words")))
            return rc;
        if ((rc = hip_status(hipMemsetAsync(h->lo_alt, 0, sizeof(int16_t) * (h->mobile_all ? VG_NPOOL : 1) * (size_t)h->n, s),
                             "clear words")))
            return rc;
    }
    if ((rc = launch_geometry(h, s))) return rc;
    if ((rc = build_offsets(h, s))) return rc;
    if ((rc = build_band(h, s))) return rc;
    if ((h->features & VG_FEAT_MG) && (rc = mg_build(h, s))) return rc;
    // the host tables must outlive the asynchronous copies
    if ((rc = hip_status(hipStreamSynchronize(s), "synchronise"))) return rc;
    h->bound = true;
    return VG_OK;
}

extern "C" int vg_step_explicit(vg_sim *h, int64_t nsteps, double dt, int64_t log_every, double *totals_log_d,
                                unsigned flags, void *stream) {
    int rc;
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt) || log_every < 0) {
        set_error("need nsteps >= 0, dt > 0, log_every >= 0");
        return VG_EINVAL;
    }
    const int64_t nlog = log_every > 0 ? nsteps / log_every : 0;
    if (nlog > 0 && !totals_log_d) { set_error("totals_log_d is NULL"); return VG_EINVAL; }
    if (flags & ~VG_FORCE) { set_error("unknown flags"); return VG_EINVAL; }
    if (!(flags & VG_FORCE) && (rc = check_stable(h, dt))) return rc;
    if ((rc = need_bound(h))) return rc;
    if (nsteps == 0 || h->n == 0) return VG_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t row = (size_t)h->nseg * 6;
    auto logged = [&](int64_t j) { return log_every > 0 && j % log_every == 0; };
    // the partials of up to tot_batch logged passes wait in their slots and
    // are reduced by one launch (rows first_row ..)
    int64_t first_row = 0;
    h->part_slot = 0;
    auto flush = [&]() -> int {
        const int rows = h->part_slot;
        h->part_slot = 0;
        const int rc2 = launch_totals_finalize(h, totals_log_d + (size_t)first_row * row, rows, s);
        first_row += rows;
        return rc2;
    };
    auto finalize = [&](int64_t) -> int {
        if (++h->part_slot < h->tot_batch) return VG_OK;
        return flush();
    };
    // four fused passes j .. j + 3 with no totals logged run as two band
    // launches when the band kernel applies
    const bool band = use_band(h);
    auto quiet = [&](int64_t j, int64_t last, int64_t len) {
        if (j + len - 1 > last) return false;
        if (log_every > 0 && (j + log_every - 1) / log_every * log_every <= j + len - 1) return false;
        return true;
    };
    auto quiet4 = [&](int64_t j, int64_t last) { return band && quiet(j, last, 4); };
    // longer quiet runs are replayed from a captured graph
    const bool graphs = graphs_wanted(h);
    auto quiet_run = [&](int64_t j, int64_t last) { return graphs && quiet(j, last, kRunPasses); };
    if (h->params.step_order == VG_ORDER_TD) {
        if ((rc = launch_pass(h, MODE_T, TOT_NONE, dt, s))) return rc;
        for (int64_t j = 1; j < nsteps; j++) {
            if (quiet_run(j, nsteps - 1)) {
                if ((rc = launch_run(h, dt, band, s))) return rc;
                j += kRunPasses - 1;
                continue;
            }
            if (quiet4(j, nsteps - 1)) {
                if ((rc = launch_band_quad(h, dt, s))) return rc;
                j += 3;
                continue;
            }
            const bool lg = logged(j);
            if ((rc = launch_pass(h, MODE_DT, lg ? TOT_MID : TOT_NONE, dt, s))) return rc;
            if (lg && (rc = finalize(j))) return rc;
        }
        const bool lg = logged(nsteps);
        if ((rc = launch_pass(h, MODE_D, lg ? TOT_OUT : TOT_NONE, dt, s))) return rc;
        if (lg && (rc = finalize(nsteps))) return rc;
    } else {
        for (int64_t j = 1; j <= nsteps; j++) {
            if (quiet_run(j, nsteps)) {
                if ((rc = launch_run(h, dt, band, s))) return rc;
                j += kRunPasses - 1;
                continue;
            }
            if (quiet4(j, nsteps)) {
                if ((rc = launch_band_quad(h, dt, s))) return rc;
                j += 3;
                continue;
            }
            const bool lg = logged(j);
            if ((rc = launch_pass(h, MODE_DT, lg ? TOT_OUT : TOT_NONE, dt, s))) return rc;
            if (lg && (rc = finalize(j))) return rc;
        }
    }
    if ((rc = flush())) return rc;
    return restore_canonical(h, s);
}

extern "C" int vg_step_subcycled(vg_sim *h, int64_t n_t, double dt_t, double dt_d, unsigned flags, void *stream) {
    int rc;
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (n_t < 0 || !(dt_t > 0) || !std::isfinite(dt_t) || !(dt_d > 0) || !std::isfinite(dt_d)) {
        set_error("need n_t >= 0, dt_t > 0, dt_d > 0");
        return VG_EINVAL;
    }
    if (flags & ~VG_FORCE) { set_error("unknown flags"); return VG_EINVAL; }
    if (!(flags & VG_FORCE) && (rc = check_stable(h, dt_d))) return rc;
    if ((rc = need_bound(h))) return rc;
    if (n_t == 0 || h->n == 0) return VG_OK;
    hipStream_t s = (hipStream_t)stream;
    // The steps in the order of their start times (a transformation first on
    // ties); a diffusion step followed by a transformation step is one fused
    // pass (diffuse, then transform: exactly the two steps in that order).
    const double t_end = (double)n_t * dt_t;
    int64_t kt = 0, kd = 0;
    auto next_is_t = [&]() -> int {   // 1: transformation, 0: diffusion, -1: done
        const bool more_t = kt < n_t, more_d = (double)kd * dt_d < t_end;
        if (!more_t && !more_d) return -1;
        return (more_t && (!more_d || (double)kt * dt_t <= (double)kd * dt_d)) ? 1 : 0;
    };
    for (int e = next_is_t(); e >= 0; e = next_is_t()) {
        if (e == 1) {
            if ((rc = launch_pass2(h, MODE_T, TOT_NONE, dt_t, dt_d, s))) return rc;
            kt++;
            continue;
        }
        const double sd = (double)kd * dt_d;
        const double len = (double)(kd + 1) * dt_d <= t_end ? dt_d : t_end - sd;
        kd++;
        if (next_is_t() == 1) {
            if ((rc = launch_pass2(h, MODE_DT, TOT_NONE, dt_t, len, s))) return rc;
            kt++;
        } else {
            if ((rc = launch_pass2(h, MODE_D, TOT_NONE, dt_t, len, s))) return rc;
        }
    }
    return restore_canonical(h, s);
}

extern "C" int vg_mass_totals(vg_sim *h, double *out_h, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (!out_h) { set_error("out_h is NULL"); return VG_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (h->n == 0) {
        for (int i = 0; i < h->nseg * 6; i++) out_h[i] = 0.0;
        return VG_OK;
    }
    h->part_slot = 0;
    if ((rc = launch_pass(h, MODE_NONE, TOT_IN, 1.0, s))) return rc;
    if ((rc = launch_totals_finalize(h, h->tot_tmp, 1, s))) return rc;
    if ((rc = hip_status(hipMemcpyAsync(out_h, h->tot_tmp, sizeof(double) * 6 * (size_t)h->nseg, hipMemcpyDeviceToHost, s),
                         "copy totals"))) return rc;
    if ((rc = hip_status(hipStreamSynchronize(s), "synchronise"))) return rc;
    for (int i = 0; i < h->nseg * 6; i++)
        if (!std::isfinite(out_h[i])) { set_error("total %d of segment %d is not finite", i % 6, i / 6); return VG_ENONFINITE; }
    return VG_OK;
}

extern "C" int vg_solve_implicit_step(vg_sim *h, double dt, double rtol, int max_iter, int *iters_h, double *relres_h,
                                      void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (!(h->features & VG_FEAT_CG)) { set_error("handle created without VG_FEAT_CG"); return VG_ESTATE; }
    if (!(dt > 0) || !std::isfinite(dt) || !(rtol > 0) || max_iter < 0) {
        set_error("need dt > 0, rtol > 0, max_iter >= 0");
        return VG_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if ((rc = launch_pass(h, MODE_T, TOT_NONE, dt, s))) return rc;
    int status = VG_OK;
    for (int p = 0; p < VG_NPOOL; p++) {
        int it = 0;
        double rr = 0.0;
        if (h->params.D[p] > 0) {
            const double a = h->params.D[p] * dt / (h->params.h * h->params.h);
            rc = run_cg(h, p, a, rtol, max_iter, &it, &rr, s);
            if (rc == VG_ENOCONV) status = VG_ENOCONV;
            else if (rc) return rc;
        }
        if (iters_h) iters_h[p] = it;
        if (relres_h) relres_h[p] = rr;
    }
    if (status == VG_ENOCONV) set_error("CG reached max_iter = %d above rtol = %g", max_iter, rtol);
    if ((rc = hip_status(hipStreamSynchronize(s), "synchronise"))) return rc;
    return status;
}

extern "C" int vg_set_preconditioner(vg_sim *h, int which) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    if (which != VG_PRECOND_JACOBI && which != VG_PRECOND_MG) { set_error("unknown preconditioner"); return VG_EINVAL; }
    if (which == VG_PRECOND_MG && !(h->features & VG_FEAT_MG)) {
        set_error("the multigrid preconditioner needs a handle created with VG_FEAT_MG");
        return VG_EINVAL;
    }
    h->precond = which;
    return VG_OK;
}

extern "C" int vg_mg_levels(const vg_sim *h, int *levels, int64_t *cells_h) {
    if (!h || !levels) { set_error("null pointer argument"); return VG_EINVAL; }
    *levels = h->mg_levels;
    if (cells_h)
        for (int l = 0; l < VG_MG_MAX_LEVELS; l++) cells_h[l] = l < h->mg_levels ? h->mg[l].n : 0;
    return VG_OK;
}

extern "C" int vg_precondition(vg_sim *h, double a, const double *r_d, double *z_d, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (!(h->features & VG_FEAT_CG)) { set_error("handle created without VG_FEAT_CG"); return VG_ESTATE; }
    if (!(a >= 0) || !std::isfinite(a)) { set_error("need a finite a >= 0"); return VG_EINVAL; }
    if (h->n > 0 && (!r_d || !z_d || r_d == z_d)) { set_error("need distinct r_d and z_d"); return VG_EINVAL; }
    return mg_apply(h, a, r_d, z_d, (hipStream_t)stream);
}

extern "C" int vg_record(vg_sim *h, int64_t nsteps, double dt, void *states_d, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (!(h->features & VG_FEAT_ADJ)) { set_error("handle created without VG_FEAT_ADJ"); return VG_ESTATE; }
    if (h->params.step_order != VG_ORDER_TD) { set_error("the adjoint supports the paper order only"); return VG_EINVAL; }
    if (h->params.sequential) { set_error("the adjoint follows Algorithm 1 only"); return VG_EINVAL; }
    if (nsteps < 0 || !(dt > 0) || (nsteps > 0 && h->n > 0 && !states_d)) { set_error("bad record arguments"); return VG_EINVAL; }
    return launch_record(h, nsteps, dt, states_d, (hipStream_t)stream);
}

extern "C" int vg_tape_rows(const vg_sim *h) {
    if (!h) { set_error("handle is NULL"); return VG_EINVAL; }
    return tape_rows(h);
}

extern "C" int vg_step_record(vg_sim *h, int64_t nsteps, double dt, void *states_d, double *totals_log_d,
                              unsigned flags, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (!(h->features & VG_FEAT_ADJ)) { set_error("handle created without VG_FEAT_ADJ"); return VG_ESTATE; }
    if (h->params.step_order != VG_ORDER_TD) { set_error("the adjoint supports the paper order only"); return VG_EINVAL; }
    if (h->params.sequential) { set_error("the adjoint follows Algorithm 1 only"); return VG_EINVAL; }
    if (flags & ~VG_FORCE) { set_error("unknown flags"); return VG_EINVAL; }
    if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt) ||
        (nsteps > 0 && h->n > 0 && (!states_d || !totals_log_d))) {
        set_error("bad step-record arguments");
        return VG_EINVAL;
    }
    if (!(flags & VG_FORCE) && (rc = check_stable(h, dt))) return rc;
    if (nsteps == 0 || h->n == 0) return VG_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t row = (size_t)h->nseg * 6;
    const int64_t n = h->n;
    const size_t esz = h->elem();
    // states[0] = x^k0, states[j] = T(D(states[j-1])) (T alone for j = 1);
    // the fused pass j >= 2 sees x^(k0+j-1) between its halves: row j-2
    if ((rc = launch_record(h, 1, dt, states_d, s))) return rc;
    int64_t first_row = 0;   // batched totals as in vg_step_explicit
    h->part_slot = 0;
    auto flush = [&]() -> int {
        const int rows = h->part_slot;
        h->part_slot = 0;
        const int rc2 = launch_totals_finalize(h, totals_log_d + (size_t)first_row * row, rows, s);
        first_row += rows;
        return rc2;
    };
    auto logged = [&]() -> int { return ++h->part_slot < h->tot_batch ? VG_OK : flush(); };
    // the passes of vg_record (with the diffused DOM kept, each fused pass
    // writes D(states[j-1])'s DOM into states[j-1])
    const void *src[VG_NPOOL];
    void *dst[VG_NPOOL];
    void *xdom;
    for (int64_t j = 1; j < nsteps; j++) {
        tape_pass_bufs(h, states_d, j - 1, src, dst, &xdom);
        if ((rc = launch_pass_bufs(h, j == 1 ? MODE_T : MODE_DT, j == 1 ? TOT_NONE : TOT_MID, dt, src, dst, s, xdom)))
            return rc;
        if (j >= 2 && (rc = logged())) return rc;
    }
    // the last two steps into the bound fields (canonical between calls):
    // T(D(states[nsteps-1])) (T alone when nsteps = 1), then D
    {
        tape_pass_bufs(h, states_d, nsteps - 1, src, dst, &xdom);
        for (int p = 0; p < VG_NPOOL; p++) dst[p] = h->fields + (size_t)p * n * esz;
        const bool one = nsteps == 1;
        if ((rc = launch_pass_bufs(h, one ? MODE_T : MODE_DT, one ? TOT_NONE : TOT_MID, dt, src, dst, s, xdom)))
            return rc;
        if (!one && (rc = logged())) return rc;
    }
    if ((rc = launch_pass(h, MODE_D, TOT_OUT, dt, s))) return rc;
    if ((rc = logged())) return rc;
    if ((rc = flush())) return rc;
    return restore_canonical(h, s);
}

extern "C" int vg_adjoint(vg_sim *h, int64_t nsteps, double dt, const void *states_d, const double *seeds_d,
                          void *lambda_d, double *grad_d, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (!(h->features & VG_FEAT_ADJ)) { set_error("handle created without VG_FEAT_ADJ"); return VG_ESTATE; }
    if (h->params.step_order != VG_ORDER_TD) { set_error("the adjoint supports the paper order only"); return VG_EINVAL; }
    if (h->params.sequential) { set_error("the adjoint follows Algorithm 1 only"); return VG_EINVAL; }
    if (nsteps < 0 || !(dt > 0)) { set_error("need nsteps >= 0 and dt > 0"); return VG_EINVAL; }
    if (nsteps > 0 && h->n > 0 && (!states_d || !seeds_d || !lambda_d || !grad_d)) {
        set_error("null pointer argument");
        return VG_EINVAL;
    }
    return launch_adjoint(h, nsteps, dt, states_d, seeds_d, lambda_d, grad_d, (hipStream_t)stream);
}

extern "C" int vg_seed_lambda(vg_sim *h, const double *seed_d, void *lambda_d, int zero, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (h->n > 0 && (!seed_d || !lambda_d)) { set_error("null pointer argument"); return VG_EINVAL; }
    return launch_seed(h, seed_d, lambda_d, zero, (hipStream_t)stream);
}

extern "C" int vg_load_state(vg_sim *h, const void *x_d, int x_precision, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (x_precision != VG_F32 && x_precision != VG_F64) { set_error("x_precision must be VG_F32 or VG_F64"); return VG_EINVAL; }
    if (h->n > 0 && !x_d) { set_error("x_d is NULL"); return VG_EINVAL; }
    return launch_load_state(h, x_d, x_precision, (hipStream_t)stream);
}

extern "C" int vg_store_state(vg_sim *h, void *x_d, int x_precision, void *stream) {
    int rc = need_bound(h);
    if (rc) return rc;
    if (x_precision != VG_F32 && x_precision != VG_F64) { set_error("x_precision must be VG_F32 or VG_F64"); return VG_EINVAL; }
    if (h->n > 0 && !x_d) { set_error("x_d is NULL"); return VG_EINVAL; }
    return launch_store_state(h, x_d, x_precision, (hipStream_t)stream);
}
