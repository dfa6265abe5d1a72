/*
 * vgsim.h -- C ABI of the MI355X (gfx950) voxel-graph diffusion-transformation
 * library (method of Klai, Monga, Jouini, Pot, arXiv:2406.04177).
 *
 * The library simulates five carbon pools on the graph of 6-connected pore
 * voxels of a binary 3D image: per voxel a transformation step (Sec. II.C,
 * eq. (3), with the clamps of Appendix A, Algorithm 1) and Fick diffusion
 * between face-neighbours, explicit (Sec. II.B.3a, Scheme 1) or implicit with
 * Jacobi-preconditioned conjugate gradients (Sec. II.B.3b, Scheme 2; Sec. III).
 * It also provides the discrete adjoint of the explicit time loop.
 *
 * Conventions (every entry point)
 *   - Returns VG_OK (0) or a negative VG_E* code; vg_last_error() gives text.
 *     Nothing throws or exits across the ABI.
 *   - Pointers named *_d are device pointers owned by the caller; the library
 *     never allocates, frees or keeps device memory beyond what the caller
 *     binds.  Host pointers (*_h and descriptor arrays) are read during the
 *     call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = legacy default
 *     stream).  Device work is enqueued asynchronously on it; calls that return
 *     a host value (vg_count_pores, vg_mass_totals, vg_solve_implicit_step)
 *     synchronise that stream before returning.
 *   - A vg_sim handle is not thread-safe; do not use one handle from two host
 *     threads or two streams at once.
 *   - Pools are numbered in the paper's order: 0 MB, 1 DOM, 2 SOM, 3 FOM
 *     (called P4 here), 4 CO2.  Fields are structure-of-arrays: pool s of
 *     voxel i is at fields[s * n + i].
 *   - Geometry: masks are uint8 [nz][ny][nx], nonzero = pore (the paper tags
 *     pore voxels with 0, Sec. II.A).  The linear index of (x, y, z) is
 *     x + nx * (y + ny * z).
 */
#ifndef VGSIM_H
#define VGSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define VG_OK          0
#define VG_EINVAL     -1   /* bad argument: null pointer, size, range, shape  */
#define VG_EUNSTABLE  -2   /* explicit dt above the positivity bound         */
#define VG_ENOCONV    -3   /* CG stopped at max_iter above rtol              */
#define VG_ENONFINITE -4   /* a mass total is NaN or infinite                */
#define VG_EHIP       -5   /* HIP runtime error (text in vg_last_error)      */
#define VG_ESTATE     -6   /* call out of sequence (e.g. no state bound)     */

/* ---- enumerations ------------------------------------------------------ */
#define VG_F32 0           /* fields stored and stepped in float32           */
#define VG_F64 1           /* fields stored and stepped in float64           */
/* Compensated float32: every pool value is held as the float hi nearest to
 * it (the bound fields, readable as plain float32) plus a 16-bit word
 * lo = (x - hi) / ulp(hi) * 2^15 rounded to an integer (|lo| <= 2^14, kept in
 * the workspace), i.e. a 39-bit significand in 6 bytes; the arithmetic of a
 * step runs in FP64 and each stored value rounds by at most 2^-39 relative
 * instead of 2^-24.  Over k steps the drift of plain float32 (slow pools
 * such as MB, SOM and CO2 change by ~1e-7 of themselves per step, about one
 * float32 rounding, Sec. II.C eq. (3)) is thereby cut by 2^15.  Covers the
 * explicit and sub-cycled steps, the totals and the implicit step; no
 * adjoint (VG_FEAT_ADJ), no rank-index or band kernel (the table or a packed
 * neighbour source is used).  Set a state with more than float32 precision
 * with vg_load_state, read it with vg_store_state. */
#define VG_F32C 2

#define VG_PERIODIC_X 1u   /* wrap-around neighbours (tests); default no-flux */
#define VG_PERIODIC_Y 2u
#define VG_PERIODIC_Z 4u

#define VG_ORDER_TD 0      /* paper order: transformation, then diffusion    */
#define VG_ORDER_DT 1      /* diffusion, then transformation                 */

#define VG_FORCE 1u        /* vg_step_explicit: skip the dt stability check  */

#define VG_NPOOL 5
#define VG_NREG 8          /* region conductance factors: volume octants     */
#define VG_NGRAD 20        /* gradient vector length, layout below           */

/* Model parameters, SI units.  a_s = D[s] * dt / h^2 is the dimensionless
 * diffusion number of pool s (voxel units give S_ij = d_ij = 1, Sec. II.B.2).
 * mort_to_p4 = 0 routes a fraction beta of dead biomass to DOM and 1 - beta to
 * SOM (Sec. II.C); 1 routes all of it to pool 3.  sequential = 0 transforms
 * with Appendix A Algorithm 1 (every flux from the pre-step masses, clamped,
 * then applied); 1 with Algorithm 2 (uptake, mortality, respiration, SOM and
 * FOM turnover one after the other, each on what the previous left, a
 * process taking at most all of its source pool; the printed algorithm's
 * slips read as corrected: each turnover is compared with its own pool,
 * moved to DOM before the pool is zeroed, and MB is zeroed when it all
 * dies).  The adjoint follows Algorithm 1 only. */
typedef struct vg_params {
    double D[VG_NPOOL];
    double h;
    double v_dom, k_dom, rho, mu, beta, v_som, v_p4;
    int32_t mort_to_p4;
    int32_t step_order;   /* VG_ORDER_TD or VG_ORDER_DT */
    int32_t sequential;   /* 0: Algorithm 1, 1: Algorithm 2 */
} vg_params;

/* ---- errors ------------------------------------------------------------ */
const char *vg_strerror(int code);
/* Text of the last error raised on the calling thread ("" if none). */
const char *vg_last_error(void);
int vg_version(void);

/* ---- graph construction (Sec. II.A, Fig. 2; Sec. III) -------------------
 * The pore voxels are enumerated in raster order (x fastest) or, with
 * brick = b > 0, brick by brick (bricks of b^3 voxels in raster order of
 * bricks, raster order inside a brick).  The enumeration is held in a "rank
 * index": one 32-bit pore bitmap word per 32 positions of the enumeration plus
 * the number of pore voxels before that word.  */

/* Bytes of the rank index for this shape and brick size. */
int vg_rank_bytes(int nx, int ny, int nz, int brick, size_t *bytes);

/* Builds the rank index of mask_d into rank_d (vg_rank_bytes bytes) and
 * returns the number of pore voxels in *n_out (host).  Synchronises stream. */
int vg_count_pores(const uint8_t *mask_d, int nx, int ny, int nz, int brick, void *rank_d,
                   int64_t *n_out, void *stream);

/* Fills the compacted pore-voxel list and neighbour table of one volume.
 *   vox_d[i]            linear index of compact voxel i (i < n)
 *   nbr_d[k * ld + i]   index_base + compact index of the neighbour in slot
 *                       k = (-x, +x, -y, +y, -z, +z), or -1 when that voxel
 *                       is solid or outside the box (no-flux faces), unless
 *                       the axis is in `periodic`.
 * n must be the count from vg_count_pores; ld >= n is the row stride of the
 * table (the total voxel count when several volumes share one table). */
int vg_build_graph(const void *rank_d, int nx, int ny, int nz, int brick, unsigned periodic,
                   int32_t index_base, int64_t n, int64_t ld, int32_t *vox_d, int32_t *nbr_d,
                   void *stream);

/* idx_d[q] = index_base + compact index of linear voxel lin_d[q], or -1 if
 * that voxel is solid or out of range. */
int vg_lookup(const void *rank_d, int nx, int ny, int nz, int brick, const int64_t *lin_d,
              int64_t count, int32_t index_base, int32_t *idx_d, void *stream);

/* Region code of every voxel for the region conductance factors: bits 0-2
 * the octant 4[z >= nz/2] + 2[y >= ny/2] + [x >= nx/2] of the voxel, bit 3+k
 * set when the neighbour position in slot k lies in another octant.  The
 * edge weight is w_ij = (c[octant(i)] + c[octant(j)]) / 2 (a generalisation
 * of the unit conductance S_ij / d_ij = 1 of Sec. II.B.2). */
int vg_region_codes(const int32_t *vox_d, int64_t n, int nx, int ny, int nz, unsigned periodic,
                    uint16_t *codes_d, void *stream);

/* Sums of x_d[0..n) over contiguous ranges: out_d[r] = sum of x_d[i] for
 * offsets_d[r] <= i < offsets_d[r+1] (r < nranges), FP64, in a fixed order.
 * x_d is float or double (precision VG_F32 / VG_F64), e.g. one pool of the
 * fields; offsets_d holds nranges + 1 int64 on the device (clamped into
 * [0, n]; an empty or inverted range sums to 0).  In raster order every
 * z-layer of a volume is one range, so this gives the mass profile per layer
 * of the diffusion comparison of Sec. IV.B. */
int vg_range_sums(const void *x_d, int precision, int64_t n, const int64_t *offsets_d, int64_t nranges,
                  double *out_d, void *stream);

/* ---- pore-network (PNGM) objectives on a brick partition (Sec. V) -------
 * The primitives are the bricks of side b of the image; a primitive holds the
 * pore voxels of its brick (v_i of them), two primitives are adjacent when a
 * pore-voxel face joins them, with contact surface S_ij = the number of such
 * faces and d_ij = the distance between their centres of gravity (the
 * paper's primitives are maximal balls; its starting conductances are
 * S_ij / d_ij, Sec. V.B). */

/* Per brick k (raster order of bricks, nbx = ceil(nx / b) ...):
 * sums_d[k][0..3] = pore voxels, sums of their x, y, z; contact_d[k][a] =
 * pore-voxel faces shared with brick k + 1 along axis a (x, y, z).  vox_d /
 * nbr_d as from vg_build_graph (any enumeration, no periodic axis).  Both
 * outputs are cleared first (uint32 [nb][3], uint64 [nb][4]). */
int vg_brick_stats(const int32_t *vox_d, const int32_t *nbr_d, int64_t n, int nx, int ny, int nz, int b,
                   uint32_t *contact_d, unsigned long long *sums_d, void *stream);

/* The primitive graph of the brick partition, assembled on the device
 * (Sec. V.B's primitives, their volumes, contact surfaces and centroid
 * distances, from which the starting conductances S_ij / d_ij follow).
 * vg_pngm_partition_bytes gives the workspace size and the capacities the
 * outputs need: max_prims = the number of bricks, max_edges = twice the
 * number of face-adjacent brick pairs.  vg_pngm_partition then writes, for
 * q primitives (the bricks holding pore voxels, in raster order of bricks)
 * and E directed edges:
 *   v_d [q]          pore voxels per primitive (FP64)
 *   offsets_d [q+1]  start of each primitive's range in a compacted list
 *                    enumerated brick by brick with bricks of side b
 *   bricks_d [q]     brick index (raster order of bricks) of each primitive
 *   row_d [q+1], col_d [E]  adjacency in CSR, columns ascending
 *   S_d [E]          pore-voxel faces joining the two primitives (FP64)
 *   dist_d [E]       distance of their centres of gravity in voxels,
 *                    sqrt((dx^2 + dy^2) + dz^2) of centroids = coordinate
 *                    sums / counts (FP64)
 * and q, E to *q_out, *e_out (host).  vox_d / nbr_d as for vg_brick_stats
 * (any enumeration of one volume, no periodic axis).  The workspace (work_d,
 * work_bytes) holds the brick statistics and is overwritten.  Synchronises
 * the stream.  VG_EINVAL for a null pointer, a bad shape or a short
 * workspace. */
int vg_pngm_partition_bytes(int nx, int ny, int nz, int b, size_t *work_bytes, int64_t *max_prims,
                            int64_t *max_edges);
int vg_pngm_partition(const int32_t *vox_d, const int32_t *nbr_d, int64_t n, int nx, int ny, int nz, int b,
                      void *work_d, size_t work_bytes, double *v_d, int64_t *offsets_d, int32_t *bricks_d,
                      int64_t *row_d, int32_t *col_d, double *S_d, double *dist_d, int64_t *q_out,
                      int64_t *e_out, void *stream);

/* Objective 1 (objective = 1: residual of the explicit scheme 3,
 * r_i = y_i - x_i + c sum_j theta_ij (x_i/v_i - x_j/v_j)) or objective 2 (the
 * implicit scheme 4, r_i = x_i - y_i - c sum_j theta_ij (y_i/v_i - y_j/v_j)),
 * L = mean over data pairs and primitives of r_i^2, c = D dt (voxel units),
 * over l data pairs X_d, Y_d ([l][q] FP64 primitive masses at t and t + dt).
 * Adjacency as CSR: row_d [q+1] int64, col_d [E] int32, theta_d [E] FP64 (one
 * parameter per ordered pair, in row i only).  Writes loss_d[0], grad_d [E]
 * (dL/dtheta) and rowloss_d [q] (each row's share, summed in a fixed order).
 * The inner term is x_j / v_j and dL2/dtheta has the minus sign of the
 * residual's derivative (the printed formulas slip on both). */
int vg_pngm_loss_grad(const double *X_d, const double *Y_d, int64_t l, int64_t q, const double *v_d,
                      const int64_t *row_d, const int32_t *col_d, const double *theta_d, double c, int objective,
                      double *rowloss_d, double *loss_d, double *grad_d, void *stream);

/* One explicit PNGM step (scheme 3): out_i = m_i - c sum_j theta_ij
 * (m_i/v_i - m_j/v_j); out_d must not alias m_d. */
int vg_pngm_step(const double *m_d, double *out_d, int64_t q, const double *v_d, const int64_t *row_d,
                 const int32_t *col_d, const double *theta_d, double c, void *stream);

/* One implicit PNGM step (scheme 4, Sec. V.A): out_d = the masses y solving
 * y_i + c sum_j theta_ij (y_i/v_i - y_j/v_j) = m_i.  Solved by Jacobi sweeps
 * on the concentrations y/v (each row is strictly diagonally dominant since
 * v_i > 0, so the sweeps converge), starting from m/v, until the residual
 * ||m - A y||_2 <= rtol ||m||_2 (checked every 8 sweeps, one host sync each).
 * work_d: caller-owned FP64 scratch of 3 q + 2 entries.  iters_out /
 * relres_out (host): sweeps taken and the result's relative residual.
 * Returns VG_ENOCONV when max_iter sweeps end above rtol (out_d then holds
 * the last checked iterate).  out_d must not alias m_d or work_d. */
int vg_pngm_implicit_step(const double *m_d, double *out_d, int64_t q, const double *v_d, const int64_t *row_d,
                          const int32_t *col_d, const double *theta_d, double c, double rtol, int max_iter,
                          double *work_d, int *iters_out, double *relres_out, void *stream);

/* For callers that cannot allocate device memory (or hand the library a
 * scratch buffer): vg_pngm_implicit_step with its 3 q + 2 FP64 scratch
 * entries in a static device array of the library instead of work_d, so the
 * call allocates nothing.  Same kernels, same results.  q is at most
 * VG_PNGM_NOALLOC_MAX_Q (larger q returns VG_EINVAL); the array
 * (3 * 65536 + 2 doubles, 1.5 MiB) exists once per GPU and is held until the
 * process ends.  All calls on one GPU share it: calls that overlap on one GPU
 * (other streams or host threads) race.  Nothing in it needs to start at
 * zero: every entry is written before it is read. */
#define VG_PNGM_NOALLOC_MAX_Q 65536
int vg_pngm_implicit_step_noalloc(const double *m_d, double *out_d, int64_t q, const double *v_d,
                                  const int64_t *row_d, const int32_t *col_d, const double *theta_d, double c,
                                  double rtol, int max_iter, int *iters_out, double *relres_out, void *stream);

/* The normalised-gradient step of Sec. V.A on count parameters:
 * theta_e <- clamp(theta_e - lr * scale_e * sign(grad_e), lo_e, hi_e), no move
 * for a zero derivative (FP64 device arrays). */
int vg_sign_update(double *theta_d, const double *grad_d, int64_t count, double lr, const double *scale_d,
                   const double *lo_d, const double *hi_d, void *stream);

/* ---- simulation handle ------------------------------------------------- */
typedef struct vg_sim vg_sim;

typedef struct vg_desc {
    int64_t n;               /* pore voxels over all volumes                 */
    int32_t nseg;            /* volumes (segments of the compact list)       */
    int32_t precision;       /* VG_F32, VG_F64 or VG_F32C                    */
    const int64_t *seg_off;  /* host [nseg + 1], seg_off[0] = 0, [nseg] = n  */
    const int32_t *nbr_d;    /* device [6][n] neighbour table                */
    const uint16_t *rcode_d; /* device [n] region codes or NULL (weights 1)  */
    int32_t mobile_all;      /* 0: only DOM may diffuse; 1: any pool may     */
    int32_t features;        /* VG_FEAT_CG | VG_FEAT_ADJ | VG_FEAT_BAND      */
    /* Optional, single volume (nseg == 1) only: the rank index built by
     * vg_count_pores for the same mask, shape, brick and periodic flags as
     * nbr_d, and the compacted list vox_d.  With them (and no periodic axis,
     * every dimension <= 1024) the explicit step finds neighbours from the
     * pore bitmap (about 46 B per voxel and step instead of 64 B); the
     * workspace then holds a 4-byte geometry word per voxel.  NULL = table. */
    const void *rank_d;
    const int32_t *vox_d;
    int32_t nx, ny, nz;      /* volume shape of rank_d                       */
    int32_t brick;           /* enumeration of rank_d (0 raster)             */
    uint32_t periodic;       /* VG_PERIODIC_* flags the table was built with */
} vg_desc;

#define VG_FEAT_CG   1
#define VG_FEAT_ADJ  2
/* Two explicit steps per pass (VG_KERNEL_BAND): for a single raster-order
 * volume with no periodic axis and a rank index (rank_d, vox_d), the
 * workspace also holds a row index ((nz * ny + 1) int32) and a second set of
 * the five fields (5 n elements of the field type). */
#define VG_FEAT_BAND 4
/* Workspace for the multigrid preconditioner (vg_set_preconditioner): needs
 * VG_FEAT_CG and a single volume with a rank index (rank_d, vox_d) and no
 * periodic axis.  Holds the hierarchy, at most about 100 B per cell of the
 * grid of half the resolution (the bound assumes every 2x2x2 block holds a
 * pore voxel), built by vg_init_state. */
#define VG_FEAT_MG   8

/* Creates a handle (host memory only) and sets default parameters. */
int vg_create(const vg_desc *desc, vg_sim **out);
int vg_destroy(vg_sim *h);
/* Neighbour source of the explicit-step kernels: VG_KERNEL_TABLE (the 6-slot
 * table), VG_KERNEL_RANK (the rank index; VG_EINVAL without one),
 * VG_KERNEL_OFFSET (two packed 32-bit words of neighbour distances per voxel)
 * or VG_KERNEL_RELATIVE (one 32-bit word of per-slot codes per voxel,
 * relative to per-64-voxel base distances).  vg_init_state builds the last
 * two from the table when no neighbour crosses a periodic wrap and the
 * distances (OFFSET), or their spread within each group of 64 voxels
 * (RELATIVE), fit the packing; choosing one that was not built is VG_EINVAL.
 * VG_KERNEL_AUTO takes the first of RELATIVE, OFFSET, RANK (when the
 * descriptor has a usable rank index) and TABLE that is available.  Results
 * are bit-identical.  vg_get_kernel reports the source the next explicit
 * pass will use. */
#define VG_KERNEL_AUTO     0
#define VG_KERNEL_TABLE    1
#define VG_KERNEL_RANK     2
#define VG_KERNEL_OFFSET   3
#define VG_KERNEL_RELATIVE 4
/* VG_KERNEL_BAND: RELATIVE codes, and runs of four consecutive fused passes
 * (steps with no totals logged) as two launches of a kernel that applies two
 * fused passes (Scheme 1 diffusion, then Algorithm 1, twice) to bands of
 * rows marching along z: the intermediate DOM of a band, its neighbour rows
 * and the planes next to it stay in LDS, so a pass pair reads and writes the
 * fields once.  Needs the workspace of VG_FEAT_BAND and the relative codes;
 * used while only DOM diffuses, with unit edge weights (no region codes) and
 * Algorithm 1; other passes run on RELATIVE.  Bit-identical to RELATIVE.
 * AUTO takes BAND for FP32 fields when it is available and the volume has
 * enough planes for chunks of at least 20 (about 512^3 and up). */
#define VG_KERNEL_BAND     5
int vg_set_kernel(vg_sim *h, int variant);

/* Launching of the explicit step.  Runs of fused passes with no totals
 * logged can be captured once as a HIP graph (on a private stream of the
 * handle, never on the caller's) and replayed on the caller's stream: the
 * same kernels with the same arguments in the same order, so the results
 * are bit-identical; what changes is the launch cost, which bounds small
 * volumes.  A captured run is re-captured after any change of parameters,
 * regions, kernel choice, bound buffers or dt.  VG_LAUNCH_GRAPHS_AUTO
 * (default): graphs for volumes of at most 2^19 pore voxels; _ON: always;
 * _OFF: plain launches. */
#define VG_LAUNCH_GRAPHS_AUTO 0u
#define VG_LAUNCH_GRAPHS_ON   1u
#define VG_LAUNCH_GRAPHS_OFF  2u
int vg_set_launch_options(vg_sim *h, unsigned flags);
int vg_get_kernel(const vg_sim *h, int *variant_in_use);
/* Sets the model parameters (validated: h > 0, K_DOM > 0, rates >= 0,
 * 0 <= beta <= 1, D >= 0; only D[1] may be nonzero unless mobile_all). */
int vg_set_params(vg_sim *h, const vg_params *p);
/* Region conductance factors c[VG_NREG] (> 0); ignored without region codes. */
int vg_set_regions(vg_sim *h, const double *c);

/* Device memory the caller binds with vg_init_state:
 *   fields  [5][n] elements of the field type (float or double; float for
 *           VG_F32C, whose compensation words live in the workspace)
 *   alt     alt_elems elements of the field type (ping-pong of mobile pools)
 *   work    workspace_bytes bytes (reduction partials, packed neighbour
 *           offsets and codes (12.5 B per voxel), geometry words with a rank
 *           index, CG vectors, adjoint ping-pong and gradient partials, as
 *           enabled by `features`). */
int vg_alt_elems(const vg_sim *h, int64_t *elems);
int vg_workspace_bytes(const vg_sim *h, size_t *bytes);

/* Binds the caller's buffers (fields already hold the initial masses),
 * uploads the small per-handle tables into the workspace and builds the
 * derived neighbour data (geometry words, packed offsets) from the graph.
 * Synchronises the stream. */
int vg_init_state(vg_sim *h, void *fields_d, void *alt_d, void *work_d, size_t work_bytes,
                  void *stream);

/* Advances nsteps time steps of the explicit method (Scheme 1 plus the
 * transformation, in params.step_order).  If log_every > 0, the totals of the
 * state after every log_every-th step go to totals_log_d[r][g][0..5]
 * (r = 0 .. nsteps / log_every - 1; pools 0-4 then total carbon, FP64).
 * Returns VG_EUNSTABLE, without stepping, when
 * dt * max_s D_s * 6 * max_r c_r / h^2 > 1, unless flags has VG_FORCE.
 * On return the bound fields hold the new state. */
int vg_step_explicit(vg_sim *h, int64_t nsteps, double dt, int64_t log_every,
                     double *totals_log_d, unsigned flags, void *stream);

/* Unequal time steps for transformation and diffusion (Sec. III: the
 * process with the smaller step is repeated).  Over [0, t_end] with
 * t_end = n_t * dt_t, transformation steps of dt_t start at k dt_t
 * (k < n_t) and Scheme 1 diffusion steps of dt_d start at k dt_d while
 * k dt_d < t_end, the last one shortened to end at t_end.  Each step uses the
 * state at its start, so the steps run in the order of their start times, a
 * transformation first when both start together (dt_t == dt_d reproduces
 * vg_step_explicit in the paper's order).  A diffusion step directly followed
 * by a transformation step runs as one fused pass.  Returns VG_EUNSTABLE,
 * without stepping, when dt_d is above the positivity bound (see
 * vg_step_explicit) unless flags has VG_FORCE.  No totals are logged; on
 * return the bound fields hold the state at t_end. */
int vg_step_subcycled(vg_sim *h, int64_t n_t, double dt_t, double dt_d, unsigned flags, void *stream);

/* One implicit step (Scheme 2): the transformation, then for each pool with
 * D_s > 0 the system (I + a_s L_w) y = x_s solved by preconditioned CG
 * (Jacobi as in the paper, or the multigrid option below) in FP64 (start
 * y = x_s; stop at ||x_s - B y||_2 <= rtol ||x_s||_2).
 * iters_h[5] / relres_h[5] (host, may be NULL) receive the iterations and
 * final relative residual per pool.  Returns VG_ENOCONV if a pool stopped at
 * max_iter (the state still takes the last iterate).  Synchronises stream. */
int vg_solve_implicit_step(vg_sim *h, double dt, double rtol, int max_iter, int *iters_h,
                           double *relres_h, void *stream);

/* Preconditioner of the implicit step's CG.  VG_PRECOND_JACOBI (default):
 * the inverse diagonal of the system matrix, as in Sec. III.
 * VG_PRECOND_MG (an addition to the paper; needs a handle created with
 * VG_FEAT_MG): one V-cycle over aggregates of 2x2x2 cells.  Level l+1 has a
 * cell for every occupied 2x2x2 block of level l's grid (level 0: the pore
 * voxels); its operator is the Galerkin product P^T B P with the piecewise-
 * constant P, i.e. again mass + a * weighted Laplacian, with the number of
 * voxels of a cell as its mass and the summed weights of the edges between
 * two cells as their weight.  Damped Jacobi (omega 0.8) once before and once
 * after each coarse correction, 8 sweeps on the coarsest level (at most 1024
 * cells).  A fixed symmetric positive
 * definite map, so the iteration is still CG with the same stopping rule; it
 * takes far fewer iterations for a = D dt / h^2 >> 1 at about twice the
 * cost of one.  Summation orders are fixed (results do not depend on
 * scheduling).  VG_EINVAL for MG without VG_FEAT_MG; with a grid that cannot
 * be coarsened (one voxel) MG falls back to Jacobi. */
#define VG_PRECOND_JACOBI 0
#define VG_PRECOND_MG     1
int vg_set_preconditioner(vg_sim *h, int which);
/* Levels of the multigrid hierarchy (0 without VG_FEAT_MG) and, if cells_h
 * is not NULL, the cells of each (cells_h[VG_MG_MAX_LEVELS], level 0 = n). */
#define VG_MG_MAX_LEVELS 12
int vg_mg_levels(const vg_sim *h, int *levels, int64_t *cells_h);
/* z = M^-1 r for the system I + a L_w: the current preconditioner applied
 * once (r_d, z_d: device [n] FP64, distinct).  Uses the CG vectors of the
 * workspace (do not overlap with an implicit step on the same handle). */
int vg_precondition(vg_sim *h, double a, const double *r_d, double *z_d, void *stream);

/* Totals of the bound state: out_h[g][0..5] (host), FP64, fixed summation
 * order.  Returns VG_ENONFINITE if any total is not finite.  Synchronises. */
int vg_mass_totals(vg_sim *h, double *out_h, void *stream);

/* Copies a state into the bound fields, converting to the handle's
 * precision: x_d [5][n] of x_precision (VG_F32 or VG_F64) on the device.
 * Float32 fields take the nearest float; compensated fields (VG_F32C) take
 * the nearest float and its compensation word (a VG_F32 source gives zero
 * words).  x_d may be the bound fields themselves (after writing them
 * directly, this clears the compensation words).  Asynchronous. */
int vg_load_state(vg_sim *h, const void *x_d, int x_precision, void *stream);

/* Writes the bound state to x_d [5][n] in x_precision (VG_F32: the float
 * part of compensated fields; VG_F64: the value, for VG_F32C hi + lo ulp(hi)
 * 2^-15, exact).  x_d must not overlap the bound buffers.  Asynchronous. */
int vg_store_state(vg_sim *h, void *x_d, int x_precision, void *stream);

/* ---- discrete adjoint of the explicit loop (paper order only) -----------
 * vg_record advances nsteps steps from the bound state x^k0 and writes what
 * the reverse sweep needs to states_d ([nsteps][rows][n], field type, rows =
 * vg_tape_rows(h)).  Five rows: states[0] = x^k0 and states[j] = T(x^(k0+j-1))
 * for j >= 1 (the state after the transformation half of step k0+j-1).
 * Four rows (the adjoint option VG_ADJ_TAPE_DOM): MB, DOM, SOM, P4 of those
 * states, except that the DOM row of states[j], j >= 1, holds the DOM of
 * x^(k0+j) (after the diffusion half), and no CO2.  The bound fields are left
 * at x^k0 (the call only reads them); the adjoint's own second lambda buffer
 * is overwritten.
 *
 * vg_adjoint runs the reverse sweep over those nsteps steps.
 *   lambda_d [5][n] (field type): in dL/dx^(k0+nsteps), out dL/dx^k0.
 *   seeds_d  [nsteps][nseg][5] FP64: dL/dTotal_{g,s} at steps k0..k0+nsteps-1
 *            (added to lambda after each reverse step; the caller seeds step
 *            k0+nsteps itself, e.g. with vg_seed_lambda).
 *   grad_d   [VG_NGRAD] FP64, accumulated (+=):
 *            [0..4] dL/dD_s, [5] v_DOM, [6] K_DOM, [7] rho, [8] mu, [9] beta,
 *            [10] v_SOM, [11] v_P4, [12..19] dL/dc_r (zero without regions).
 * dt must equal the one used for the forward steps.  Both calls return
 * VG_EINVAL for params.sequential = 1 (the reverse sweep differentiates
 * Algorithm 1) and for the diffuse-first step order. */
int vg_record(vg_sim *h, int64_t nsteps, double dt, void *states_d, void *stream);
/* Rows per recorded state of vg_record, vg_step_record and vg_adjoint under
 * the handle's current adjoint options: 5, or 4 with VG_ADJ_TAPE_DOM (when
 * not every pool diffuses); VG_EINVAL for a NULL handle. */
int vg_tape_rows(const vg_sim *h);
/* The forward run and its record in one: advances the bound state nsteps
 * steps, writes to states_d what vg_record writes for the same start, and
 * logs the totals after every step to totals_log_d[nsteps][nseg][6] (as
 * vg_step_explicit with log_every = 1).  The same kernels in the same order,
 * so the state and the totals are bit-identical to vg_step_explicit's and
 * the states to vg_record's; it lets a caller that can hold the states of a
 * whole segment skip the segment's second forward run.  Same validation as
 * vg_record plus the stability bound (VG_FORCE in flags skips it). */
int vg_step_record(vg_sim *h, int64_t nsteps, double dt, void *states_d, double *totals_log_d, unsigned flags,
                   void *stream);
int vg_adjoint(vg_sim *h, int64_t nsteps, double dt, const void *states_d, const double *seeds_d,
               void *lambda_d, double *grad_d, void *stream);
/* lambda_d[s][i] = (zero ? 0 : lambda_d[s][i]) + seed_d[g(i)][s] (seed_d
 * [nseg][5] FP64 on the device). */
int vg_seed_lambda(vg_sim *h, const double *seed_d, void *lambda_d, int zero, void *stream);

/* Options of vg_adjoint.  VG_ADJ_SKIP_STATIC_D: dL/dD_s is not computed for
 * the pools that do not diffuse in this handle (every pool but DOM unless
 * mobile_all) and grad_d[s] is set to NaN for them; this saves the six
 * neighbour gathers of each of their adjoints per voxel and step.  The other
 * gradients and lambda are unchanged.  Default: every dL/dD_s computed.
 * VG_ADJ_TAPE_DOM (ignored with mobile_all): vg_record and vg_step_record
 * write four rows per recorded state (see vg_record): MB, SOM and P4 of the
 * state and, for j >= 1, the DOM after the diffusion half of the step that
 * follows it (the x^(k0+j) of the paper's order), which the recording pass
 * has at hand; the transformed DOM and CO2 that the recording needs to go on
 * stay in the adjoint's second lambda buffer.  16 B per FP32 voxel and step
 * instead of 20, and vg_adjoint reads each step's x^k directly instead of
 * gathering the stored DOM at six neighbours to form it (Sec. II.B.3a
 * Scheme 1 applied in the forward, not again in the reverse).  lambda and
 * the gradient are bit-identical to the five-row recording.  The flag must
 * be the same for the recording and its vg_adjoint; such states hold no CO2,
 * so vg_adjoint returns VG_EINVAL for them when dL/dD_CO2 is asked for (no
 * VG_ADJ_SKIP_STATIC_D) with a CO2 adjoint that varies within a volume. */
#define VG_ADJ_SKIP_STATIC_D 1u
#define VG_ADJ_TAPE_DOM      2u
int vg_set_adjoint_options(vg_sim *h, unsigned flags);

#ifdef __cplusplus
}
#endif
#endif /* VGSIM_H */
