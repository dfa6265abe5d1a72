/*
 * vg_oracle.c -- plain FP64 CPU oracle of the voxel-graph
 * diffusion-transformation method (Klai, Monga, Jouini, Pot,
 * arXiv:2406.04177).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the HIP path: it is written from the paper, slowly and literally, so that a
 * reader can check every line against the cited passage.
 *
 * Arrays
 *   mask   uint8 [nz][ny][nx], nonzero = pore voxel
 *   vox    int32 [n]       linear index x + nx*(y + ny*z) of compact voxel i
 *   nbr    int32 [6][n]    compact index of the neighbour in slot
 *                          k = (-x, +x, -y, +y, -z, +z), -1 if absent
 *   w      double [6][n]   edge weight per slot (NULL: every weight is 1)
 *   x      double [5][n]   pools MB, DOM, SOM, P4 (the paper's FOM), CO2
 *
 * Parameter vector prm[15]
 *   prm[0..4] D_s (m^2/s)   prm[5] h (m)
 *   prm[6] v_DOM  prm[7] K_DOM  prm[8] rho  prm[9] mu  prm[10] beta
 *   prm[11] v_SOM prm[12] v_FOM prm[13] mortality routing (0: paper, 1: to P4)
 *   prm[14] transformation algorithm (0: Algorithm 1, 1: Algorithm 2)
 *
 * Gradient vector g[12 + R]
 *   g[0..4] dL/dD_s, g[5] v_DOM, g[6] K_DOM, g[7] rho, g[8] mu, g[9] beta,
 *   g[10] v_SOM, g[11] v_FOM, g[12 + r] dL/dc_r (region conductance factors)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NPOOL 5
#define NPARAM_BASE 12

enum { P_D = 0, P_H = 5, P_VDOM = 6, P_KDOM = 7, P_RHO = 8, P_MU = 9, P_BETA = 10,
       P_VSOM = 11, P_VFOM = 12, P_ROUTE = 13, P_ALG = 14 };

/* ------------------------------------------------------------------------ */
/* Graph (Sec. II.A, Fig. 2; Sec. III): the pore voxels are the nodes, and two
 * nodes are joined when the voxels share a face (6-connectivity).           */
/* ------------------------------------------------------------------------ */

int64_t orc_count(const uint8_t *mask, int64_t nvox)
{
    int64_t n = 0;
    for (int64_t v = 0; v < nvox; v++)
        if (mask[v]) n++;
    return n;
}

/* Enumeration order of the pore voxels.  brick <= 0: raster (x fastest).
 * brick = b > 0: bricks of b^3 voxels in raster order of bricks, voxels in
 * raster order inside each brick.  The paper leaves the order open.        */
int orc_build_graph(const uint8_t *mask, int nx, int ny, int nz, int brick,
                    int periodic, int32_t *vox, int32_t *nbr, int64_t n)
{
    int64_t nvox = (int64_t)nx * ny * nz;
    int64_t *map = (int64_t *)malloc(sizeof(int64_t) * (size_t)nvox);
    if (!map) return -1;
    for (int64_t v = 0; v < nvox; v++) map[v] = -1;

    int64_t i = 0;
    if (brick <= 0) {
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    int64_t v = x + (int64_t)nx * (y + (int64_t)ny * z);
                    if (mask[v]) { if (i >= n) { free(map); return -2; }
                                   vox[i] = (int32_t)v; map[v] = i; i++; }
                }
    } else {
        int b = brick;
        for (int bz = 0; bz < nz; bz += b)
            for (int by = 0; by < ny; by += b)
                for (int bx = 0; bx < nx; bx += b)
                    for (int z = bz; z < bz + b && z < nz; z++)
                        for (int y = by; y < by + b && y < ny; y++)
                            for (int x = bx; x < bx + b && x < nx; x++) {
                                int64_t v = x + (int64_t)nx * (y + (int64_t)ny * z);
                                if (mask[v]) { if (i >= n) { free(map); return -2; }
                                               vox[i] = (int32_t)v; map[v] = i; i++; }
                            }
    }
    if (i != n) { free(map); return -2; }

    static const int off[6][3] = { {-1,0,0}, {1,0,0}, {0,-1,0}, {0,1,0}, {0,0,-1}, {0,0,1} };
    int dims[3] = { nx, ny, nz };
    for (int64_t c = 0; c < n; c++) {
        int64_t v = vox[c];
        int p[3] = { (int)(v % nx), (int)((v / nx) % ny), (int)(v / ((int64_t)nx * ny)) };
        for (int k = 0; k < 6; k++) {
            int q[3];
            int inside = 1;
            for (int a = 0; a < 3; a++) {
                q[a] = p[a] + off[k][a];
                if (q[a] < 0 || q[a] >= dims[a]) {
                    if (periodic & (1 << a)) q[a] = (q[a] + dims[a]) % dims[a];
                    else inside = 0;
                }
            }
            int32_t j = -1;
            if (inside) {
                int64_t u = q[0] + (int64_t)nx * (q[1] + (int64_t)ny * q[2]);
                if (mask[u]) j = (int32_t)map[u];
            }
            nbr[(int64_t)k * n + c] = j;
        }
    }
    free(map);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Transformation (Sec. II.C eq. (3); Appendix A, Algorithm 1): all fluxes of
 * a voxel are computed from its pre-step masses, clamped so that no pool can
 * give more than it holds, and then applied.  Alg. 1 names mortality to DOM
 * and SOM "mortaDOM"/"mortaSOM" and later "morDOM"/"morSOM"; they are the
 * same quantities.                                                          */
/* ------------------------------------------------------------------------ */

static void transform_one(const double *prm, double dt, double *x1, double *x2,
                          double *x3, double *x4, double *x5)
{
    double v_dom = prm[P_VDOM], k_dom = prm[P_KDOM], rho = prm[P_RHO], mu = prm[P_MU];
    double beta = prm[P_BETA], v_som = prm[P_VSOM], v_fom = prm[P_VFOM];
    double m1 = *x1, m2 = *x2, m3 = *x3, m4 = *x4, m5 = *x5;

    double uptake = v_dom * m2 / (k_dom + m2) * m1 * dt;   /* Monod uptake */
    if (uptake > m2) uptake = m2;
    double resp = rho * m1 * dt;                           /* respiration */
    double morta = mu * m1 * dt;                           /* mortality */
    if (resp + morta > m1) {
        if (morta > m1) { morta = m1; resp = 0.0; }
        else resp = m1 - morta;
    }
    double morta_dom, morta_som, morta_p4;
    if (prm[P_ROUTE] == 0.0) {            /* paper: beta to DOM, 1-beta to SOM */
        morta_som = (1.0 - beta) * morta;
        morta_dom = beta * morta;
        morta_p4 = 0.0;
    } else {                              /* alternative: all to pool 4 */
        morta_som = 0.0;
        morta_dom = 0.0;
        morta_p4 = morta;
    }
    double turn_fom = v_fom * m4 * dt;
    if (turn_fom > m4) turn_fom = m4;
    double turn_som = v_som * m3 * dt;
    if (turn_som > m3) turn_som = m3;

    *x1 = m1 + (uptake - morta - resp);
    *x2 = m2 + (morta_dom - uptake + turn_fom + turn_som);
    *x3 = m3 + (morta_som - turn_som);
    if (prm[P_ROUTE] == 0.0) *x4 = m4 - turn_fom;
    else *x4 = m4 + (morta_p4 - turn_fom);
    *x5 = m5 + resp;
}

/* Transformation, Appendix A Algorithm 2: the processes of a voxel update
 * its masses one after the other, each from the masses the previous one
 * left: uptake (MB grows on DOM), mortality (dead MB to DOM and SOM, or to
 * pool 4), respiration (MB to CO2), then SOM and FOM turnover to DOM.  A
 * process that would take more than its source pool holds takes all of it.
 * As printed the algorithm tests "resp" instead of each turnover against its
 * own pool, zeroes SOM / FOM before adding them to DOM (losing that mass)
 * and leaves MB in place when all of it dies; those three slips are read as
 * corrected here: each turnover is compared with its own pool, the pool is
 * moved to DOM before it is zeroed, and MB is zeroed when it all dies.      */
static void transform_seq_one(const double *prm, double dt, double *x1, double *x2,
                              double *x3, double *x4, double *x5)
{
    double v_dom = prm[P_VDOM], k_dom = prm[P_KDOM], rho = prm[P_RHO], mu = prm[P_MU];
    double beta = prm[P_BETA], v_som = prm[P_VSOM], v_fom = prm[P_VFOM];
    int paper_route = prm[P_ROUTE] == 0.0;
    double m1 = *x1, m2 = *x2, m3 = *x3, m4 = *x4, m5 = *x5;

    if (m1 > 0.0) {
        if (m2 > 0.0) {
            double uptake = v_dom * m2 / (k_dom + m2) * m1 * dt;
            if (uptake < m2) { m1 = m1 + uptake; m2 = m2 - uptake; }
            else { m1 = m1 + m2; m2 = 0.0; }
        }
        double morta = mu * m1 * dt;
        if (morta < m1) {
            m1 = m1 - morta;
            if (paper_route) { m2 = m2 + beta * morta; m3 = m3 + (1.0 - beta) * morta; }
            else m4 = m4 + morta;
        } else {
            if (paper_route) { m2 = m2 + beta * m1; m3 = m3 + (1.0 - beta) * m1; }
            else m4 = m4 + m1;
            m1 = 0.0;
        }
        double resp = rho * m1 * dt;
        if (resp < m1) { m1 = m1 - resp; m5 = m5 + resp; }
        else { m5 = m5 + m1; m1 = 0.0; }
    }
    if (m3 > 0.0) {
        double turn_som = v_som * m3 * dt;
        if (turn_som < m3) { m3 = m3 - turn_som; m2 = m2 + turn_som; }
        else { m2 = m2 + m3; m3 = 0.0; }
    }
    if (m4 > 0.0) {
        double turn_fom = v_fom * m4 * dt;
        if (turn_fom < m4) { m4 = m4 - turn_fom; m2 = m2 + turn_fom; }
        else { m2 = m2 + m4; m4 = 0.0; }
    }
    *x1 = m1; *x2 = m2; *x3 = m3; *x4 = m4; *x5 = m5;
}

void orc_transform(const double *prm, double dt, int64_t n, double *x)
{
    int seq = prm[P_ALG] != 0.0;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (seq) transform_seq_one(prm, dt, &x[i], &x[n + i], &x[2 * n + i], &x[3 * n + i], &x[4 * n + i]);
        else transform_one(prm, dt, &x[i], &x[n + i], &x[2 * n + i], &x[3 * n + i], &x[4 * n + i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Diffusion, explicit (Sec. II.B.3a, Scheme 1): m_i <- m_i + a * sum_j
 * w_ij (m_j - m_i) with a = D dt / h^2 (voxel units make S_ij = d_ij = 1,
 * Sec. II.B.2; w_ij generalises that unit conductance).  The six slot terms
 * are added in the fixed order ((d0+d1)+(d2+d3))+(d4+d5).                  */
/* ------------------------------------------------------------------------ */

static double slot_term(const int32_t *nbr, const double *w, const double *m,
                        int64_t n, int64_t i, int k)
{
    int32_t j = nbr[(int64_t)k * n + i];
    if (j < 0) return 0.0;
    double diff = m[j] - m[i];
    return w ? w[(int64_t)k * n + i] * diff : diff;
}

static void diffuse_pool(double a, int64_t n, const int32_t *nbr, const double *w,
                         const double *m, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double d0 = slot_term(nbr, w, m, n, i, 0), d1 = slot_term(nbr, w, m, n, i, 1);
        double d2 = slot_term(nbr, w, m, n, i, 2), d3 = slot_term(nbr, w, m, n, i, 3);
        double d4 = slot_term(nbr, w, m, n, i, 4), d5 = slot_term(nbr, w, m, n, i, 5);
        double s = ((d0 + d1) + (d2 + d3)) + (d4 + d5);
        out[i] = m[i] + a * s;
    }
}

static double coef_a(const double *prm, int s, double dt)
{
    return prm[P_D + s] * dt / (prm[P_H] * prm[P_H]);
}

void orc_diffuse(const double *prm, double dt, int64_t n, const int32_t *nbr,
                 const double *w, double *x, double *tmp)
{
    for (int s = 0; s < NPOOL; s++) {
        if (prm[P_D + s] == 0.0) continue;
        double a = coef_a(prm, s, dt);
        diffuse_pool(a, n, nbr, w, &x[(int64_t)s * n], tmp);
        memcpy(&x[(int64_t)s * n], tmp, sizeof(double) * (size_t)n);
    }
}

/* Graph Laplacian (Sec. II.B.2): (L_w m)_i = sum_j w_ij (m_i - m_j).     */
void orc_laplacian(int64_t n, const int32_t *nbr, const double *w, const double *m, double *out)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int k = 0; k < 6; k++) {
            int32_t j = nbr[(int64_t)k * n + i];
            if (j < 0) continue;
            double wk = w ? w[(int64_t)k * n + i] : 1.0;
            s += wk * (m[i] - m[j]);
        }
        out[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Mass totals: Neumaier-compensated FP64 sums per segment and pool, plus the
 * total carbon of the segment in slot 5.  out[nseg][6].                    */
/* ------------------------------------------------------------------------ */

static void neumaier_add(double *sum, double *comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v)) *comp += (*sum - t) + v;
    else *comp += (v - t) + *sum;
    *sum = t;
}

void orc_totals(int64_t n, const double *x, int nseg, const int64_t *seg_off, double *out)
{
    for (int g = 0; g < nseg; g++) {
        int64_t lo = seg_off ? seg_off[g] : 0, hi = seg_off ? seg_off[g + 1] : n;
        double all = 0.0, allc = 0.0;
        for (int s = 0; s < NPOOL; s++) {
            double sum = 0.0, comp = 0.0;
            for (int64_t i = lo; i < hi; i++) neumaier_add(&sum, &comp, x[(int64_t)s * n + i]);
            out[g * 6 + s] = sum + comp;
            neumaier_add(&all, &allc, sum + comp);
        }
        out[g * 6 + 5] = all + allc;
    }
}

/* ------------------------------------------------------------------------ */
/* Time loop (Sec. II.A; Sec. III): each step transforms every voxel, then
 * diffuses.  order = 0 is that paper order, order = 1 diffuses first.
 * totals (optional) receives [nsteps+1][nseg][6]: the state before the first
 * step and after every step.                                               */
/* ------------------------------------------------------------------------ */

int orc_run(const double *prm, double dt, int order, int64_t n, const int32_t *nbr,
            const double *w, double *x, int64_t nsteps, int nseg, const int64_t *seg_off,
            double *totals)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!tmp) return -1;
    if (totals) orc_totals(n, x, nseg, seg_off, totals);
    for (int64_t t = 0; t < nsteps; t++) {
        if (order == 0) {
            orc_transform(prm, dt, n, x);
            orc_diffuse(prm, dt, n, nbr, w, x, tmp);
        } else {
            orc_diffuse(prm, dt, n, nbr, w, x, tmp);
            orc_transform(prm, dt, n, x);
        }
        if (totals) orc_totals(n, x, nseg, seg_off, totals + (t + 1) * nseg * 6);
    }
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Unequal time steps (Sec. III: the process with the smaller step is
 * repeated).  Over [0, t_end], t_end = nt * dt_t, transformation steps of
 * dt_t start at k dt_t (k < nt) and diffusion steps of dt_d start at k dt_d
 * while k dt_d < t_end, the last one shortened to end at t_end.  Every step
 * is explicit and uses the state at its start, so the steps are applied in
 * the order of their start times, a transformation first when both start
 * together (with dt_t = dt_d this is the paper's T-then-D step).            */
/* ------------------------------------------------------------------------ */

int orc_run_subcycled(const double *prm, double dt_t, double dt_d, int64_t nt, int64_t n,
                      const int32_t *nbr, const double *w, double *x)
{
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!tmp) return -1;
    double t_end = (double)nt * dt_t;
    int64_t kt = 0, kd = 0;
    for (;;) {
        double st = (double)kt * dt_t;       /* start of the next transformation step */
        double sd = (double)kd * dt_d;       /* start of the next diffusion step */
        int more_t = kt < nt, more_d = sd < t_end;
        if (!more_t && !more_d) break;
        if (more_t && (!more_d || st <= sd)) {
            orc_transform(prm, dt_t, n, x);
            kt++;
        } else {
            double len = (double)(kd + 1) * dt_d <= t_end ? dt_d : t_end - sd;
            orc_diffuse(prm, len, n, nbr, w, x, tmp);
            kd++;
        }
    }
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diffusion, implicit (Sec. II.B.3b, Scheme 2): solve (I + a L_w) y = m with
 * the conjugate gradient method preconditioned by the inverse diagonal of the
 * system matrix (Sec. III).  Starts from y = m; stops when
 * ||m - B y||_2 <= rtol ||m||_2.                                            */
/* ------------------------------------------------------------------------ */

void orc_apply_B(double a, int64_t n, const int32_t *nbr, const double *w, const double *p, double *q)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int k = 0; k < 6; k++) {
            int32_t j = nbr[(int64_t)k * n + i];
            if (j < 0) continue;
            double wk = w ? w[(int64_t)k * n + i] : 1.0;
            s += wk * (p[i] - p[j]);
        }
        q[i] = p[i] + a * s;
    }
}

static double dot(int64_t n, const double *u, const double *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += u[i] * v[i];
    return s;
}

int orc_pcg(double a, int64_t n, const int32_t *nbr, const double *w, const double *b,
            double *y, double rtol, int max_iter, int *iters, double *relres)
{
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    double *tinv = malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q || !tinv) { free(r); free(z); free(p); free(q); free(tinv); return -1; }

    for (int64_t i = 0; i < n; i++) {               /* T = diag(B)^-1 */
        double deg = 0.0;
        for (int k = 0; k < 6; k++)
            if (nbr[(int64_t)k * n + i] >= 0) deg += w ? w[(int64_t)k * n + i] : 1.0;
        tinv[i] = 1.0 / (1.0 + a * deg);
    }
    memcpy(y, b, sizeof(double) * (size_t)n);
    orc_apply_B(a, n, nbr, w, y, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    for (int64_t i = 0; i < n; i++) z[i] = tinv[i] * r[i];
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rz = dot(n, r, z);
    double bnorm = sqrt(dot(n, b, b));
    double rnorm = sqrt(dot(n, r, r));
    int it = 0;
    while (!(rnorm <= rtol * bnorm) && it < max_iter) {
        orc_apply_B(a, n, nbr, w, p, q);
        double alpha = rz / dot(n, p, q);
        for (int64_t i = 0; i < n; i++) y[i] += alpha * p[i];
        for (int64_t i = 0; i < n; i++) r[i] -= alpha * q[i];
        for (int64_t i = 0; i < n; i++) z[i] = tinv[i] * r[i];
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        rnorm = sqrt(dot(n, r, r));
        it++;
    }
    if (iters) *iters = it;
    if (relres) *relres = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    free(r); free(z); free(p); free(q); free(tinv);
    return (rnorm <= rtol * bnorm) ? 0 : 1;
}

/* One implicit step: transformation, then Scheme 2 for every pool with
 * D_s > 0.  iters/relres receive one entry per pool (0 for immobile ones). */
int orc_implicit_step(const double *prm, double dt, int64_t n, const int32_t *nbr,
                      const double *w, double *x, double rtol, int max_iter,
                      int *iters, double *relres)
{
    double *y = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!y) return -1;
    int status = 0;
    orc_transform(prm, dt, n, x);
    for (int s = 0; s < NPOOL; s++) {
        if (iters) iters[s] = 0;
        if (relres) relres[s] = 0.0;
        if (prm[P_D + s] == 0.0) continue;
        int rc = orc_pcg(coef_a(prm, s, dt), n, nbr, w, &x[(int64_t)s * n], y, rtol, max_iter,
                         iters ? &iters[s] : NULL, relres ? &relres[s] : NULL);
        if (rc < 0) { free(y); return rc; }
        if (rc > 0) status = 1;
        memcpy(&x[(int64_t)s * n], y, sizeof(double) * (size_t)n);
    }
    free(y);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Discrete adjoint of the explicit time loop.  The loss L is any function
 * of the per-segment pool totals after every step; seeds[t][g][s] =
 * dL/dTotal_{g,s}(t) for t = 0..nsteps.  states holds x^0..x^nsteps as
 * [nsteps+1][5][n].  lam_final (optional, [5][n]) is an extra adjoint
 * seeded on the last state.  Output: lam0 = dL/dx^0 ([5][n]) and grad
 * (layout in the header).  Written as plain reverse-mode differentiation of
 * transform_one and diffuse_pool above; every scatter is serial.  dL/dD_s
 * is computed for every pool, including those with D_s = 0.              */
/* ------------------------------------------------------------------------ */

/* reverse of transform_one: x = pre-step masses, ybar = adjoint of the
 * outputs (in place: becomes the adjoint of the inputs), gk += dL/d(rates) */
static void transform_one_adj(const double *prm, double dt, const double *xin,
                              double *bar, double *gk)
{
    double v_dom = prm[P_VDOM], k_dom = prm[P_KDOM], rho = prm[P_RHO], mu = prm[P_MU];
    double beta = prm[P_BETA], v_som = prm[P_VSOM], v_fom = prm[P_VFOM];
    double m1 = xin[0], m2 = xin[1], m3 = xin[2], m4 = xin[3];
    int paper_route = prm[P_ROUTE] == 0.0;

    /* forward again, keeping the branch taken */
    double uptake_raw = v_dom * m2 / (k_dom + m2) * m1 * dt;
    int up_clamped = uptake_raw > m2;
    double resp0 = rho * m1 * dt, morta0 = mu * m1 * dt;
    int case_rm = 0;                    /* 0: free, 1: all dies, 2: resp gets the rest */
    double morta = morta0;
    if (resp0 + morta0 > m1) {
        if (morta0 > m1) { case_rm = 1; morta = m1; }
        else case_rm = 2;
    }
    double tf_raw = v_fom * m4 * dt, ts_raw = v_som * m3 * dt;
    int tf_clamped = tf_raw > m4, ts_clamped = ts_raw > m3;

    double y1 = bar[0], y2 = bar[1], y3 = bar[2], y4 = bar[3], y5 = bar[4];
    double x1b = y1, x2b = y2, x3b = y3, x4b = y4, x5b = y5;

    double upb = y1 - y2;
    double mortb, betab;
    if (paper_route) { mortb = -y1 + beta * y2 + (1.0 - beta) * y3; betab = morta * (y2 - y3); }
    else { mortb = -y1 + y4; betab = 0.0; }
    double respb = -y1 + y5;
    double tfb = y2 - y4;
    double tsb = y2 - y3;

    if (up_clamped) {
        x2b += upb;
    } else {
        double den = k_dom + m2;
        double g = m2 / den;
        x1b += upb * v_dom * g * dt;
        x2b += upb * v_dom * m1 * dt * k_dom / (den * den);
        gk[0] += upb * g * m1 * dt;                              /* v_DOM */
        gk[1] += -upb * v_dom * m1 * dt * m2 / (den * den);      /* K_DOM */
    }
    if (case_rm == 0) {
        x1b += respb * rho * dt + mortb * mu * dt;
        gk[2] += respb * m1 * dt;                                /* rho */
        gk[3] += mortb * m1 * dt;                                /* mu */
    } else if (case_rm == 1) {
        x1b += mortb;
    } else {
        double mt = mortb - respb;
        x1b += respb + mt * mu * dt;
        gk[3] += mt * m1 * dt;
    }
    gk[4] += betab;                                              /* beta */
    if (ts_clamped) x3b += tsb;
    else { x3b += tsb * v_som * dt; gk[5] += tsb * m3 * dt; }    /* v_SOM */
    if (tf_clamped) x4b += tfb;
    else { x4b += tfb * v_fom * dt; gk[6] += tfb * m4 * dt; }    /* v_FOM */

    bar[0] = x1b; bar[1] = x2b; bar[2] = x3b; bar[3] = x4b; bar[4] = x5b;
}

/* reverse of diffuse_pool for one pool: u = input, lam = adjoint of the
 * output (overwritten by the adjoint of the input).  ga += dL/da,
 * gw[6][n] += dL/dw (if gw != NULL).                                      */
static void diffuse_pool_adj(double a, int64_t n, const int32_t *nbr, const double *w,
                             const double *u, double *lam, double *tmp, double *ga, double *gw)
{
    for (int64_t i = 0; i < n; i++) tmp[i] = lam[i];        /* identity term */
    for (int64_t i = 0; i < n; i++) {
        double sbar = a * lam[i];
        double d[6];
        for (int k = 0; k < 6; k++) {
            int32_t j = nbr[(int64_t)k * n + i];
            d[k] = 0.0;
            if (j < 0) continue;
            double wk = w ? w[(int64_t)k * n + i] : 1.0;
            double diff = u[j] - u[i];
            d[k] = wk * diff;
            tmp[j] += wk * sbar;
            tmp[i] -= wk * sbar;
            if (gw) gw[(int64_t)k * n + i] += sbar * diff;
        }
        double s = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + d[5]);
        *ga += lam[i] * s;
    }
    memcpy(lam, tmp, sizeof(double) * (size_t)n);
}

static void add_seeds(int64_t n, double *lam, int nseg, const int64_t *seg_off, const double *seed_t)
{
    for (int g = 0; g < nseg; g++) {
        int64_t lo = seg_off ? seg_off[g] : 0, hi = seg_off ? seg_off[g + 1] : n;
        for (int s = 0; s < NPOOL; s++) {
            double v = seed_t[g * NPOOL + s];
            if (v == 0.0) continue;
            for (int64_t i = lo; i < hi; i++) lam[(int64_t)s * n + i] += v;
        }
    }
}

int orc_adjoint(const double *prm, double dt, int order, int64_t n, const int32_t *nbr,
                const double *w, const int32_t *region, int nreg, int64_t nsteps,
                const double *states, int nseg, const int64_t *seg_off, const double *seeds,
                const double *lam_final, double *lam0, double *grad)
{
    if (prm[P_ALG] != 0.0) return -2;     /* the adjoint follows Algorithm 1 only */
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *lam = lam0;
    double *u = malloc(sizeof(double) * NPOOL * nn);
    double *tmp = malloc(sizeof(double) * nn);
    double *gw = (region && nreg > 0) ? calloc(6 * nn, sizeof(double)) : NULL;
    if (!u || !tmp || (region && nreg > 0 && !gw)) { free(u); free(tmp); free(gw); return -1; }
    for (int q = 0; q < NPARAM_BASE + nreg; q++) grad[q] = 0.0;
    if (lam_final) memcpy(lam, lam_final, sizeof(double) * NPOOL * (size_t)n);
    else memset(lam, 0, sizeof(double) * NPOOL * nn);
    add_seeds(n, lam, nseg, seg_off, seeds + nsteps * nseg * NPOOL);

    double hh = prm[P_H] * prm[P_H];
    for (int64_t t = nsteps - 1; t >= 0; t--) {
        const double *xk = states + t * NPOOL * (int64_t)n;
        double ga[NPOOL] = {0, 0, 0, 0, 0};
        if (order == 0) {
            /* forward: u = T(x^t); x^{t+1} = D(u) */
            memcpy(u, xk, sizeof(double) * NPOOL * (size_t)n);
            for (int64_t i = 0; i < n; i++)
                transform_one(prm, dt, &u[i], &u[n + i], &u[2 * n + i], &u[3 * n + i], &u[4 * n + i]);
            for (int s = 0; s < NPOOL; s++) {
                diffuse_pool_adj(coef_a(prm, s, dt), n, nbr, w, &u[(int64_t)s * n],
                                 &lam[(int64_t)s * n], tmp, &ga[s], gw);
            }
            for (int64_t i = 0; i < n; i++) {
                double xin[5], bar[5];
                for (int s = 0; s < NPOOL; s++) { xin[s] = xk[(int64_t)s * n + i]; bar[s] = lam[(int64_t)s * n + i]; }
                transform_one_adj(prm, dt, xin, bar, &grad[5]);
                for (int s = 0; s < NPOOL; s++) lam[(int64_t)s * n + i] = bar[s];
            }
        } else {
            /* forward: u = D(x^t); x^{t+1} = T(u) */
            memcpy(u, xk, sizeof(double) * NPOOL * (size_t)n);
            for (int s = 0; s < NPOOL; s++) {
                if (prm[P_D + s] == 0.0) continue;
                diffuse_pool(coef_a(prm, s, dt), n, nbr, w, &xk[(int64_t)s * n], &u[(int64_t)s * n]);
            }
            for (int64_t i = 0; i < n; i++) {
                double xin[5], bar[5];
                for (int s = 0; s < NPOOL; s++) { xin[s] = u[(int64_t)s * n + i]; bar[s] = lam[(int64_t)s * n + i]; }
                transform_one_adj(prm, dt, xin, bar, &grad[5]);
                for (int s = 0; s < NPOOL; s++) lam[(int64_t)s * n + i] = bar[s];
            }
            for (int s = 0; s < NPOOL; s++) {
                diffuse_pool_adj(coef_a(prm, s, dt), n, nbr, w, &xk[(int64_t)s * n],
                                 &lam[(int64_t)s * n], tmp, &ga[s], gw);
            }
        }
        for (int s = 0; s < NPOOL; s++) grad[s] += ga[s] * dt / hh;   /* a_s = D_s dt / h^2 */
        add_seeds(n, lam, nseg, seg_off, seeds + t * nseg * NPOOL);
    }

    /* w_ij = (c_{r(i)} + c_{r(j)}) / 2, so dw_ij/dc_r = ([r(i)=r] + [r(j)=r]) / 2 */
    if (gw) {
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < 6; k++) {
                int32_t j = nbr[(int64_t)k * n + i];
                if (j < 0) continue;
                double g = gw[(int64_t)k * n + i];
                grad[NPARAM_BASE + region[i]] += 0.5 * g;
                grad[NPARAM_BASE + region[j]] += 0.5 * g;
            }
    }
    free(u); free(tmp); free(gw);
    return 0;
}
