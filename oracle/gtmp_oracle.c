/*
 * gtmp_oracle.c -- plain, slow FP64 reference of the layered-graph planner
 * (Global Tensor Motion Planning with a straight-line local planner).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The HIP product path
 * never links, calls or includes anything from here, and this file includes
 * nothing from the product path: the two implementations share no code.
 *
 * Every routine follows the definition it cites, written out with plain loops
 * in double precision.  Inputs (scenes, robot models, samples) are float32
 * arrays, the precision the planner stores; they are promoted exactly to
 * double on entry.
 *
 * Paper: "Anytime Global Tensor Motion Planning" (Coumar, Le, Kingston).
 *   Sec. III        configuration space, open free space (boundary = collision)
 *   Sec. III-A      layered sampling model, vertex sets V_0 = {q0}, V_m, goals
 *   Sec. III-B      local planner LP, edge present iff LP succeeds
 *   Alg. 1 (gtmp)   cost matrices C_s, C_h, C_l; value tensor; argmin
 *                   extraction
 *   Sec. IV-B       Bellman recursion on the layered DAG, absent edge = +inf
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads the OpenMP loops of this file use. */
int or_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11).  Ten rounds of the */
/* 4x32 S-box: two 32x32->64 multiplications, xor with the other two counter */
/* words and the key, followed by a Weyl increment of the key.               */
/* ------------------------------------------------------------------------ */
#define OR_PHILOX_MULT_A 0xD2511F53u
#define OR_PHILOX_MULT_B 0xCD9E8D57u
#define OR_PHILOX_WEYL_A 0x9E3779B9u
#define OR_PHILOX_WEYL_B 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_WEYL_A;
            k1 += OR_PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)OR_PHILOX_MULT_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)OR_PHILOX_MULT_B * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* a1: uniform layer samples (Alg. 1: "uniformly sample Q in R^{MxNxd}";     */
/* Sec. III-A: N independent samples per intermediate layer).               */
/*                                                                          */
/* Random word for (layer m, sample n, coordinate j) at stage `stage`:      */
/*   key     = (seed mod 2^32, seed div 2^32)                               */
/*   counter = (n, m, stage mod 2^32, stream * 2^16 + j div 4)              */
/*   word    = Philox4x32-10(counter, key)[j mod 4]                         */
/* u = (word >> 8) * 2^-24 in [0,1); the stored sample is the float32       */
/* rounding of lo_j + u * w_j with w_j the float32 difference hi_j - lo_j.  */
/* ------------------------------------------------------------------------ */
double or_unit_from_word(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

void or_words(uint64_t seed, uint64_t stage, uint32_t stream, uint32_t n, uint32_t m, uint32_t blk,
              uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {n, m, (uint32_t)(stage & 0xffffffffu), (stream << 16) | blk};
    or_philox4x32_10(ctr, key, out);
}

void or_sample_layers(int M, int N, int d, const float *lo, const float *hi, uint64_t seed,
                      uint64_t stage, float *Q /* [M][N][d] */)
{
    for (int m = 0; m < M; ++m)
        for (int n = 0; n < N; ++n)
            for (int j = 0; j < d; ++j) {
                uint32_t w[4];
                or_words(seed, stage, 0u, (uint32_t)n, (uint32_t)m, (uint32_t)(j / 4), w);
                double u = or_unit_from_word(w[j % 4]);
                double width = (double)(float)((double)hi[j] - (double)lo[j]);
                Q[((size_t)m * N + n) * d + j] = (float)((double)lo[j] + u * width);
            }
}

/* ------------------------------------------------------------------------ */
/* Collision model (Sec. III: C_free is open, so a configuration whose       */
/* signed distance to the obstacles is <= 0 is in collision).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind;            /* 0: point robot, configuration = workspace point; 1: serial arm */
    int d;               /* configuration dimension */
    int wdim;            /* workspace dimension of the obstacles (2 or 3) */
    int n_joints;        /* arm: number of revolute joints (== d) */
    const float *dh;     /* arm: [n_joints][4] = (a, alpha, d, theta_offset), standard DH */
    int n_rsph;          /* arm: collision spheres */
    const int *rsph_link;  /* [n_rsph] link index 1..n_joints */
    const float *rsph_t;   /* [n_rsph] fraction along the link o_{i-1} -> o_i */
    const float *rsph_r;   /* [n_rsph] radius */
    int n_osph;          /* sphere / circle obstacles */
    const float *osph;   /* [n_osph][wdim + 1] = (centre, radius) */
    int n_obox;          /* axis-aligned box obstacles */
    const float *obox;   /* [n_obox][2 * wdim] = (centre, half extents) */
} or_model;

/* Euclidean distance from p to the sphere surface: |p - c| - r. */
static double or_sd_sphere(int wdim, const double *p, const float *s)
{
    double acc = 0.0;
    for (int i = 0; i < wdim; ++i) {
        double t = p[i] - (double)s[i];
        acc += t * t;
    }
    return sqrt(acc) - (double)s[wdim];
}

/* Exact signed distance to an axis-aligned box with centre c, half extents h:
 * q = |p - c| - h;  sd = |max(q, 0)| + min(max_i q_i, 0). */
static double or_sd_box(int wdim, const double *p, const float *b)
{
    double outside = 0.0, inside = -INFINITY;
    for (int i = 0; i < wdim; ++i) {
        double q = fabs(p[i] - (double)b[i]) - (double)b[wdim + i];
        double qp = q > 0.0 ? q : 0.0;
        outside += qp * qp;
        if (q > inside) inside = q;
    }
    return sqrt(outside) + (inside < 0.0 ? inside : 0.0);
}

double or_sd_point(const or_model *mdl, const double *p)
{
    double best = INFINITY;
    for (int o = 0; o < mdl->n_osph; ++o) {
        double v = or_sd_sphere(mdl->wdim, p, mdl->osph + (size_t)o * (mdl->wdim + 1));
        if (v < best) best = v;
    }
    for (int o = 0; o < mdl->n_obox; ++o) {
        double v = or_sd_box(mdl->wdim, p, mdl->obox + (size_t)o * 2 * mdl->wdim);
        if (v < best) best = v;
    }
    return best;
}

/* Standard Denavit-Hartenberg forward kinematics.  Link transform
 *   A_i = Rz(theta_i) Tz(d_i) Tx(a_i) Rx(alpha_i),  theta_i = q_i + offset_i,
 * chained from the base frame (identity at the origin): T_i = T_{i-1} A_i.
 * Writes the frame origins o_0 (= base origin) .. o_J, [J + 1][3]. */
void or_fk_origins(int J, const float *dh, const double *q, double *o)
{
    double T[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    o[0] = o[1] = o[2] = 0.0;
    for (int i = 0; i < J; ++i) {
        double a = dh[4 * i + 0], alpha = dh[4 * i + 1], dz = dh[4 * i + 2], off = dh[4 * i + 3];
        double th = q[i] + off;
        double ct = cos(th), st = sin(th), ca = cos(alpha), sa = sin(alpha);
        double A[4][4] = {{ct, -st * ca, st * sa, a * ct},
                          {st, ct * ca, -ct * sa, a * st},
                          {0.0, sa, ca, dz},
                          {0.0, 0.0, 0.0, 1.0}};
        double R[4][4];
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += T[r][k] * A[k][c];
                R[r][c] = acc;
            }
        memcpy(T, R, sizeof(T));
        o[3 * (i + 1) + 0] = T[0][3];
        o[3 * (i + 1) + 1] = T[1][3];
        o[3 * (i + 1) + 2] = T[2][3];
    }
}

/* Centres of the arm's collision spheres: c_k = o_{L-1} + t_k (o_L - o_{L-1}). */
void or_arm_spheres(const or_model *mdl, const double *q, double *centres /* [n_rsph][3] */)
{
    double o[3 * 33];
    or_fk_origins(mdl->n_joints, mdl->dh, q, o);
    for (int k = 0; k < mdl->n_rsph; ++k) {
        int L = mdl->rsph_link[k];
        double t = mdl->rsph_t[k];
        for (int i = 0; i < 3; ++i)
            centres[3 * k + i] = o[3 * (L - 1) + i] + t * (o[3 * L + i] - o[3 * (L - 1) + i]);
    }
}

/* Signed distance of a configuration to the obstacle set. */
double or_state_sd(const or_model *mdl, const double *q)
{
    if (mdl->kind == 0) return or_sd_point(mdl, q);
    double c[3 * 256];
    or_arm_spheres(mdl, q, c);
    double best = INFINITY;
    for (int k = 0; k < mdl->n_rsph; ++k) {
        double v = or_sd_point(mdl, c + 3 * k) - (double)mdl->rsph_r[k];
        if (v < best) best = v;
    }
    return best;
}

void or_state_sd_batch(const or_model *mdl, long n, const float *X /* [n][d] */, double *sd)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; ++i) {
        double q[64];
        for (int j = 0; j < mdl->d; ++j) q[j] = X[(size_t)i * mdl->d + j];
        sd[i] = or_state_sd(mdl, q);
    }
}

/* ------------------------------------------------------------------------ */
/* a2-a4: straight-line local planner on one edge (Sec. III-B; SEV in       */
/* Sec. V).  The edge is realised by the H states x_h = u + (h/(H-1))(v-u), */
/* h = 0..H-1 (both endpoints included).  The LP fails (edge absent) iff a  */
/* state is in collision or |v - u| exceeds the length limit.  An edge that */
/* succeeds costs its length; a failed edge costs length + penalty, and     */
/* +inf when the penalty is +inf (absent edge, Sec. IV-B).                  */
/* ------------------------------------------------------------------------ */
void or_edge(const or_model *mdl, int H, double penalty, double max_len, const float *u,
             const float *v, double *cost, double *minsd, int *flag)
{
    int d = mdl->d;
    double du[64], dv[64], x[64];
    double len2 = 0.0;
    for (int j = 0; j < d; ++j) {
        du[j] = u[j];
        dv[j] = v[j];
        len2 += (dv[j] - du[j]) * (dv[j] - du[j]);
    }
    double len = sqrt(len2);
    double best = INFINITY;
    for (int h = 0; h < H; ++h) {
        double t = (double)h / (double)(H - 1);
        for (int j = 0; j < d; ++j) x[j] = du[j] + t * (dv[j] - du[j]);
        double sd = or_state_sd(mdl, x);
        if (sd < best) best = sd;
    }
    int f = (best <= 0.0) || (len > max_len);
    *flag = f;
    *minsd = best;
    *cost = f ? len + penalty : len;
}

/* Flattened edge numbering used by the subset routine:
 *   [0, N)                         start -> layer 0 vertex u
 *   [N, N + (M-1) N^2)             layer m vertex u -> layer m+1 vertex v, (m, u, v) row-major
 *   [N + (M-1) N^2, ... + N G)     layer M-1 vertex u -> goal g, (u, g) row-major       */
static void or_edge_endpoints(int M, int N, int G, int d, const float *q0, const float *goals,
                              const float *Q, long e, const float **pu, const float **pv)
{
    long nin = (long)(M - 1) * N * N;
    if (e < N) {
        *pu = q0;
        *pv = Q + (size_t)e * d; /* layer 0 */
    } else if (e < N + nin) {
        long r = e - N;
        long m = r / ((long)N * N), uv = r % ((long)N * N);
        *pu = Q + ((size_t)m * N + uv / N) * d;
        *pv = Q + ((size_t)(m + 1) * N + uv % N) * d;
    } else {
        long r = e - N - nin;
        *pu = Q + ((size_t)(M - 1) * N + r / G) * d;
        *pv = goals + (size_t)(r % G) * d;
    }
}

void or_edge_subset(const or_model *mdl, int M, int N, int G, int H, double penalty, double max_len,
                    const float *q0, const float *goals, const float *Q, long n_sel,
                    const long *edge_ids, double *cost, double *minsd, int *flag)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < n_sel; ++i) {
        const float *pu, *pv;
        or_edge_endpoints(M, N, G, mdl->d, q0, goals, Q, edge_ids[i], &pu, &pv);
        or_edge(mdl, H, penalty, max_len, pu, pv, &cost[i], &minsd[i], &flag[i]);
    }
}

/* All edges: C_s[N], C_h[M-1][N][N] (row = source in layer m, column =
 * destination in layer m+1), C_l[N][G]; the same shape for minsd and flags. */
void or_edge_costs(const or_model *mdl, int M, int N, int G, int H, double penalty, double max_len,
                   const float *q0, const float *goals, const float *Q, double *cost /* [E] */,
                   double *minsd /* [E] */, int *flag /* [E] */)
{
    long E = (long)N + (long)(M - 1) * N * N + (long)N * G;
#pragma omp parallel for schedule(dynamic, 64)
    for (long e = 0; e < E; ++e) {
        const float *pu, *pv;
        or_edge_endpoints(M, N, G, mdl->d, q0, goals, Q, e, &pu, &pv);
        or_edge(mdl, H, penalty, max_len, pu, pv, &cost[e], &minsd[e], &flag[e]);
    }
}

/* ------------------------------------------------------------------------ */
/* a5: backward value iteration on the layered DAG (Sec. IV-B):             */
/*   J at the goals = V_g (0 unless given);                                  */
/*   V[M-1][u] = min_g C_l[u][g] + V_g[g];                                   */
/*   V[m][u]   = min_v C_h[m][u][v] + V[m+1][v],   m = M-2 .. 0;             */
/*   V_s       = min_u C_s[u] + V[0][u].                                     */
/* A holds a minimiser (the lowest index among equal values); a row whose    */
/* minimum is +inf has no minimiser and stores -1.                           */
/* ------------------------------------------------------------------------ */
static void or_row_min(int n, const double *c, const double *next, double *val, int *arg)
{
    double best = INFINITY;
    int who = -1;
    for (int v = 0; v < n; ++v) {
        double s = c[v] + next[v];
        if (s < best) {
            best = s;
            who = v;
        }
    }
    *val = best;
    *arg = who;
}

void or_minplus(int M, int N, int G, const double *Cs, const double *Ch, const double *Cl,
                const double *Vg, double *V /* [M][N] */, int *A /* [M][N] */, double *Vs, int *as)
{
    double *vg = (double *)malloc(sizeof(double) * (size_t)G);
    for (int g = 0; g < G; ++g) vg[g] = Vg ? Vg[g] : 0.0;
    for (int u = 0; u < N; ++u)
        or_row_min(G, Cl + (size_t)u * G, vg, &V[(size_t)(M - 1) * N + u], &A[(size_t)(M - 1) * N + u]);
    for (int m = M - 2; m >= 0; --m)
        for (int u = 0; u < N; ++u)
            or_row_min(N, Ch + ((size_t)m * N + u) * N, V + (size_t)(m + 1) * N, &V[(size_t)m * N + u],
                       &A[(size_t)m * N + u]);
    or_row_min(N, Cs, V, Vs, as);
    free(vg);
}

/* ------------------------------------------------------------------------ */
/* a6: follow the minimisers from the start (Alg. 1 extraction; Sec. IV-B   */
/* "applying it repeatedly from q0").  idx[m] = vertex of layer m           */
/* (m = 0..M-1), idx[M] = goal index; waypoints [q0, Q[0][idx0], ...,       */
/* Q[M-1][idx_{M-1}], goals[idx_M]].  Returns 0, or 1 when there is no path */
/* (V_s = +inf), in which case idx is filled with -1.                       */
/* ------------------------------------------------------------------------ */
int or_extract(int M, int N, int G, int d, int as, const int *A, double Vs, const float *Q,
               const float *q0, const float *goals, int *idx /* [M+1] */, double *wp /* [M+2][d] */,
               double *cost)
{
    (void)G;
    *cost = Vs;
    if (as < 0 || isinf(Vs)) {
        for (int m = 0; m <= M; ++m) idx[m] = -1;
        return 1;
    }
    int i = as;
    for (int j = 0; j < d; ++j) wp[j] = q0[j];
    for (int m = 0; m < M; ++m) {
        idx[m] = i;
        for (int j = 0; j < d; ++j) wp[(size_t)(m + 1) * d + j] = Q[((size_t)m * N + i) * d + j];
        i = A[(size_t)m * N + i];
    }
    idx[M] = i;
    for (int j = 0; j < d; ++j) wp[(size_t)(M + 1) * d + j] = goals[(size_t)i * d + j];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* a7: growing-budget sampler (Alg. 1 expand-samples; Sec. IV-E).           */
/*                                                                          */
/* Uniform half: a uniform draw from the informed set                       */
/*   X_f(c) = {x : |x - q0| + |x - q_g| <= c}   (Sec. IV-E)                  */
/* intersected with the sampling box B, by rejection from one of two        */
/* proposal regions that both contain X_f(c) n B:                           */
/*   R: the hyperspheroid's own frame box.  A point y of the cube [-1, 1]^d */
/*      is kept iff |y| < 1 (a uniform point of the unit ball), scaled per  */
/*      axis to the radii (c/2, sqrt(c^2 - c_min^2)/2, ...), rotated so     */
/*      that the first axis points from q0 to q_g and moved to the centre   */
/*      (q0 + q_g)/2 (the direct map of Gammell et al. 2018); the mapped    */
/*      point is kept iff it lies in B.                                     */
/*   C: the axis-aligned bounding box of the hyperspheroid clipped to B.    */
/*      A uniform point of C is kept iff |x - q0| + |x - q_g| <= c.         */
/* Both accept exactly the points of X_f(c) n B, so either gives a uniform  */
/* draw of it; the one with the smaller volume (|R| = prod 2 r_i against    */
/* |C| = prod of C's side lengths) accepts more often and is used.  R wins  */
/* for thin hyperspheroids inside the box, C as soon as the hyperspheroid   */
/* reaches beyond the box, where R alone accepts rarely.                    */
/* Without a bound (c = +inf or c >= the edge penalty) the draw is uniform  */
/* in the box.                                                              */
/*                                                                          */
/* The sample is defined as an FP32 computation with a fixed operation     */
/* order (no fused multiply-add), which this file reproduces with float     */
/* arithmetic (compiled with -ffp-contract=off):                            */
/*   y_i = (w_i >> 8) * 2^-23 - 1                                           */
/*   R: accept iff sum_i y_i^2 < 1 (summed in i); z = (r1 y_1, r2 y_2, ...);*/
/*      x_i = centre_i + sum_j H_ij z_j (summed in j); accept iff x in B    */
/*   C: x_i = mid_i + half_i y_i; accept iff x in B and                     */
/*      sqrt(sum_i (x_i - q0_i)^2) + sqrt(sum_i (x_i - qg_i)^2) <= c        */
/* with the Householder reflection H = I - s w w^T, w = e_1 - a_1,          */
/* s = 2 / (w^T w), a_1 = (q_g - q0)/c_min, H = I when w = 0; the bounding  */
/* half-extents e_i = sqrt(sum_j (H_ij r_j)^2) * (1 + 2^-10) (the factor    */
/* keeps FP32 rounding from shaving the hyperspheroid's extreme points off),*/
/* C = [max(lo, centre - e), min(hi, centre + e)], mid = (C_lo + C_hi)/2,   */
/* half = (C_hi - C_lo)/2, |R| = prod_i (2 r_i) and |C| = prod_i (C_hi_i -  */
/* C_lo_i) multiplied in i; C is used iff |C| < |R|.                        */
/* Random words: key (seed lo, seed hi), counter                            */
/*   (n, m, stage, (1 << 16) | (2 * attempt + block)), block = j div 4.     */
/* Attempts are unbounded in the definition; the implementation stops after */
/* OR_INFORMED_ATTEMPTS (at least 3 % of the proposals are accepted on      */
/* every workload and bound measured, so the cap is reached with            */
/* probability below 0.97^16384 < e^-499) and then returns the centre, a    */
/* point of X_f(c) n B, with the count -1.                                  */
/* ------------------------------------------------------------------------ */
#define OR_INFORMED_ATTEMPTS 16384

void or_informed_params(int d, const float *q0, const float *qg, float c, float *centre, float *H,
                        float *r1, float *r2, float *cmin_out)
{
    float acc = 0.0f;
    for (int i = 0; i < d; ++i) {
        float t = qg[i] - q0[i];
        acc = acc + t * t;
    }
    float cmin = sqrtf(acc);
    *cmin_out = cmin;
    for (int i = 0; i < d; ++i) centre[i] = (q0[i] + qg[i]) * 0.5f;
    *r1 = c * 0.5f;
    float sq = c * c - cmin * cmin;
    *r2 = sqrtf(sq > 0.0f ? sq : 0.0f) * 0.5f;
    float w[16];
    float ww = 0.0f;
    for (int i = 0; i < d; ++i) {
        float a = (qg[i] - q0[i]) / cmin;
        w[i] = (i == 0 ? 1.0f : 0.0f) - a;
        ww = ww + w[i] * w[i];
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            float delta = i == j ? 1.0f : 0.0f;
            if (ww == 0.0f) {
                H[i * d + j] = delta;
            } else {
                float s = 2.0f / ww;
                H[i * d + j] = delta - (s * w[i]) * w[j];
            }
        }
}

/* Proposal choice of the uniform half: writes C's bounds and returns 1 when
 * the clipped bounding box C is used, 0 for the frame box R. */
int or_informed_proposal(int d, const float *lo, const float *hi, const float *centre, const float *H, float r1,
                         float r2, float *c_lo, float *c_hi)
{
    float vol_r = 1.0f, vol_c = 1.0f;
    for (int i = 0; i < d; ++i) {
        float acc = 0.0f;
        for (int j = 0; j < d; ++j) {
            float t = H[i * d + j] * (j == 0 ? r1 : r2);
            acc = acc + t * t;
        }
        float e = sqrtf(acc) * 1.0009765625f;
        float a = centre[i] - e, b = centre[i] + e;
        c_lo[i] = a > lo[i] ? a : lo[i];
        c_hi[i] = b < hi[i] ? b : hi[i];
        vol_r = vol_r * ((i == 0 ? r1 : r2) * 2.0f);
        vol_c = vol_c * (c_hi[i] - c_lo[i]);
    }
    return vol_c < vol_r ? 1 : 0;
}

/* Returns the number of attempts used (0 for an unbounded draw), or -1 when
 * the attempt cap was reached. */
int or_sample_informed(int d, const float *lo, const float *hi, const float *q0, const float *qg, float c,
                       float penalty, uint64_t seed, uint64_t stage, uint32_t m, uint32_t n, int max_attempts,
                       float *out)
{
    int bounded = !(isinf(c) || c >= penalty);
    if (bounded) {
        float centre[16], H[256], r1, r2, cmin, c_lo[16], c_hi[16], mid[16], half[16];
        or_informed_params(d, q0, qg, c, centre, H, &r1, &r2, &cmin);
        int clipped = or_informed_proposal(d, lo, hi, centre, H, r1, r2, c_lo, c_hi);
        for (int i = 0; i < d; ++i) {
            mid[i] = (c_lo[i] + c_hi[i]) * 0.5f;
            half[i] = (c_hi[i] - c_lo[i]) * 0.5f;
        }
        if (max_attempts > OR_INFORMED_ATTEMPTS) max_attempts = OR_INFORMED_ATTEMPTS;
        for (int a = 0; a < max_attempts; ++a) {
            float y[16], x[16];
            for (int i = 0; i < d; ++i) {
                uint32_t w[4];
                or_words(seed, stage, 1u, n, m, (uint32_t)(2 * a + i / 4), w);
                y[i] = (float)(w[i % 4] >> 8) * (1.0f / 8388608.0f) - 1.0f;
            }
            int inside = 1;
            if (clipped) {
                float s0 = 0.0f, s1 = 0.0f;
                for (int i = 0; i < d; ++i) {
                    x[i] = mid[i] + half[i] * y[i];
                    if (!(x[i] >= lo[i] && x[i] <= hi[i])) inside = 0;
                    float t0 = x[i] - q0[i], t1 = x[i] - qg[i];
                    s0 = s0 + t0 * t0;
                    s1 = s1 + t1 * t1;
                }
                if (!(sqrtf(s0) + sqrtf(s1) <= c)) inside = 0;
            } else {
                float s2 = 0.0f;
                for (int i = 0; i < d; ++i) s2 = s2 + y[i] * y[i];
                if (!(s2 < 1.0f)) continue;
                float z[16];
                for (int i = 0; i < d; ++i) z[i] = (i == 0 ? r1 : r2) * y[i];
                for (int i = 0; i < d; ++i) {
                    float acc = 0.0f;
                    for (int j = 0; j < d; ++j) acc = acc + H[i * d + j] * z[j];
                    x[i] = centre[i] + acc;
                    if (!(x[i] >= lo[i] && x[i] <= hi[i])) inside = 0;
                }
            }
            if (!inside) continue;
            for (int i = 0; i < d; ++i) out[i] = x[i];
            return a + 1;
        }
        for (int i = 0; i < d; ++i) out[i] = centre[i];
        return -1;
    }
    for (int i = 0; i < d; ++i) {
        uint32_t w[4];
        or_words(seed, stage, 1u, n, m, (uint32_t)(i / 4), w);
        double u = or_unit_from_word(w[i % 4]);
        double width = (double)(float)((double)hi[i] - (double)lo[i]);
        out[i] = (float)((double)lo[i] + u * width);
    }
    return 0;
}

/* Coin of the sample mixture (Sec. III-A): heuristic half iff the top bit of
 * word 0 at counter (n, m, stage, 2 << 16) is set. */
int or_coin_heuristic(uint64_t seed, uint64_t stage, uint32_t m, uint32_t n)
{
    uint32_t w[4];
    or_words(seed, stage, 2u, n, m, 0u, w);
    return (int)(w[0] >> 31);
}

/* Squared distance between two configurations, FP32, summed in coordinate
 * order without fused multiply-add: the ranking of sample pairs by it is an
 * integer decision both sides take in the same precision. */
float or_pair_d2(int d, const float *u, const float *v)
{
    float acc = 0.0f;
    for (int i = 0; i < d; ++i) {
        float t = u[i] - v[i];
        acc = acc + t * t;
    }
    return acc;
}

void or_pair_d2_all(int d, int nu, const float *U, int nv, const float *V, float *out /* [nu][nv] */)
{
#pragma omp parallel for schedule(static)
    for (int a = 0; a < nu; ++a)
        for (int b = 0; b < nv; ++b) out[(size_t)a * nv + b] = or_pair_d2(d, U + (size_t)a * d, V + (size_t)b * d);
}

/* ------------------------------------------------------------------------ */
/* RRT-Connect local planner LP(x, y; s, ell) (Sec. III, generalized GTMP   */
/* graph; construction in the proof of the local-planner reach proposition  */
/* of the appendix): confined to the query ellipsoid E(x, y; ell) = {z :    */
/* |z - x| + |z - y| <= ell}, ell = ell_factor |y - x|, the straight line   */
/* already having failed (short-range exactness is the caller's straight-   */
/* line check).  Two trees rooted at x and y; iteration i (i < s) draws one */
/* uniform sample of the ellipsoid intersected with the box, extends tree A */
/* towards it by at most eta, and on success connects tree B greedily to    */
/* the new node; then the trees swap roles.                                 */
/*                                                                          */
/* Decisions are FP32 computations with a fixed operation order (this file  */
/* is compiled without contraction):                                        */
/*   sample   attempt a of iteration i: y_j = (w_j >> 8) 2^-23 - 1, words   */
/*            from Philox at counter (e, i, stage, (3 << 16) | (2a + j/4));  */
/*            accepted iff sum y_j^2 < 1 and x = c + H (r1 y_1, r2 y_2, ...) */
/*            lies in the box (the hyperspheroid map of the informed set    */
/*            with foci x, y and major axis ell); at most 4096 attempts,    */
/*            none accepted = no extension this iteration                   */
/*   nearest  least FP32 squared distance summed in coordinate order,       */
/*            lowest node index on ties                                     */
/*   steer    dist = sqrt(d2); dist <= eta: the target itself (Reached);    */
/*            else p + (eta / dist) (q - p), each operation rounded         */
/*   check    the segment p -> q_new at H_s = max(2, ceil(len / res) + 1)   */
/*            states (len its FP32 length), signed distance <= 0 collides   */
/*   full     a tree holding `cap` nodes extends no further (Trapped)       */
/* A path is x -> ... -> q_new -> ... -> y along the two trees; its cost is */
/* its length.  Collision decisions are FP64 signed distances here; a       */
/* segment whose minimum lies within `band` of zero sets *near_band, so a   */
/* test can excuse calls whose result hinges on such a state.               */
/* ------------------------------------------------------------------------ */
#define OR_RRTC_TRAPPED 0
#define OR_RRTC_ADVANCED 1
#define OR_RRTC_REACHED 2
#define OR_RRTC_ATTEMPTS 4096

typedef struct {
    float *pos; /* [cap][d] */
    int *par;   /* [cap] */
    int n;
} or_tree;

static int or_segment_free(const or_model *mdl, const float *a, const float *b, float res, double band,
                           int *near_band)
{
    int d = mdl->d;
    float len = sqrtf(or_pair_d2(d, a, b));
    int Hs = (int)ceilf(len / res) + 1;
    if (Hs < 2) Hs = 2;
    double c, sd;
    int f;
    or_edge(mdl, Hs, INFINITY, INFINITY, a, b, &c, &sd, &f);
    if (fabs(sd) <= band) *near_band = 1;
    return f == 0;
}

static int or_extend(const or_model *mdl, or_tree *T, int cap, const float *q, float eta, float res, double band,
                     int *near_band, int *new_idx)
{
    int d = mdl->d;
    if (T->n >= cap) return OR_RRTC_TRAPPED;
    int near = 0;
    float best = or_pair_d2(d, T->pos, q);
    for (int j = 1; j < T->n; ++j) {
        float v = or_pair_d2(d, T->pos + (size_t)j * d, q);
        if (v < best) {
            best = v;
            near = j;
        }
    }
    const float *p = T->pos + (size_t)near * d;
    float dist = sqrtf(best);
    float qn[16];
    int reached = dist <= eta;
    if (reached) {
        for (int i = 0; i < d; ++i) qn[i] = q[i];
    } else {
        float f = eta / dist;
        for (int i = 0; i < d; ++i) qn[i] = p[i] + f * (q[i] - p[i]);
    }
    if (!or_segment_free(mdl, p, qn, res, band, near_band)) return OR_RRTC_TRAPPED;
    memcpy(T->pos + (size_t)T->n * d, qn, sizeof(float) * d);
    T->par[T->n] = near;
    *new_idx = T->n;
    T->n += 1;
    return reached ? OR_RRTC_REACHED : OR_RRTC_ADVANCED;
}

/* Sample of iteration i: 1 and the point in q, or 0 when no attempt passed. */
int or_rrtc_sample(int d, const float *lo, const float *hi, const float *centre, const float *H, float r1, float r2,
                   uint64_t seed, uint64_t stage, uint32_t e, uint32_t i, float *q)
{
    for (int a = 0; a < OR_RRTC_ATTEMPTS; ++a) {
        float y[16], z[16];
        float s2 = 0.0f;
        for (int j = 0; j < d; ++j) {
            uint32_t w[4];
            or_words(seed, stage, 3u, e, i, (uint32_t)(2 * a + j / 4), w);
            y[j] = (float)(w[j % 4] >> 8) * (1.0f / 8388608.0f) - 1.0f;
            s2 = s2 + y[j] * y[j];
        }
        if (!(s2 < 1.0f)) continue;
        for (int j = 0; j < d; ++j) z[j] = (j == 0 ? r1 : r2) * y[j];
        int inside = 1;
        for (int r = 0; r < d; ++r) {
            float acc = 0.0f;
            for (int c = 0; c < d; ++c) acc = acc + H[r * d + c] * z[c];
            q[r] = centre[r] + acc;
            if (!(q[r] >= lo[r] && q[r] <= hi[r])) inside = 0;
        }
        if (inside) return 1;
    }
    return 0;
}

/* One call.  Returns 1 on success.  path [2 cap][d] (may be NULL) receives
 * the waypoints from x to y, *n_path their count; *cost the path length
 * (FP64 sum of segment lengths); *iters the iterations run; sizes[2] the
 * node counts of the x and y trees; trees (may be NULL) [2][cap][d] and
 * parents (may be NULL) [2][cap] the trees themselves. */
int or_rrtc(const or_model *mdl, const float *x, const float *y, const float *lo, const float *hi, int budget,
            int cap, float eta, float res, float ell_factor, uint64_t seed, uint64_t stage, uint32_t e, double band,
            float *path, int *n_path, double *cost, int *iters, int *sizes, int *near_band, float *trees,
            int *parents)
{
    int d = mdl->d;
    or_tree TX, TY;
    TX.pos = (float *)malloc(sizeof(float) * (size_t)cap * d);
    TY.pos = (float *)malloc(sizeof(float) * (size_t)cap * d);
    TX.par = (int *)malloc(sizeof(int) * (size_t)cap);
    TY.par = (int *)malloc(sizeof(int) * (size_t)cap);
    memcpy(TX.pos, x, sizeof(float) * d);
    memcpy(TY.pos, y, sizeof(float) * d);
    TX.par[0] = TY.par[0] = -1;
    TX.n = TY.n = 1;
    *near_band = 0;
    float cmin = sqrtf(or_pair_d2(d, x, y));
    float ell = ell_factor * cmin;
    float centre[16], H[256], r1, r2, cm2;
    or_informed_params(d, x, y, ell, centre, H, &r1, &r2, &cm2);
    or_tree *Ta = &TX, *Tb = &TY;
    int ok = 0, ax = -1, ay = -1, it = 0;
    for (it = 0; it < budget && !ok; ++it) {
        float q[16];
        if (or_rrtc_sample(d, lo, hi, centre, H, r1, r2, seed, stage, e, (uint32_t)it, q)) {
            int ia = -1;
            if (or_extend(mdl, Ta, cap, q, eta, res, band, near_band, &ia) != OR_RRTC_TRAPPED) {
                float qn[16];
                memcpy(qn, Ta->pos + (size_t)ia * d, sizeof(float) * d);
                int ib = -1, st;
                do {
                    st = or_extend(mdl, Tb, cap, qn, eta, res, band, near_band, &ib);
                } while (st == OR_RRTC_ADVANCED);
                if (st == OR_RRTC_REACHED) {
                    ok = 1;
                    ax = Ta == &TX ? ia : ib;
                    ay = Ta == &TX ? ib : ia;
                }
            }
        }
        or_tree *t = Ta;
        Ta = Tb;
        Tb = t;
    }
    *iters = it;
    sizes[0] = TX.n;
    sizes[1] = TY.n;
    *cost = INFINITY;
    *n_path = 0;
    if (ok) {
        /* x-tree chain root -> ax, then the y-tree chain from the parent of ay
         * (ay duplicates the junction) to its root */
        int chain[2 * 4096 + 2];
        int nx = 0;
        for (int j = ax; j >= 0; j = TX.par[j]) chain[nx++] = j;
        int np = 0;
        double L = 0.0;
        const float *prev = NULL;
        for (int k = nx - 1; k >= 0; --k) {
            const float *p = TX.pos + (size_t)chain[k] * d;
            if (path) memcpy(path + (size_t)np * d, p, sizeof(float) * d);
            if (prev) {
                double s2 = 0.0;
                for (int i = 0; i < d; ++i) s2 += ((double)p[i] - prev[i]) * ((double)p[i] - prev[i]);
                L += sqrt(s2);
            }
            prev = p;
            ++np;
        }
        for (int j = TY.par[ay]; j >= 0; j = TY.par[j]) {
            const float *p = TY.pos + (size_t)j * d;
            if (path) memcpy(path + (size_t)np * d, p, sizeof(float) * d);
            double s2 = 0.0;
            for (int i = 0; i < d; ++i) s2 += ((double)p[i] - prev[i]) * ((double)p[i] - prev[i]);
            L += sqrt(s2);
            prev = p;
            ++np;
        }
        *n_path = np;
        *cost = L;
    }
    if (trees) {
        memcpy(trees, TX.pos, sizeof(float) * (size_t)TX.n * d);
        memcpy(trees + (size_t)cap * d, TY.pos, sizeof(float) * (size_t)TY.n * d);
    }
    if (parents) {
        memcpy(parents, TX.par, sizeof(int) * (size_t)TX.n);
        memcpy(parents + cap, TY.par, sizeof(int) * (size_t)TY.n);
    }
    free(TX.pos);
    free(TY.pos);
    free(TX.par);
    free(TY.par);
    return ok;
}

/* Many calls (OpenMP over calls): X, Y [n][d], ids [n] the edge ids that key
 * the random streams; outputs per call. */
void or_rrtc_batch(const or_model *mdl, int n, const float *X, const float *Y, const uint32_t *ids,
                   const float *lo, const float *hi, int budget, int cap, float eta, float res, float ell_factor,
                   uint64_t seed, uint64_t stage, double band, int *ok, double *cost, int *iters, int *sizes,
                   int *near_band, int *n_path)
{
    int d = mdl->d;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n; ++k)
        ok[k] = or_rrtc(mdl, X + (size_t)k * d, Y + (size_t)k * d, lo, hi, budget, cap, eta, res, ell_factor, seed,
                        stage, ids[k], band, NULL, &n_path[k], &cost[k], &iters[k], sizes + 2 * k, &near_band[k],
                        NULL, NULL);
}
