/*
 * rxcond_oracle.c -- plain FP64 CPU oracle for the paper's receiver-
 * conditioned radiance (RxGS, arXiv 2605.24290): the directional basis of
 * App. E.2, the global (FiLM) branch of Sec. 4.3.2 eqs. (film, film_apply),
 * the local branch of eqs. (transmittance, local, combined_local) with the
 * occupancy grid of App. E.5, and the reduction of Alg. 1 stage 2
 * (rxcond.forward_batched, then eval_fle against the shared basis).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path never
 * calls it, and it shares no code, header, table or helper with the HIP path.
 *
 * Per Gaussian k: base coefficients phi_k[l][c] = a + i b (complex), one per
 * basis component l = (deg, ord) with index deg^2 + deg + ord, and channel c.
 * Per receiver j (position r) and Gaussian k (position p, seen from the view
 * centre t along d = (p - t) / |p - t|):
 *
 *   gamma(r)   = [sin(W_i . r), cos(W_i . r)]_{i < 3F}           (eq. rx_enc)
 *   (alpha, beta)_{l,c} = MLP_g([gamma(r); (deg, ord) / max(lmax, 1); e_l])
 *                                                                (eq. film)
 *   phi~ = (1 + alpha) phi_k + beta    (complex, per l and c)    (eq. film_apply)
 *   probes q_s = p + t_s (r - p), t_s = 0.05 + 0.9 s / (S - 1)   (App. E.5)
 *   T_k = prod_s (1 - V(q_s)), rho_k = mean_s V(q_s)             (eq. transmittance)
 *   (alpha', beta')_c = MLP_l([(r - p)/|r - p|; |r - p|; T_k; rho_k])
 *                                                                (eq. local)
 *   phi_{l,c} = (1 + alpha'_c) phi~_{l,c} + beta'_c              (eq. combined_local)
 *   s_c = sum_l phi_{l,c} B_l(d)                                 (App. E.2; Alg. 1 l. eval_fle)
 *
 * with complex products throughout.  The local branch gives one complex
 * scale and shift per (receiver, Gaussian, channel), shared by every
 * component: App. E.5 calls them per-Gaussian parameters (the global ones
 * per-component), and Sec. 4.3.2 puts the conditioning's cost at O(L + K).
 * B_l is the basis:
 *   FLE (complex): B_{deg,ord} = N P_deg^|ord|(cos th) e^{i ord ph}, so that
 *     Re s = sum [a cos(ord ph) - b sin(ord ph)] N P and
 *     Im s = sum [a sin(ord ph) + b cos(ord ph)] N P       (App. E.2)
 *   SH (real): Y_{deg,0} = N P, Y_{deg,ord>0} = sqrt2 N P cos(ord ph),
 *     Y_{deg,ord<0} = sqrt2 N P_deg^|ord| sin(|ord| ph); s = sum phi_l Y_l
 *   N = sqrt((2 deg + 1)/(4 pi) (deg - |ord|)! / (deg + |ord|)!), P the
 *   associated Legendre function without the Condon-Shortley phase, th the
 *   polar angle of d from +z and ph its azimuth.
 *
 * The occupancy grid V (App. E.5: the frozen Gaussians splatted into a G^3
 * grid with a 2 sigma radius): over the box spanned by the means, voxel
 * centres x = lo + (i + 1/2) (hi - lo) / G per axis, and
 *   V(x) = 1 - prod_k (1 - o_k exp(-|x - p_k|^2 / (2 sigma_k^2)))
 * over the Gaussians with |x - p_k| <= 2 sigma_k, o_k = sigmoid(logit_k) and
 * sigma_k the largest of its three scales.  A probe reads the voxel that
 * contains it (nearest voxel centre); a probe outside the box reads 0.
 *
 * MLPs are three Linear layers with ReLU after the first two (App. E.5:
 * "3-layer ReLU MLP"); the hidden width is a parameter.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RC_EMB 16   /* component embedding width d_c (App. E Table 4) */

/* ------------------------------------------------------------------------ */
/* associated Legendre P_deg^ord(x), 0 <= ord <= deg <= lmax, without the
 * Condon-Shortley phase, by the three-term recurrence in deg; s = sin(th) */
static void legendre(int lmax, double x, double s, double *P /* (lmax+1)^2, index deg*(lmax+1)+ord */)
{
    const int n = lmax + 1;
    for (int i = 0; i < n * n; i++) P[i] = 0.0;
    double pmm = 1.0;
    for (int m = 0; m <= lmax; m++) {
        if (m > 0) pmm = pmm * (2.0 * m - 1.0) * s;      /* P_m^m = (2m-1)!! s^m */
        P[m * n + m] = pmm;
        if (m + 1 <= lmax) P[(m + 1) * n + m] = x * (2.0 * m + 1.0) * pmm;
        for (int l = m + 2; l <= lmax; l++)
            P[l * n + m] = ((2.0 * l - 1.0) * x * P[(l - 1) * n + m] - (l + m - 1.0) * P[(l - 2) * n + m]) / (l - m);
    }
}

static double norm_lm(int l, int m)
{
    double r = (2.0 * l + 1.0) / (4.0 * M_PI);
    for (int i = l - m + 1; i <= l + m; i++) r /= (double)i;   /* (l-m)!/(l+m)! */
    return sqrt(r);
}

/*
 * Basis at direction (dx, dy, dz) (any length > 0): B[2 idx] = Re, B[2 idx + 1]
 * = Im for idx = deg^2 + deg + ord.  kind 0: FLE (complex), 1: real SH (Im = 0).
 */
int orc_basis(int kind, int lmax, double dx, double dy, double dz, double *B)
{
    if (lmax < 0 || lmax > 20 || (kind != 0 && kind != 1)) return -1;
    const double h = sqrt(dx * dx + dy * dy);
    const double rho = sqrt(h * h + dz * dz);
    if (!(rho > 0.0)) return -1;
    const double x = dz / rho, s = h / rho;
    const double ph = atan2(dy, dx);
    const int n = lmax + 1;
    double *P = malloc(sizeof(double) * (size_t)n * n);
    legendre(lmax, x, s, P);
    for (int l = 0; l <= lmax; l++)
        for (int m = -l; m <= l; m++) {
            const int am = m < 0 ? -m : m;
            const double np = norm_lm(l, am) * P[l * n + am];
            const int idx = l * l + l + m;
            if (kind == 0) {
                B[2 * idx] = np * cos(m * ph);
                B[2 * idx + 1] = np * sin(m * ph);
            } else {
                B[2 * idx] = m == 0 ? np : (m > 0 ? sqrt(2.0) * np * cos(am * ph) : sqrt(2.0) * np * sin(am * ph));
                B[2 * idx + 1] = 0.0;
            }
        }
    free(P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* occupancy grid */
typedef struct {
    int K, G, nthreads;
    const double *means, *ls, *logits;
    double lo[3], hi[3];
    double *acc;   /* nthreads x G^3 sums of log(1 - o G) */
    long next;
} occ_ctx;

static void *occ_worker(void *arg)
{
    occ_ctx *c = arg;
    for (;;) {
        long it = __atomic_fetch_add(&c->next, 1, __ATOMIC_SEQ_CST);
        if (it >= (long)c->nthreads) break;
        const int tid = (int)it;
        double *acc = c->acc + (size_t)tid * c->G * c->G * c->G;
        const int G = c->G;
        double vs[3];
        for (int a = 0; a < 3; a++) vs[a] = (c->hi[a] - c->lo[a]) / G;
        for (int k = tid; k < c->K; k += c->nthreads) {
            const double *p = c->means + 3 * k;
            double lsm = c->ls[3 * k];
            if (c->ls[3 * k + 1] > lsm) lsm = c->ls[3 * k + 1];
            if (c->ls[3 * k + 2] > lsm) lsm = c->ls[3 * k + 2];
            const double sig = exp(lsm);
            const double o = 1.0 / (1.0 + exp(-c->logits[k]));
            const double r2 = 4.0 * sig * sig;
            int i0[3], i1[3];
            for (int a = 0; a < 3; a++) {
                /* conservative voxel range of the 2 sigma ball (one voxel of slack) */
                i0[a] = (int)floor((p[a] - 2.0 * sig - c->lo[a]) / vs[a]) - 1;
                i1[a] = (int)floor((p[a] + 2.0 * sig - c->lo[a]) / vs[a]) + 1;
                if (i0[a] < 0) i0[a] = 0;
                if (i1[a] > G - 1) i1[a] = G - 1;
            }
            for (int iz = i0[2]; iz <= i1[2]; iz++)
                for (int iy = i0[1]; iy <= i1[1]; iy++)
                    for (int ix = i0[0]; ix <= i1[0]; ix++) {
                        const double xx = c->lo[0] + (ix + 0.5) * vs[0] - p[0];
                        const double yy = c->lo[1] + (iy + 0.5) * vs[1] - p[1];
                        const double zz = c->lo[2] + (iz + 0.5) * vs[2] - p[2];
                        const double d2 = xx * xx + yy * yy + zz * zz;
                        if (!(d2 <= r2)) continue;
                        acc[((size_t)iz * G + iy) * G + ix] += log1p(-o * exp(-0.5 * d2 / (sig * sig)));
                    }
        }
    }
    return NULL;
}

/*
 * Occupancy grid of K Gaussians (means K x 3, log-scales K x 3, logits K):
 * lo / hi (3 each, out) = the componentwise min / max of the means (an axis of
 * zero extent gets hi = lo + 1e-6); grid (out) G^3 values, x fastest.
 */
int orc_occupancy(int K, const double *means, const double *log_scales, const double *logits, int G,
                  int nthreads, double *lo, double *hi, double *grid)
{
    if (K < 0 || G < 1 || G > 1024) return -1;
    for (int a = 0; a < 3; a++) {
        lo[a] = K > 0 ? means[a] : 0.0;
        hi[a] = K > 0 ? means[a] : 0.0;
    }
    for (int k = 0; k < K; k++)
        for (int a = 0; a < 3; a++) {
            if (means[3 * k + a] < lo[a]) lo[a] = means[3 * k + a];
            if (means[3 * k + a] > hi[a]) hi[a] = means[3 * k + a];
        }
    for (int a = 0; a < 3; a++)
        if (!(hi[a] - lo[a] >= 1e-6)) hi[a] = lo[a] + 1e-6;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    const size_t n3 = (size_t)G * G * G;
    occ_ctx c;
    memset(&c, 0, sizeof c);
    c.K = K; c.G = G; c.nthreads = nthreads; c.means = means; c.ls = log_scales; c.logits = logits;
    memcpy(c.lo, lo, sizeof c.lo);
    memcpy(c.hi, hi, sizeof c.hi);
    c.acc = calloc((size_t)nthreads * n3, sizeof(double));
    if (!c.acc) return -2;
    pthread_t th[64];
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, occ_worker, &c);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    for (size_t i = 0; i < n3; i++) {
        double s = 0.0;
        for (int t = 0; t < nthreads; t++) s += c.acc[(size_t)t * n3 + i];
        grid[i] = -expm1(s);   /* 1 - prod (1 - o G) */
    }
    free(c.acc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* parameters of the conditioning, one flat vector in this order:
 *   W  (3F x 3)      Fourier frequency vectors (eq. rx_enc)
 *   E  (L x 16)      component embeddings e_l
 *   global MLP: W1 (Hd x (6F + 2 + 16)), b1 (Hd), W2 (Hd x Hd), b2 (Hd),
 *               W3 (4C x Hd), b3 (4C); output rows 4c + (alpha re, alpha im,
 *               beta re, beta im)
 *   local MLP:  W1 (Hd x 6), b1 (Hd), W2 (Hd x Hd), b2 (Hd),
 *               W3 (4C x Hd), b3 (4C); output rows 4c + (...)
 * Matrices row-major (out x in). */
typedef struct {
    int L, C, F, H;
    const double *W, *E;
    const double *g1, *gb1, *g2, *gb2, *g3, *gb3;
    const double *l1, *lb1, *l2, *lb2, *l3, *lb3;
} rc_params;

static long rc_count(int lmax, int C, int F, int H)
{
    const long L = (long)(lmax + 1) * (lmax + 1);
    const long gin = 6L * F + 2 + RC_EMB;
    return 9L * F + L * RC_EMB + (H * gin + H + (long)H * H + H + 4L * C * H + 4L * C) +
           (H * 6L + H + (long)H * H + H + 4L * C * H + 4L * C);
}

long orc_rxcond_param_count(int lmax, int C, int F, int H) { return rc_count(lmax, C, F, H); }

static rc_params rc_view(const double *q, int lmax, int C, int F, int H)
{
    rc_params r;
    r.L = (lmax + 1) * (lmax + 1); r.C = C; r.F = F; r.H = H;
    const int gin = 6 * F + 2 + RC_EMB;
    r.W = q; q += 9 * F;
    r.E = q; q += r.L * RC_EMB;
    r.g1 = q; q += H * gin;
    r.gb1 = q; q += H;
    r.g2 = q; q += H * H;
    r.gb2 = q; q += H;
    r.g3 = q; q += 4 * C * H;
    r.gb3 = q; q += 4 * C;
    r.l1 = q; q += H * 6;
    r.lb1 = q; q += H;
    r.l2 = q; q += H * H;
    r.lb2 = q; q += H;
    r.l3 = q; q += 4 * C * H;
    r.lb3 = q;
    return r;
}

/* three Linear layers, ReLU after the first two; out has nout values */
static void mlp3(const double *x, int nin, int H, int nout, const double *W1, const double *b1, const double *W2,
                 const double *b2, const double *W3, const double *b3, double *h1, double *h2, double *out)
{
    for (int o = 0; o < H; o++) {
        double a = b1[o];
        for (int i = 0; i < nin; i++) a += W1[o * nin + i] * x[i];
        h1[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < H; o++) {
        double a = b2[o];
        for (int i = 0; i < H; i++) a += W2[o * H + i] * h1[i];
        h2[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < nout; o++) {
        double a = b3[o];
        for (int i = 0; i < H; i++) a += W3[o * H + i] * h2[i];
        out[o] = a;
    }
}

/* global branch of one receiver: ab (L x C x 4) */
static void global_branch(const rc_params *P, int lmax, const double *r, double *ab)
{
    const int gin = 6 * P->F + 2 + RC_EMB;
    double *x = malloc(sizeof(double) * gin);
    double *h1 = malloc(sizeof(double) * P->H), *h2 = malloc(sizeof(double) * P->H);
    for (int i = 0; i < 3 * P->F; i++) {
        const double a = P->W[3 * i] * r[0] + P->W[3 * i + 1] * r[1] + P->W[3 * i + 2] * r[2];
        x[2 * i] = sin(a);
        x[2 * i + 1] = cos(a);
    }
    const double dn = lmax > 0 ? (double)lmax : 1.0;
    for (int l = 0; l <= lmax; l++)
        for (int m = -l; m <= l; m++) {
            const int idx = l * l + l + m;
            x[6 * P->F] = l / dn;
            x[6 * P->F + 1] = m / dn;
            for (int e = 0; e < RC_EMB; e++) x[6 * P->F + 2 + e] = P->E[idx * RC_EMB + e];
            mlp3(x, gin, P->H, 4 * P->C, P->g1, P->gb1, P->g2, P->gb2, P->g3, P->gb3, h1, h2,
                 ab + (size_t)idx * P->C * 4);
        }
    free(x); free(h1); free(h2);
}

/* local features of (receiver r, Gaussian p): the 6 inputs of eq. local */
static void local_features(const double *r, const double *p, const double *grid, int G, const double *lo,
                           const double *hi, int S, double *f)
{
    const double vx = r[0] - p[0], vy = r[1] - p[1], vz = r[2] - p[2];
    const double d = sqrt(vx * vx + vy * vy + vz * vz);
    double inv[3];
    for (int a = 0; a < 3; a++) inv[a] = (double)G / (hi[a] - lo[a]);
    double T = 1.0, sum = 0.0;
    for (int s = 0; s < S; s++) {
        double t = 0.9 * (double)s;
        t = t / (double)(S - 1);
        t = 0.05 + t;
        int idx[3], inside = 1;
        for (int a = 0; a < 3; a++) {
            const double q = p[a] + t * (r[a] - p[a]);
            const double u = (q - lo[a]) * inv[a];
            const double fl = floor(u);
            if (!(fl >= 0.0 && fl <= (double)(G - 1))) inside = 0;
            idx[a] = inside ? (int)fl : 0;
        }
        const double v = inside ? grid[((size_t)idx[2] * G + idx[1]) * G + idx[0]] : 0.0;
        T *= 1.0 - v;
        sum += v;
    }
    f[0] = d > 0.0 ? vx / d : 0.0;
    f[1] = d > 0.0 ? vy / d : 0.0;
    f[2] = d > 0.0 ? vz / d : 0.0;
    f[3] = d;
    f[4] = T;
    f[5] = sum / (double)S;
}

/* complex a * b */
static void cmul(double ar, double ai, double br, double bi, double *cr, double *ci)
{
    *cr = ar * br - ai * bi;
    *ci = ar * bi + ai * br;
}

typedef struct {
    int K, N, lmax, kind, C, F, H, S, G;
    const double *means, *coeffs, *centres, *rx, *grid, *lo, *hi;
    const int *rx_view;
    rc_params P;
    double *rad;     /* N x C x K x 2 */
    double *feats;   /* optional N x K x 6 */
    long next, n;
} rad_ctx;

static void *rad_worker(void *arg)
{
    rad_ctx *c = arg;
    const int L = c->P.L, C = c->C, H = c->H;
    double *ab = malloc(sizeof(double) * (size_t)L * C * 4);
    double *loc = malloc(sizeof(double) * (size_t)C * 4);
    double *h1 = malloc(sizeof(double) * H), *h2 = malloc(sizeof(double) * H);
    double *B = malloc(sizeof(double) * (size_t)L * 2);
    for (;;) {
        long j = __atomic_fetch_add(&c->next, 1, __ATOMIC_SEQ_CST);
        if (j >= c->n) break;
        const double *r = c->rx + 3 * j;
        const double *cen = c->centres + 3 * c->rx_view[j];
        global_branch(&c->P, c->lmax, r, ab);
        for (int k = 0; k < c->K; k++) {
            const double *p = c->means + 3 * k;
            double f[6];
            local_features(r, p, c->grid, c->G, c->lo, c->hi, c->S, f);
            if (c->feats) memcpy(c->feats + ((size_t)j * c->K + k) * 6, f, sizeof f);
            mlp3(f, 6, H, 4 * C, c->P.l1, c->P.lb1, c->P.l2, c->P.lb2, c->P.l3, c->P.lb3, h1, h2, loc);
            const double dx = p[0] - cen[0], dy = p[1] - cen[1], dz = p[2] - cen[2];
            if (orc_basis(c->kind, c->lmax, dx, dy, dz, B) != 0)
                for (int i = 0; i < 2 * L; i++) B[i] = 0.0;   /* Gaussian at the view centre */
            for (int ch = 0; ch < C; ch++) {
                double sr = 0.0, si = 0.0;
                for (int l = 0; l < L; l++) {
                    const double *g = ab + ((size_t)l * C + ch) * 4;
                    const double *q = loc + (size_t)ch * 4;
                    const double *ph = c->coeffs + (((size_t)k * L + l) * C + ch) * 2;
                    double tr, ti, ur, ui, vr, vi;
                    cmul(1.0 + g[0], g[1], ph[0], ph[1], &tr, &ti);         /* (1 + alpha) phi */
                    tr += g[2]; ti += g[3];                                  /* + beta */
                    cmul(1.0 + q[0], q[1], tr, ti, &ur, &ui);               /* (1 + alpha') phi~ */
                    ur += q[2]; ui += q[3];                                  /* + beta' */
                    cmul(ur, ui, B[2 * l], B[2 * l + 1], &vr, &vi);         /* times the basis */
                    sr += vr; si += vi;
                }
                double *o = c->rad + (((size_t)j * C + ch) * c->K + k) * 2;
                o[0] = sr; o[1] = si;
            }
        }
    }
    free(ab); free(loc); free(h1); free(h2); free(B);
    return NULL;
}

/*
 * Conditioned radiance of every (receiver, Gaussian, channel).
 *   kind 0 FLE, 1 real SH; lmax; C channels; F bands; H hidden width; S probes;
 *   means K x 3; coeffs K x L x C x 2; params (orc_rxcond_param_count values);
 *   centres V x 3 view centres; rx N x 3 receivers; rx_view N;
 *   grid G^3 with its box lo / hi (orc_occupancy).
 * Out: rad N x C x K x 2; feats (optional) N x K x 6 local-branch inputs.
 */
int orc_rxcond_radiance(int kind, int lmax, int C, int F, int H, int S, int K, const double *means,
                        const double *coeffs, const double *params, int V, const double *centres, int N,
                        const double *rx, const int *rx_view, int G, const double *lo, const double *hi,
                        const double *grid, int nthreads, double *rad, double *feats)
{
    if (lmax < 0 || lmax > 20 || C < 1 || F < 1 || H < 1 || S < 2 || K < 0 || N < 0 || V < 1 || G < 1) return -1;
    for (int j = 0; j < N; j++)
        if (rx_view[j] < 0 || rx_view[j] >= V) return -1;
    rad_ctx c;
    memset(&c, 0, sizeof c);
    c.K = K; c.N = N; c.lmax = lmax; c.kind = kind; c.C = C; c.F = F; c.H = H; c.S = S; c.G = G;
    c.means = means; c.coeffs = coeffs; c.centres = centres; c.rx = rx; c.grid = grid; c.lo = lo; c.hi = hi;
    c.rx_view = rx_view; c.P = rc_view(params, lmax, C, F, H); c.rad = rad; c.feats = feats; c.n = N;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, rad_worker, &c);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    return 0;
}
