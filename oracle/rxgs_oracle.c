/*
 * rxgs_oracle.c -- plain FP64 CPU oracle for multi-receiver Gaussian
 * rasterization (RxGS, arXiv 2605.24290).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path never
 * calls it, and it shares no code, header, table or helper with the HIP path.
 *
 * What it computes, each step as the plain definition (no tiling, no fusion):
 *   - Gaussian state and covariance Sigma = R S S^T R^T, with log-space scales,
 *     a (w,x,y,z) quaternion normalised inside, and a sigmoid opacity
 *     (Sec. 2 eq. (1); App. E.1).
 *   - Projection of every Gaussian onto the angular (azimuth x elevation)
 *     grid centred at a view point (Alg. 1 stage 1), linearised at the mean:
 *     Sigma_px = M Sigma M^T + 0.3 I with M the Jacobian of (az/daz, el/del).
 *     The Jacobian of all projected quantities with respect to the 11 raw
 *     Gaussian parameters comes from forward-mode dual numbers.
 *   - Per pixel, all Gaussians of the view in ascending (FP32 squared-distance
 *     key, index) order, composited front to back (Alg. 1 stage 3):
 *       w = min(0.99, o exp(-q/2)); skip if w < 1/255; C += T w s;
 *       T <- T (1 - w); stop once T < 1e-4 (after including that Gaussian).
 *   - Radiance: direct per-Gaussian values, or the conditioning MLP on
 *     [gamma(r_j); f_k] with gamma the per-axis sin/cos Fourier encoding of the
 *     receiver position (Sec. 4.3.2 eq. rx_enc; F = 6 bands, App. E Table 4).
 *   - Outputs: spectrum C, received power P = sum_p |C|^2, coherent sum
 *     S = sum_p C (App. A Def. 2, the aggregation over rays).
 *   - Reverse mode: explicit per-entry transmittances (no division), chained
 *     through the dual-number projection Jacobian and the MLP.
 *   - Integer tile binning of FP32 projection records, for bit-exact checks
 *     of the device-side binning and sort (Alg. 1 stage 1, the sort over
 *     (tile, depth) keys, extended with a view index).
 *
 * Everything is FP64 except the depth key, which is, by definition, the bit
 * pattern of the FP32 value ((dx*dx + dy*dy) + dz*dz) with dx = fl32(px - cx),
 * each operation rounded to FP32 with no fused multiply-add.  Build with
 * -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ALPHA_MIN (1.0 / 255.0)
#define ORC_W_MAX 0.99
#define ORC_T_EPS 1e-4
#define ORC_DILATE 0.3
#define ORC_H_MIN 1e-6
#define ORC_NEAR2_F 0.04f
#define ORC_FEAT 32
#define ORC_ENC 36
#define ORC_HID 64
#define ORC_IN (ORC_ENC + ORC_FEAT)
#define ORC_NMLP (ORC_HID * ORC_IN + ORC_HID + ORC_HID * ORC_HID + ORC_HID + 2 * ORC_HID + 2)

/* ------------------------------------------------------------------------ */
/* forward-mode dual numbers over the 11 raw parameters of one Gaussian:
 * mean (0..2), log-scale (3..5), quaternion w,x,y,z (6..9), opacity logit (10) */
#define NP 11
typedef struct { double v, d[NP]; } dual;

static dual dc(double v) { dual r; r.v = v; memset(r.d, 0, sizeof r.d); return r; }
static dual dvar(double v, int i) { dual r = dc(v); r.d[i] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int i = 0; i < NP; i++) r.d[i] = a.d[i] + b.d[i]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int i = 0; i < NP; i++) r.d[i] = a.d[i] - b.d[i]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int i = 0; i < NP; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
static dual ddiv(dual a, dual b)
{
    dual r; r.v = a.v / b.v;
    for (int i = 0; i < NP; i++) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int i = 0; i < NP; i++) r.d[i] = a.d[i] * s; return r; }
static dual daddc(dual a, double c) { a.v += c; return a; }
static dual dneg(dual a) { return dscale(a, -1.0); }
static dual dsqrt_(dual a) { dual r; r.v = sqrt(a.v); for (int i = 0; i < NP; i++) r.d[i] = a.d[i] / (2.0 * r.v); return r; }
static dual dexp_(dual a) { dual r; r.v = exp(a.v); for (int i = 0; i < NP; i++) r.d[i] = r.v * a.d[i]; return r; }
static dual datan2_(dual y, dual x)
{
    dual r; r.v = atan2(y.v, x.v);
    double den = x.v * x.v + y.v * y.v;
    for (int i = 0; i < NP; i++) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / den;
    return r;
}

/* projected quantities of one (view, Gaussian) */
enum { PU, PV, PA, PB, PC, PO, PCOVA, PCOVB, PCOVC, NPROJ };

typedef struct {
    int H, W;
    double el0, del, daz;
} orc_grid;

static orc_grid mkgrid(int H, int W, double el0, double del)
{
    orc_grid g; g.H = H; g.W = W; g.el0 = el0; g.del = del; g.daz = 2.0 * M_PI / (double)W;
    return g;
}

/* out[NPROJ] duals: u, v, conic a, b, c, opacity, covariance A, B, Cc */
static void project_dual(const double *p, const double *ls, const double *q, double logit,
                         const double *c, const orc_grid *g, dual *out)
{
    dual px = dvar(p[0], 0), py = dvar(p[1], 1), pz = dvar(p[2], 2);
    dual l0 = dvar(ls[0], 3), l1 = dvar(ls[1], 4), l2 = dvar(ls[2], 5);
    dual qw = dvar(q[0], 6), qx = dvar(q[1], 7), qy = dvar(q[2], 8), qz = dvar(q[3], 9);
    dual lg = dvar(logit, 10);

    dual dx = daddc(px, -c[0]), dy = daddc(py, -c[1]), dz = daddc(pz, -c[2]);
    dual h = dsqrt_(dadd(dmul(dx, dx), dmul(dy, dy)));
    if (!(h.v >= ORC_H_MIN)) h = dc(ORC_H_MIN);
    dual az = datan2_(dy, dx);
    if (az.v < 0.0) az.v += 2.0 * M_PI;
    dual el = datan2_(dz, h);
    out[PU] = daddc(dscale(az, 1.0 / g->daz), -0.5);
    out[PV] = daddc(dscale(dsub(daddc(el, 0.0), dc(g->el0)), 1.0 / g->del), -0.5);

    /* Jacobian rows of az and el with respect to the mean */
    dual hh = dmul(h, h);
    dual rh2 = dadd(hh, dmul(dz, dz));
    dual jaz[3], jel[3];
    jaz[0] = ddiv(dneg(dy), hh);
    jaz[1] = ddiv(dx, hh);
    jaz[2] = dc(0.0);
    dual rh2h = dmul(rh2, h);
    jel[0] = ddiv(dneg(dmul(dx, dz)), rh2h);
    jel[1] = ddiv(dneg(dmul(dy, dz)), rh2h);
    jel[2] = ddiv(h, rh2);
    dual mu[3], mv[3];
    for (int i = 0; i < 3; i++) { mu[i] = dscale(jaz[i], 1.0 / g->daz); mv[i] = dscale(jel[i], 1.0 / g->del); }

    /* Sigma = R diag(s^2) R^T, R from the normalised quaternion */
    dual qn2 = dadd(dadd(dmul(qw, qw), dmul(qx, qx)), dadd(dmul(qy, qy), dmul(qz, qz)));
    dual qn = dsqrt_(qn2);
    dual w = ddiv(qw, qn), x = ddiv(qx, qn), y = ddiv(qy, qn), z = ddiv(qz, qn);
    dual R[3][3];
    dual one = dc(1.0);
    R[0][0] = dsub(one, dscale(dadd(dmul(y, y), dmul(z, z)), 2.0));
    R[0][1] = dscale(dsub(dmul(x, y), dmul(w, z)), 2.0);
    R[0][2] = dscale(dadd(dmul(x, z), dmul(w, y)), 2.0);
    R[1][0] = dscale(dadd(dmul(x, y), dmul(w, z)), 2.0);
    R[1][1] = dsub(one, dscale(dadd(dmul(x, x), dmul(z, z)), 2.0));
    R[1][2] = dscale(dsub(dmul(y, z), dmul(w, x)), 2.0);
    R[2][0] = dscale(dsub(dmul(x, z), dmul(w, y)), 2.0);
    R[2][1] = dscale(dadd(dmul(y, z), dmul(w, x)), 2.0);
    R[2][2] = dsub(one, dscale(dadd(dmul(x, x), dmul(y, y)), 2.0));
    dual s2[3];
    s2[0] = dexp_(dscale(l0, 2.0));
    s2[1] = dexp_(dscale(l1, 2.0));
    s2[2] = dexp_(dscale(l2, 2.0));
    dual S[3][3];
    for (int r = 0; r < 3; r++)
        for (int cc = 0; cc < 3; cc++) {
            dual acc = dc(0.0);
            for (int i = 0; i < 3; i++) acc = dadd(acc, dmul(dmul(R[r][i], s2[i]), R[cc][i]));
            S[r][cc] = acc;
        }
    dual Smu[3], Smv[3];
    for (int r = 0; r < 3; r++) {
        Smu[r] = dc(0.0); Smv[r] = dc(0.0);
        for (int i = 0; i < 3; i++) { Smu[r] = dadd(Smu[r], dmul(S[r][i], mu[i])); Smv[r] = dadd(Smv[r], dmul(S[r][i], mv[i])); }
    }
    dual A = dc(ORC_DILATE), B = dc(0.0), Cc = dc(ORC_DILATE);
    for (int i = 0; i < 3; i++) {
        A = dadd(A, dmul(mu[i], Smu[i]));
        B = dadd(B, dmul(mu[i], Smv[i]));
        Cc = dadd(Cc, dmul(mv[i], Smv[i]));
    }
    dual det = dsub(dmul(A, Cc), dmul(B, B));
    out[PA] = ddiv(Cc, det);
    out[PB] = ddiv(dneg(B), det);
    out[PC] = ddiv(A, det);
    out[PO] = ddiv(one, dadd(one, dexp_(dneg(lg))));
    out[PCOVA] = A; out[PCOVB] = B; out[PCOVC] = Cc;
}

static float key_float(const double *p, const double *c)
{
    float dx = (float)p[0] - (float)c[0];
    float dy = (float)p[1] - (float)c[1];
    float dz = (float)p[2] - (float)c[2];
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    s = s + zz;
    return s;
}

static uint32_t f2bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* ------------------------------------------------------------------------ */
/* per-view preprocessing: projected values and depth order */
typedef struct {
    int n;              /* visible (not near-culled) Gaussians */
    int *order;         /* Gaussian indices in ascending (key, index) order */
    double *pv;         /* K x NPROJ values */
    double *lnoa;       /* ln(o / alpha_min) per Gaussian */
} view_t;

typedef struct { uint32_t key; int k; } kk_t;
static int cmp_kk(const void *a, const void *b)
{
    const kk_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->k > y->k) - (x->k < y->k);
}

static void view_build(view_t *vw, int K, const double *means, const double *ls, const double *q,
                       const double *logit, const double *c, const orc_grid *g)
{
    vw->pv = malloc(sizeof(double) * (size_t)K * NPROJ);
    vw->lnoa = malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
    vw->order = malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    kk_t *tmp = malloc(sizeof(kk_t) * (size_t)(K > 0 ? K : 1));
    int n = 0;
    for (int k = 0; k < K; k++) {
        float kf = key_float(means + 3 * k, c);
        if (kf < ORC_NEAR2_F) continue;
        dual out[NPROJ];
        project_dual(means + 3 * k, ls + 3 * k, q + 4 * k, logit[k], c, g, out);
        for (int i = 0; i < NPROJ; i++) vw->pv[(size_t)k * NPROJ + i] = out[i].v;
        vw->lnoa[k] = log(out[PO].v / ORC_ALPHA_MIN);
        tmp[n].key = f2bits(kf); tmp[n].k = k; n++;
    }
    qsort(tmp, (size_t)n, sizeof(kk_t), cmp_kk);
    for (int i = 0; i < n; i++) vw->order[i] = tmp[i].k;
    vw->n = n;
    free(tmp);
}

static void view_free(view_t *vw) { free(vw->pv); free(vw->lnoa); free(vw->order); }

/* ------------------------------------------------------------------------ */
/* radiance: receiver encoding and the conditioning MLP */
static void encode_rx(const double *r, double *gam)
{
    for (int d = 0; d < 3; d++)
        for (int f = 0; f < 6; f++) {
            double a = ldexp(r[d], f);
            gam[12 * d + 2 * f + 0] = sin(a);
            gam[12 * d + 2 * f + 1] = cos(a);
        }
}

typedef struct { const double *W1, *b1, *W2, *b2, *W3, *b3; } mlp_t;
static mlp_t mlp_view(const double *m)
{
    mlp_t r;
    r.W1 = m; m += ORC_HID * ORC_IN;
    r.b1 = m; m += ORC_HID;
    r.W2 = m; m += ORC_HID * ORC_HID;
    r.b2 = m; m += ORC_HID;
    r.W3 = m; m += 2 * ORC_HID;
    r.b3 = m;
    return r;
}

/* x (68) -> s (2); keeps pre-activations when z1, z2 are given */
static void mlp_forward(const mlp_t *m, const double *x, double *s, double *z1, double *z2)
{
    double h1[ORC_HID], h2[ORC_HID], a1[ORC_HID], a2[ORC_HID];
    for (int o = 0; o < ORC_HID; o++) {
        double acc = m->b1[o];
        for (int i = 0; i < ORC_IN; i++) acc += m->W1[o * ORC_IN + i] * x[i];
        a1[o] = acc; h1[o] = acc > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < ORC_HID; o++) {
        double acc = m->b2[o];
        for (int i = 0; i < ORC_HID; i++) acc += m->W2[o * ORC_HID + i] * h1[i];
        a2[o] = acc; h2[o] = acc > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < 2; o++) {
        double acc = m->b3[o];
        for (int i = 0; i < ORC_HID; i++) acc += m->W3[o * ORC_HID + i] * h2[i];
        s[o] = acc;
    }
    if (z1) memcpy(z1, a1, sizeof a1);
    if (z2) memcpy(z2, a2, sizeof a2);
}

/* ------------------------------------------------------------------------ */
/* simple thread pool over work items */
typedef struct {
    void (*fn)(void *ctx, long item, int tid);
    void *ctx;
    long n;
    long next;
    int tid_next;
} pool_t;

static void *pool_worker(void *arg)
{
    pool_t *p = arg;
    int tid = __atomic_fetch_add(&p->tid_next, 1, __ATOMIC_SEQ_CST);
    for (;;) {
        long it = __atomic_fetch_add(&p->next, 1, __ATOMIC_SEQ_CST);
        if (it >= p->n) break;
        p->fn(p->ctx, it, tid);
    }
    return NULL;
}

static void pool_run(int nthreads, long n, void (*fn)(void *, long, int), void *ctx)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pool_t p; p.fn = fn; p.ctx = ctx; p.n = n; p.next = 0; p.tid_next = 0;
    if (nthreads == 1) { pool_worker(&p); return; }
    pthread_t th[256];
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, pool_worker, &p);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int K, V, N;
    const double *means, *ls, *quats, *logits, *radiance, *features, *mlp, *centres, *rx;
    const int *rx_view;
    orc_grid g;
    view_t *views;
    double *rad;        /* N x K x 2 */
    const double *rad_rx;   /* given per-receiver radiance N x K x 2, or NULL */
} scene_t;

static void rad_item(void *vctx, long item, int tid)
{
    (void)tid;
    scene_t *s = vctx;
    int j = (int)item;
    if (s->features) {
        mlp_t m = mlp_view(s->mlp);
        double x[ORC_IN], r[3] = { s->rx[3 * j], s->rx[3 * j + 1], s->rx[3 * j + 2] };
        encode_rx(r, x);
        for (int k = 0; k < s->K; k++) {
            for (int i = 0; i < ORC_FEAT; i++) x[ORC_ENC + i] = s->features[(size_t)k * ORC_FEAT + i];
            mlp_forward(&m, x, s->rad + ((size_t)j * s->K + k) * 2, NULL, NULL);
        }
    } else {
        for (int k = 0; k < s->K; k++) {
            s->rad[((size_t)j * s->K + k) * 2 + 0] = s->radiance[2 * k + 0];
            s->rad[((size_t)j * s->K + k) * 2 + 1] = s->radiance[2 * k + 1];
        }
    }
}

static void view_item(void *vctx, long item, int tid)
{
    (void)tid;
    scene_t *s = vctx;
    int v = (int)item;
    view_build(&s->views[v], s->K, s->means, s->ls, s->quats, s->logits, s->centres + 3 * v, &s->g);
}

static int scene_setup(scene_t *s, int nthreads)
{
    s->views = calloc((size_t)(s->V > 0 ? s->V : 1), sizeof(view_t));
    s->rad = malloc(sizeof(double) * 2 * (size_t)(s->N > 0 ? s->N : 1) * (size_t)(s->K > 0 ? s->K : 1));
    if (!s->views || !s->rad) return -1;
    pool_run(nthreads, s->V, view_item, s);
    if (s->rad_rx)
        memcpy(s->rad, s->rad_rx, sizeof(double) * 2 * (size_t)s->N * (size_t)s->K);
    else
        pool_run(nthreads, s->N, rad_item, s);
    return 0;
}

static void scene_free(scene_t *s)
{
    for (int v = 0; v < s->V; v++) view_free(&s->views[v]);
    free(s->views); free(s->rad);
}

/* one composited entry of a pixel */
typedef struct { int k; double T, w, G, du, dv; int clamped; } entry_t;

/* Composite one pixel.  Returns the number of composited entries; fills C,
 * T_final, the decision margin and (optionally) the entry list. */
static int composite_pixel(const scene_t *s, int j, int row, int col, double *C, double *Tfin,
                           double *margin, entry_t *ent, uint64_t *hash, int *nclamp)
{
    const view_t *vw = &s->views[s->rx_view[j]];
    const double W = s->g.W, halfW = 0.5 * s->g.W;
    const double *rad = s->rad + (size_t)j * s->K * 2;
    double T = 1.0, cr = 0.0, ci = 0.0, marg = INFINITY;
    int n = 0, ncl = 0;
    for (int idx = 0; idx < vw->n; idx++) {
        int k = vw->order[idx];
        const double *pv = vw->pv + (size_t)k * NPROJ;
        double du = (double)col - pv[PU];
        double duraw = du;
        if (du >= halfW) du -= W;
        else if (du < -halfW) du += W;
        double dv = (double)row - pv[PV];
        double q = pv[PA] * du * du + 2.0 * pv[PB] * du * dv + pv[PC] * dv * dv;
        /* exact shortcut: q/2 - ln(o/alpha) > 1e-3 means w < alpha with a
         * relative margin above 1e-3, so the entry is skipped either way */
        double lq = 0.5 * q - vw->lnoa[k];
        if (lq > 1e-3) continue;
        double G = exp(-0.5 * q);
        double ow = pv[PO] * G;
        double w = ow < ORC_W_MAX ? ow : ORC_W_MAX;
        double m1 = fabs(w - ORC_ALPHA_MIN) / ORC_ALPHA_MIN;
        if (m1 < marg) marg = m1;
        if (w < ORC_ALPHA_MIN) continue;
        double m2 = fabs(ow - ORC_W_MAX) / ORC_W_MAX;
        if (m2 < marg) marg = m2;
        double m3 = fmin(fabs(duraw - halfW), fabs(duraw + halfW));
        if (m3 < marg) marg = m3;
        if (ent) {
            ent[n].k = k; ent[n].T = T; ent[n].w = w; ent[n].G = G;
            ent[n].du = du; ent[n].dv = dv; ent[n].clamped = ow >= ORC_W_MAX;
        }
        if (hash) {
            uint64_t h = *hash;
            h ^= (uint64_t)(uint32_t)k + ((uint64_t)(ow >= ORC_W_MAX) << 32);
            h *= 1099511628211ULL;
            *hash = h;
        }
        ncl += ow >= ORC_W_MAX;
        cr += T * w * rad[2 * k + 0];
        ci += T * w * rad[2 * k + 1];
        T = T * (1.0 - w);
        n++;
        double m4 = fabs(T - ORC_T_EPS) / ORC_T_EPS;
        if (m4 < marg) marg = m4;
        if (T < ORC_T_EPS) break;
    }
    C[0] = cr; C[1] = ci; *Tfin = T;
    if (margin) *margin = marg;
    if (nclamp) *nclamp = ncl;
    return n;
}

typedef struct {
    scene_t *s;
    double *C, *Tfin, *margin;
    int *ncomp;
    uint64_t *rowhash;
    int *nclamp;
} render_ctx;

static void render_item(void *vctx, long item, int tid)
{
    (void)tid;
    render_ctx *r = vctx;
    const scene_t *s = r->s;
    int H = s->g.H, W = s->g.W;
    int j = (int)(item / H), row = (int)(item % H);
    uint64_t h = 1469598103934665603ULL;
    for (int col = 0; col < W; col++) {
        size_t p = (size_t)row * W + col;
        size_t P = (size_t)H * W;
        double C[2], T, m;
        int ncl = 0;
        int n = composite_pixel(s, j, row, col, C, &T, &m, NULL, r->rowhash ? &h : NULL, &ncl);
        if (r->nclamp) r->nclamp[(size_t)j * P + p] = ncl;
        r->C[((size_t)j * 2 + 0) * P + p] = C[0];
        r->C[((size_t)j * 2 + 1) * P + p] = C[1];
        if (r->Tfin) r->Tfin[(size_t)j * P + p] = T;
        if (r->ncomp) r->ncomp[(size_t)j * P + p] = n;
        if (r->margin) r->margin[(size_t)j * P + p] = m;
        if (r->rowhash) { h ^= (uint64_t)n + 0x9e3779b97f4a7c15ULL; h *= 1099511628211ULL; }
    }
    if (r->rowhash) r->rowhash[item] = h;
}

/*
 * Forward render.  Arrays are row-major doubles (FP32-valued inputs widened).
 * means K x 3, log_scales K x 3, quats K x 4 (w,x,y,z), logits K;
 * radiance K x 2 (direct) or NULL with features K x 32 and mlp (8706 values:
 * W1 64x68, b1, W2 64x64, b2, W3 2x64, b3);  centres V x 3 view points;
 * rx N x 3 receiver positions (MLP input); rx_view N view index per receiver.
 * Outputs: C N x 2 x H x W; optional T_final / ncomp / margin N x H x W;
 * power N; csum N x 2; rowhash N x H decision fingerprints (optional);
 * nclamp N x H x W composited entries whose weight was clamped (optional).
 * Returns 0 on success.
 */
static int render_impl(int K, const double *means, const double *log_scales, const double *quats,
                       const double *logits, const double *radiance, const double *features,
                       const double *mlp, const double *rad_rx, int V, const double *centres, int N,
                       const double *rx, const int *rx_view, int H, int W, double el0, double del,
                       int nthreads, double *C, double *T_final, int *ncomp, double *margin, double *power,
                       double *csum, uint64_t *rowhash, int *nclamp)
{
    if (K < 0 || V < 1 || N < 0 || H < 1 || W < 1) return -1;
    if (!radiance && !rad_rx && (!features || !mlp)) return -1;
    for (int j = 0; j < N; j++) if (rx_view[j] < 0 || rx_view[j] >= V) return -1;
    scene_t s;
    memset(&s, 0, sizeof s);
    s.K = K; s.V = V; s.N = N;
    s.means = means; s.ls = log_scales; s.quats = quats; s.logits = logits;
    s.radiance = radiance; s.features = features; s.mlp = mlp; s.centres = centres;
    s.rad_rx = rad_rx;
    s.rx = rx; s.rx_view = rx_view; s.g = mkgrid(H, W, el0, del);
    if (scene_setup(&s, nthreads)) return -2;
    render_ctx r = { &s, C, T_final, margin, ncomp, rowhash, nclamp };
    pool_run(nthreads, (long)N * H, render_item, &r);
    size_t P = (size_t)H * W;
    for (int j = 0; j < N; j++) {
        double pw = 0.0, sr = 0.0, si = 0.0;
        for (size_t p = 0; p < P; p++) {
            double re = C[((size_t)j * 2) * P + p], im = C[((size_t)j * 2 + 1) * P + p];
            pw += re * re + im * im; sr += re; si += im;
        }
        if (power) power[j] = pw;
        if (csum) { csum[2 * j] = sr; csum[2 * j + 1] = si; }
    }
    scene_free(&s);
    return 0;
}

int orc_render(int K, const double *means, const double *log_scales, const double *quats,
               const double *logits, const double *radiance, const double *features,
               const double *mlp, int V, const double *centres, int N, const double *rx,
               const int *rx_view, int H, int W, double el0, double del, int nthreads,
               double *C, double *T_final, int *ncomp, double *margin, double *power,
               double *csum, uint64_t *rowhash, int *nclamp)
{
    return render_impl(K, means, log_scales, quats, logits, radiance, features, mlp, NULL, V, centres, N, rx,
                       rx_view, H, W, el0, del, nthreads, C, T_final, ncomp, margin, power, csum, rowhash,
                       nclamp);
}

/*
 * The forward render with per-receiver radiance given (rad_rx N x K x 2, row
 * j for receiver j), e.g. from orc_rxcond_radiance with one row per
 * (receiver, channel).  Other arguments and outputs as orc_render.
 */
int orc_render_rad(int K, const double *means, const double *log_scales, const double *quats,
                   const double *logits, const double *rad_rx, int V, const double *centres, int N,
                   const int *rx_view, int H, int W, double el0, double del, int nthreads, double *C,
                   double *T_final, int *ncomp, double *margin, double *power, double *csum, uint64_t *rowhash,
                   int *nclamp)
{
    if (!rad_rx) return -1;
    return render_impl(K, means, log_scales, quats, logits, NULL, NULL, NULL, rad_rx, V, centres, N, NULL,
                       rx_view, H, W, el0, del, nthreads, C, T_final, ncomp, margin, power, csum, rowhash,
                       nclamp);
}

/*
 * Projection only: per (view v, Gaussian k), row-major V x K.
 * keybits: FP32 depth-key bits; nearcull: 1 if the FP32 key < 0.04;
 * proj: V x K x 9 doubles = u, v, conic a, b, c, opacity, cov A, B, Cc
 * (zeros for near-culled entries).
 */
int orc_project(int K, const double *means, const double *log_scales, const double *quats,
                const double *logits, int V, const double *centres, int H, int W, double el0,
                double del, uint32_t *keybits, int *nearcull, double *proj)
{
    orc_grid g = mkgrid(H, W, el0, del);
    for (int v = 0; v < V; v++)
        for (int k = 0; k < K; k++) {
            size_t i = (size_t)v * K + k;
            float kf = key_float(means + 3 * k, centres + 3 * v);
            keybits[i] = f2bits(kf);
            nearcull[i] = kf < ORC_NEAR2_F;
            dual out[NPROJ];
            if (nearcull[i]) { for (int t = 0; t < NPROJ; t++) proj[i * NPROJ + t] = 0.0; continue; }
            project_dual(means + 3 * k, log_scales + 3 * k, quats + 4 * k, logits[k], centres + 3 * v, &g, out);
            for (int t = 0; t < NPROJ; t++) proj[i * NPROJ + t] = out[t].v;
        }
    return 0;
}

/* Jacobian of the projected quantities (u, v, a, b, c, o) with respect to the
 * 11 raw parameters, for one (view, Gaussian): jac 6 x 11 row-major. */
int orc_project_jacobian(const double *p, const double *ls, const double *q, double logit,
                         const double *centre, int H, int W, double el0, double del, double *jac)
{
    orc_grid g = mkgrid(H, W, el0, del);
    dual out[NPROJ];
    project_dual(p, ls, q, logit, centre, &g, out);
    for (int r = 0; r < 6; r++)
        for (int i = 0; i < NP; i++) jac[r * NP + i] = out[r].d[i];
    return 0;
}

/* Radiance of every (receiver, Gaussian) pair: rad N x K x 2. */
int orc_radiance(int K, const double *radiance, const double *features, const double *mlp,
                 int N, const double *rx, int nthreads, double *rad)
{
    scene_t s;
    memset(&s, 0, sizeof s);
    s.K = K; s.N = N; s.radiance = radiance; s.features = features; s.mlp = mlp; s.rx = rx;
    s.rad = rad;
    pool_run(nthreads, N, rad_item, &s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* reverse mode */
typedef struct {
    scene_t *s;
    const double *dC, *dP;
    double *g2d;     /* per thread: V x K x 6 (u, v, a, b, c, o) */
    double *dS;      /* per thread: N x K x 2 */
    int nthreads;
    entry_t **ents;  /* per thread scratch */
} bwd_ctx;

static void bwd_item(void *vctx, long item, int tid)
{
    bwd_ctx *b = vctx;
    const scene_t *s = b->s;
    int H = s->g.H, W = s->g.W, K = s->K;
    int j = (int)(item / H), row = (int)(item % H);
    int v = s->rx_view[j];
    size_t P = (size_t)H * W;
    double *g2d = b->g2d + (size_t)tid * s->V * K * 6 + (size_t)v * K * 6;
    double *dS = b->dS + (size_t)tid * s->N * K * 2 + (size_t)j * K * 2;
    const double *rad = s->rad + (size_t)j * K * 2;
    const view_t *vw = &s->views[v];
    entry_t *ent = b->ents[tid];
    for (int col = 0; col < W; col++) {
        size_t p = (size_t)row * W + col;
        double C[2], T;
        int n = composite_pixel(s, j, row, col, C, &T, NULL, ent, NULL, NULL);
        double gp0 = b->dC[((size_t)j * 2) * P + p], gp1 = b->dC[((size_t)j * 2 + 1) * P + p];
        if (b->dP) { gp0 += 2.0 * b->dP[j] * C[0]; gp1 += 2.0 * b->dP[j] * C[1]; }
        double A0 = 0.0, A1 = 0.0;   /* sum over later entries of T_m w_m s_m */
        for (int e = n - 1; e >= 0; e--) {
            int k = ent[e].k;
            double Te = ent[e].T, we = ent[e].w;
            double s0 = rad[2 * k], s1 = rad[2 * k + 1];
            dS[2 * k + 0] += Te * we * gp0;
            dS[2 * k + 1] += Te * we * gp1;
            double dw = gp0 * (Te * s0 - A0 / (1.0 - we)) + gp1 * (Te * s1 - A1 / (1.0 - we));
            A0 += Te * we * s0;
            A1 += Te * we * s1;
            if (ent[e].clamped) continue;
            const double *pv = vw->pv + (size_t)k * NPROJ;
            double du = ent[e].du, dv = ent[e].dv;
            double *gk = g2d + (size_t)k * 6;
            gk[5] += dw * ent[e].G;                 /* d opacity */
            double dq = -0.5 * we * dw;
            gk[2] += dq * du * du;                  /* d conic a */
            gk[3] += dq * 2.0 * du * dv;            /* d conic b */
            gk[4] += dq * dv * dv;                  /* d conic c */
            gk[0] += -dq * (2.0 * pv[PA] * du + 2.0 * pv[PB] * dv);   /* d u */
            gk[1] += -dq * (2.0 * pv[PB] * du + 2.0 * pv[PC] * dv);   /* d v */
        }
    }
}

/*
 * Gradient of a loss L(C, P) given dL/dC (N x 2 x H x W) and optionally dL/dP (N).
 * Outputs (overwritten): d_means K x 3, d_log_scales K x 3, d_quats K x 4,
 * d_logits K, and d_radiance K x 2 (direct radiance) or d_features K x 32 and
 * d_mlp 8706 (MLP radiance).  Unused outputs may be NULL.
 */
int orc_backward(int K, const double *means, const double *log_scales, const double *quats,
                 const double *logits, const double *radiance, const double *features,
                 const double *mlp, int V, const double *centres, int N, const double *rx,
                 const int *rx_view, int H, int W, double el0, double del, int nthreads,
                 const double *dC, const double *dP, double *d_means, double *d_log_scales,
                 double *d_quats, double *d_logits, double *d_radiance, double *d_features,
                 double *d_mlp)
{
    if (K < 0 || V < 1 || N < 0 || H < 1 || W < 1) return -1;
    if (!radiance && (!features || !mlp)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    scene_t s;
    memset(&s, 0, sizeof s);
    s.K = K; s.V = V; s.N = N;
    s.means = means; s.ls = log_scales; s.quats = quats; s.logits = logits;
    s.radiance = radiance; s.features = features; s.mlp = mlp; s.centres = centres;
    s.rx = rx; s.rx_view = rx_view; s.g = mkgrid(H, W, el0, del);
    if (scene_setup(&s, nthreads)) return -2;

    bwd_ctx b;
    b.s = &s; b.dC = dC; b.dP = dP; b.nthreads = nthreads;
    b.g2d = calloc((size_t)nthreads * V * (size_t)(K > 0 ? K : 1) * 6, sizeof(double));
    b.dS = calloc((size_t)nthreads * (size_t)(N > 0 ? N : 1) * (size_t)(K > 0 ? K : 1) * 2, sizeof(double));
    b.ents = malloc(sizeof(entry_t *) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) b.ents[t] = malloc(sizeof(entry_t) * (size_t)(K > 0 ? K : 1));
    if (!b.g2d || !b.dS) return -2;
    pool_run(nthreads, (long)N * H, bwd_item, &b);
    for (int t = 1; t < nthreads; t++)
        for (size_t i = 0; i < (size_t)N * K * 2; i++) b.dS[i] += b.dS[(size_t)t * N * K * 2 + i];

    if (d_means) memset(d_means, 0, sizeof(double) * 3 * (size_t)K);
    if (d_log_scales) memset(d_log_scales, 0, sizeof(double) * 3 * (size_t)K);
    if (d_quats) memset(d_quats, 0, sizeof(double) * 4 * (size_t)K);
    if (d_logits) memset(d_logits, 0, sizeof(double) * (size_t)K);
    orc_grid g = s.g;
    for (int v = 0; v < V; v++)
        for (int k = 0; k < K; k++) {
            double g6[6] = { 0, 0, 0, 0, 0, 0 };
            for (int t = 0; t < nthreads; t++)
                for (int i = 0; i < 6; i++) g6[i] += b.g2d[(size_t)t * V * K * 6 + ((size_t)v * K + k) * 6 + i];
            if (g6[0] == 0 && g6[1] == 0 && g6[2] == 0 && g6[3] == 0 && g6[4] == 0 && g6[5] == 0) continue;
            dual out[NPROJ];
            project_dual(means + 3 * k, log_scales + 3 * k, quats + 4 * k, logits[k], centres + 3 * v, &g, out);
            double gp[NP];
            for (int i = 0; i < NP; i++) {
                gp[i] = 0.0;
                for (int r = 0; r < 6; r++) gp[i] += g6[r] * out[r].d[i];
            }
            if (d_means) for (int i = 0; i < 3; i++) d_means[3 * k + i] += gp[i];
            if (d_log_scales) for (int i = 0; i < 3; i++) d_log_scales[3 * k + i] += gp[3 + i];
            if (d_quats) for (int i = 0; i < 4; i++) d_quats[4 * k + i] += gp[6 + i];
            if (d_logits) d_logits[k] += gp[10];
        }

    if (radiance) {
        if (d_radiance) {
            memset(d_radiance, 0, sizeof(double) * 2 * (size_t)K);
            for (int j = 0; j < N; j++)
                for (int k = 0; k < K; k++) {
                    d_radiance[2 * k] += b.dS[((size_t)j * K + k) * 2];
                    d_radiance[2 * k + 1] += b.dS[((size_t)j * K + k) * 2 + 1];
                }
        }
    } else {
        mlp_t m = mlp_view(mlp);
        double *dm = calloc(ORC_NMLP, sizeof(double));
        double *dW1 = dm, *db1 = dW1 + ORC_HID * ORC_IN, *dW2 = db1 + ORC_HID;
        double *db2 = dW2 + ORC_HID * ORC_HID, *dW3 = db2 + ORC_HID, *db3 = dW3 + 2 * ORC_HID;
        if (d_features) memset(d_features, 0, sizeof(double) * ORC_FEAT * (size_t)K);
        for (int j = 0; j < N; j++) {
            double x[ORC_IN], r[3] = { rx[3 * j], rx[3 * j + 1], rx[3 * j + 2] };
            encode_rx(r, x);
            for (int k = 0; k < K; k++) {
                double ds0 = b.dS[((size_t)j * K + k) * 2], ds1 = b.dS[((size_t)j * K + k) * 2 + 1];
                if (ds0 == 0.0 && ds1 == 0.0) continue;
                for (int i = 0; i < ORC_FEAT; i++) x[ORC_ENC + i] = features[(size_t)k * ORC_FEAT + i];
                double sv[2], z1[ORC_HID], z2[ORC_HID], h1[ORC_HID], h2[ORC_HID];
                mlp_forward(&m, x, sv, z1, z2);
                for (int i = 0; i < ORC_HID; i++) { h1[i] = z1[i] > 0 ? z1[i] : 0; h2[i] = z2[i] > 0 ? z2[i] : 0; }
                double ds[2] = { ds0, ds1 }, dz2[ORC_HID], dz1[ORC_HID];
                for (int o = 0; o < 2; o++) {
                    db3[o] += ds[o];
                    for (int i = 0; i < ORC_HID; i++) dW3[o * ORC_HID + i] += ds[o] * h2[i];
                }
                for (int i = 0; i < ORC_HID; i++) {
                    double acc = m.W3[i] * ds[0] + m.W3[ORC_HID + i] * ds[1];
                    dz2[i] = z2[i] > 0 ? acc : 0.0;
                }
                for (int o = 0; o < ORC_HID; o++) {
                    db2[o] += dz2[o];
                    for (int i = 0; i < ORC_HID; i++) dW2[o * ORC_HID + i] += dz2[o] * h1[i];
                }
                for (int i = 0; i < ORC_HID; i++) {
                    double acc = 0.0;
                    for (int o = 0; o < ORC_HID; o++) acc += m.W2[o * ORC_HID + i] * dz2[o];
                    dz1[i] = z1[i] > 0 ? acc : 0.0;
                }
                for (int o = 0; o < ORC_HID; o++) {
                    db1[o] += dz1[o];
                    for (int i = 0; i < ORC_IN; i++) dW1[o * ORC_IN + i] += dz1[o] * x[i];
                }
                if (d_features)
                    for (int i = 0; i < ORC_FEAT; i++) {
                        double acc = 0.0;
                        for (int o = 0; o < ORC_HID; o++) acc += m.W1[o * ORC_IN + ORC_ENC + i] * dz1[o];
                        d_features[(size_t)k * ORC_FEAT + i] += acc;
                    }
            }
        }
        if (d_mlp) memcpy(d_mlp, dm, sizeof(double) * ORC_NMLP);
        free(dm);
    }
    for (int t = 0; t < nthreads; t++) free(b.ents[t]);
    free(b.ents); free(b.g2d); free(b.dS);
    scene_free(&s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* integer tile binning of FP32 projection records */
typedef struct { int64_t seg; uint32_t key; int32_t k; } pair_t;
static int cmp_pair(const void *a, const void *b)
{
    const pair_t *x = a, *y = b;
    if (x->seg != y->seg) return x->seg < y->seg ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->k > y->k) - (x->k < y->k);
}

/* tile columns covered by one record; returns the count and fills tx[] */
static int bin_cols(float u, float rup, int W, int TW, int *tx)
{
    int nTx = (W + TW - 1) / TW;
    int n = 0;
    if (rup >= 0.5f * (float)(W - TW - 2)) {
        for (int t = 0; t < nTx; t++) tx[n++] = t;
        return n;
    }
    int c0 = (int)ceilf(u - rup);
    int c1 = (int)floorf(u + rup);
    if (c0 > c1) return 0;
    int m = ((c0 % W) + W) % W;
    int e = m + (c1 - c0);
    if (e < W) {
        for (int t = m / TW; t <= e / TW; t++) tx[n++] = t;
    } else {
        for (int t = m / TW; t <= (W - 1) / TW; t++) tx[n++] = t;
        for (int t = 0; t <= (e - W) / TW; t++) tx[n++] = t;
    }
    return n;
}

/*
 * Expected (segment, Gaussian) pairs in final sorted order from FP32 records
 * (V x K each: u, v, padded half-extents rup / rvp, opacity o, depth-key bits).
 * A record takes part when key >= bits(0.04f) and o >= 1/255 (FP32); rows
 * [ceil(max(v - rvp, 0)), floor(min(v + rvp, H - 1))]; columns
 * [ceil(u - rup), floor(u + rup)] taken modulo W, or every tile column once
 * rup >= (W - TW - 2) / 2.  seg = v * tiles + ty * tiles_x + tx.  Sorted by
 * (seg, key, index).  Writes at most cap pairs; returns the total count.
 */
int64_t orc_bin(int V, int K, const float *u, const float *v, const float *rup, const float *rvp,
                const float *o, const uint32_t *keybits, int H, int W, int TW, int TH,
                int64_t *seg_out, int32_t *k_out, int64_t cap)
{
    int nTx = (W + TW - 1) / TW, nTy = (H + TH - 1) / TH;
    int64_t T = (int64_t)nTx * nTy;
    const float alpha = 1.0f / 255.0f;
    const float near2 = ORC_NEAR2_F;
    uint32_t nearbits; memcpy(&nearbits, &near2, 4);
    int64_t total = 0, alloc = 1024;
    pair_t *pairs = malloc(sizeof(pair_t) * (size_t)alloc);
    int *tx = malloc(sizeof(int) * (size_t)(nTx + 2));
    for (int vv = 0; vv < V; vv++)
        for (int k = 0; k < K; k++) {
            size_t i = (size_t)vv * K + k;
            if (keybits[i] < nearbits) continue;
            if (!(o[i] >= alpha)) continue;
            float lo = fmaxf(v[i] - rvp[i], 0.0f);
            float hi = fminf(v[i] + rvp[i], (float)(H - 1));
            int i0 = (int)ceilf(lo), i1 = (int)floorf(hi);
            if (i0 > i1) continue;
            int ncol = bin_cols(u[i], rup[i], W, TW, tx);
            for (int ty = i0 / TH; ty <= i1 / TH; ty++)
                for (int c = 0; c < ncol; c++) {
                    if (total == alloc) { alloc *= 2; pairs = realloc(pairs, sizeof(pair_t) * (size_t)alloc); }
                    pairs[total].seg = (int64_t)vv * T + (int64_t)ty * nTx + tx[c];
                    pairs[total].key = keybits[i];
                    pairs[total].k = k;
                    total++;
                }
        }
    qsort(pairs, (size_t)total, sizeof(pair_t), cmp_pair);
    for (int64_t t = 0; t < total && t < cap; t++) {
        if (seg_out) seg_out[t] = pairs[t].seg;
        if (k_out) k_out[t] = pairs[t].k;
    }
    free(pairs); free(tx);
    return total;
}
