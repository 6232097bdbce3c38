/*
 * swe_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, double-precision reference for the explicit finite-volume
 * step of the 2D shallow-water equations (Delmas & Soulaimani, "Parallel
 * high-order resolution of the Shallow-water equations on real large-scale
 * meshes with complex bathymetries", Sec. 6), and for the ghost-layer
 * machinery of one sub-domain (Sec. 3.2 - 3.3).
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code with the HIP library.
 * Every function cites the passage it follows; where the paper is silent or
 * its printed formula is garbled the reading used is stated in a comment.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 *
 * Pinned by tests/test_oracle_*.py (lake at rest, Stoker / Ritter dam
 * breaks, mass balance, mirror symmetry, special-case reductions of the
 * Riemann solvers and limiters, brute-force ghost lists, finite-difference
 * gradients of the limiter network).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- enums mirrored by oracle/oracle.py ------------------------------- */
enum { OR_HLLC1 = 0, OR_MUSCL = 1, OR_WAF = 2 };
enum { OR_EULER = 0, OR_RK2 = 1 };
enum { OR_MINMOD = 0, OR_SUPERBEE = 1, OR_VANALBADA = 2, OR_LEARNED = 3,
       OR_ZEROSLOPE = 4 };
enum { OR_WAF_SUPERBEE = 0, OR_WAF_GODUNOV = 1, OR_WAF_UNLIMITED = 2 };
enum { BC_WALL = -1, BC_TRANSMISSIVE = -2, BC_INFLOW = -3, BC_OUTFLOW = -4,
       BC_HALO = -5 };
enum { FL_NONFINITE = 1, FL_NEGDEPTH = 2, FL_CLIPPED = 4 };

#define MLP_IN 14
#define MLP_H 32
#define MLP_NPAR (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

typedef struct {
    double g, cfl, eps, dt_max;
    int scheme, integrator, limiter, waf_limiter, cfl_rule, mlp_bf16;
    double inflow_q, inflow_len, outflow_stage;
    int n_series, pad;
    const double *series_t, *series_q;
    const double *mlp; /* MLP_NPAR weights, layout of mlp_unpack() */
    int waf_pos;       /* WAF: 1 = mass flux kept within each donor cell's share (below) */
    int phi_every;     /* learned limiter: phi evaluated on steps 0, k, 2k, ... of a run
                          (the steps between keep the last phi); 0 or 1: every step */
} or_params;

typedef struct {
    int nn, nc, n_owned;
    double *xy;
    int *tri, *nbr, *nbr_edge;
    int64_t *gid;
    double *b, *man;
    double *area, *cx, *cy, *inr;      /* per cell */
    double *enx, *eny, *elen, *emx, *emy; /* per half-edge 3c+m */
    /* work arrays */
    double *rh, *rb, *run, *rut;  /* interface values per half-edge (own normal frame) */
    double *fx0, *fx1, *fx2;      /* half-edge flux incl. HR correction (global frame) */
    double *u0h, *u0u, *u0v, *u1h, *u1u, *u1v;
    double *phi;                  /* learned limiter: phi of every half-edge for this step */
} or_mesh;

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------
 * Geometry (Sec. 6.1, eq. vlap2 and the CFL paragraph): area |Omega_i|,
 * edge lengths L_ij, unit outward normals n_ij, inscribed radius R_i.
 * Local edge m joins nodes m and m+1 (mod 3); triangles are counter-
 * clockwise, so the outward normal of the edge vector (dx, dy) is
 * (dy, -dx)/L.  R = 2|Omega|/perimeter.
 * ---------------------------------------------------------------------- */
static int geometry(or_mesh *M)
{
    for (int c = 0; c < M->nc; ++c) {
        const int *t = M->tri + 3 * c;
        double x[3], y[3];
        for (int k = 0; k < 3; ++k) { x[k] = M->xy[2 * t[k]]; y[k] = M->xy[2 * t[k] + 1]; }
        double a2 = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
        if (!(a2 > 0.0)) return -1;
        M->area[c] = 0.5 * a2;
        M->cx[c] = ((x[0] + x[1]) + x[2]) / 3.0;
        M->cy[c] = ((y[0] + y[1]) + y[2]) / 3.0;
        double per = 0.0;
        for (int m = 0; m < 3; ++m) {
            int p = m, q = (m + 1) % 3;
            double dx = x[q] - x[p], dy = y[q] - y[p];
            double L = sqrt(dx * dx + dy * dy);
            M->elen[3 * c + m] = L;
            M->enx[3 * c + m] = dy / L;
            M->eny[3 * c + m] = -dx / L;
            M->emx[3 * c + m] = 0.5 * (x[p] + x[q]);
            M->emy[3 * c + m] = 0.5 * (y[p] + y[q]);
            per += L;
        }
        M->inr[c] = 2.0 * M->area[c] / per;
    }
    return 0;
}

/* Local edge of cell k that faces cell c (same two nodes). */
static int facing_edge(const or_mesh *M, int k, int c)
{
    for (int m = 0; m < 3; ++m)
        if (M->nbr[3 * k + m] == c) return m;
    return -1;
}

void or_mesh_free(or_mesh *M)
{
    if (!M) return;
    void **p[] = {(void **)&M->xy, (void **)&M->tri, (void **)&M->nbr, (void **)&M->nbr_edge,
                  (void **)&M->gid, (void **)&M->b, (void **)&M->man, (void **)&M->area,
                  (void **)&M->cx, (void **)&M->cy, (void **)&M->inr, (void **)&M->enx,
                  (void **)&M->eny, (void **)&M->elen, (void **)&M->emx, (void **)&M->emy,
                  (void **)&M->rh, (void **)&M->rb, (void **)&M->run, (void **)&M->rut,
                  (void **)&M->fx0, (void **)&M->fx1, (void **)&M->fx2, (void **)&M->u0h,
                  (void **)&M->u0u, (void **)&M->u0v, (void **)&M->u1h, (void **)&M->u1u,
                  (void **)&M->u1v, (void **)&M->phi};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); ++i) free(*p[i]);
    free(M);
}

/* nbr: [3*nc] local neighbour index (>=0) or a negative boundary tag. */
or_mesh *or_mesh_new(int nn, const double *xy, int nc, int n_owned, const int *tri,
                     const int64_t *gid, const int *nbr, const double *b, const double *man)
{
    or_mesh *M = (or_mesh *)calloc(1, sizeof(or_mesh));
    M->nn = nn; M->nc = nc; M->n_owned = n_owned;
    size_t n3 = 3 * (size_t)nc;
    M->xy = malloc(sizeof(double) * 2 * nn); memcpy(M->xy, xy, sizeof(double) * 2 * nn);
    M->tri = malloc(sizeof(int) * n3); memcpy(M->tri, tri, sizeof(int) * n3);
    M->nbr = malloc(sizeof(int) * n3); memcpy(M->nbr, nbr, sizeof(int) * n3);
    M->gid = malloc(sizeof(int64_t) * nc); memcpy(M->gid, gid, sizeof(int64_t) * nc);
    M->b = malloc(sizeof(double) * nc); memcpy(M->b, b, sizeof(double) * nc);
    M->man = malloc(sizeof(double) * nc); memcpy(M->man, man, sizeof(double) * nc);
    M->nbr_edge = malloc(sizeof(int) * n3);
    double **pc[] = {&M->area, &M->cx, &M->cy, &M->inr, &M->u0h, &M->u0u, &M->u0v,
                     &M->u1h, &M->u1u, &M->u1v};
    for (size_t i = 0; i < sizeof(pc) / sizeof(pc[0]); ++i) *pc[i] = malloc(sizeof(double) * nc);
    double **pe[] = {&M->enx, &M->eny, &M->elen, &M->emx, &M->emy, &M->rh, &M->rb, &M->run,
                     &M->rut, &M->fx0, &M->fx1, &M->fx2, &M->phi};
    for (size_t i = 0; i < sizeof(pe) / sizeof(pe[0]); ++i) *pe[i] = malloc(sizeof(double) * n3);
    if (geometry(M) != 0) { or_mesh_free(M); return NULL; }
    for (int c = 0; c < nc; ++c)
        for (int m = 0; m < 3; ++m) {
            int k = M->nbr[3 * c + m];
            M->nbr_edge[3 * c + m] = -1;
            if (k >= 0) {
                if (k >= nc) { or_mesh_free(M); return NULL; }
                int f = facing_edge(M, k, c);
                if (f < 0) { or_mesh_free(M); return NULL; }
                M->nbr_edge[3 * c + m] = f;
            }
        }
    return M;
}

int or_mesh_geometry(const or_mesh *M, double *area, double *cx, double *cy, double *inr,
                     double *enx, double *eny, double *elen)
{
    size_t n = M->nc, n3 = 3 * n;
    memcpy(area, M->area, n * sizeof(double)); memcpy(cx, M->cx, n * sizeof(double));
    memcpy(cy, M->cy, n * sizeof(double)); memcpy(inr, M->inr, n * sizeof(double));
    memcpy(enx, M->enx, n3 * sizeof(double)); memcpy(eny, M->eny, n3 * sizeof(double));
    memcpy(elen, M->elen, n3 * sizeof(double));
    return 0;
}

/* ------------------------------------------------------------------------
 * HLL / HLLC flux in the edge-normal frame (Sec. 6.2.1, eq. hll and the
 * wave-speed estimates that follow it).  U = (h, q_n, q_t).
 * Readings: p_k is Toro's sqrt((h*+h_k) h* / (2 h_k^2)) (the printed form is
 * dimensionally inconsistent); S* uses the capital S_L, S_R; the third
 * component is upwinded with v_L when S* >= 0 and v_R otherwise (the printed
 * branch is inverted with respect to the S_L >= 0 limit and to the WAF
 * weights); dry states use Toro's dry-bed speeds.
 * ---------------------------------------------------------------------- */
typedef struct {
    double hL, hR, uL, uR, vL, vR, qL, qR; /* q = normal discharge */
    double GL[3], GR[3], Fs[2];            /* physical fluxes, HLL star flux (1,2) */
    double SL, SR, Ss;
    int dry;                               /* both sides dry: zero flux */
} wave_fan;

static void wave_speeds(double g, double eps, const double UL[3], const double UR[3], wave_fan *W)
{
    W->hL = UL[0]; W->hR = UR[0];
    W->dry = (W->hL <= eps && W->hR <= eps);
    W->uL = W->hL > eps ? UL[1] / W->hL : 0.0;
    W->vL = W->hL > eps ? UL[2] / W->hL : 0.0;
    W->uR = W->hR > eps ? UR[1] / W->hR : 0.0;
    W->vR = W->hR > eps ? UR[2] / W->hR : 0.0;
    W->qL = W->hL > eps ? UL[1] : 0.0;
    W->qR = W->hR > eps ? UR[1] : 0.0;
    if (W->dry) return;
    double hL = W->hL, hR = W->hR, uL = W->uL, uR = W->uR;
    double aL = sqrt(g * hL), aR = sqrt(g * hR);
    if (hR <= eps) {            /* dry bed on the right */
        W->SL = uL - aL; W->SR = uL + 2.0 * aL; W->Ss = W->SR;
    } else if (hL <= eps) {     /* dry bed on the left */
        W->SL = uR - 2.0 * aR; W->SR = uR + aR; W->Ss = W->SL;
    } else {
        double h0 = 0.5 * (hL + hR) - 0.25 * (uR - uL) * (hL + hR) / (aR + aL);
        double hs;
        if (h0 <= dmin(hL, hR)) {              /* two-rarefaction estimate */
            double t = 0.5 * (aR + aL) + 0.25 * (uL - uR);
            hs = t > 0.0 ? t * t / g : 0.0;
        } else {                               /* two-shock estimate */
            double gL = sqrt(g * (h0 + hL) / (2.0 * h0 * hL));
            double gR = sqrt(g * (h0 + hR) / (2.0 * h0 * hR));
            hs = (hL * gL + hR * gR + uL - uR) / (gL + gR);
        }
        double pL = hs > hL ? sqrt((hs + hL) * hs / (2.0 * hL * hL)) : 1.0;
        double pR = hs > hR ? sqrt((hs + hR) * hs / (2.0 * hR * hR)) : 1.0;
        W->SL = uL - aL * pL;
        W->SR = uR + aR * pR;
        W->Ss = (W->SL * hR * (uR - W->SR) - W->SR * hL * (uL - W->SL)) /
                (hR * (uR - W->SR) - hL * (uL - W->SL));
    }
    /* physical fluxes G(U) of eq. eqswefinal in the normal frame */
    W->GL[0] = W->qL; W->GL[1] = W->qL * uL + 0.5 * g * hL * hL; W->GL[2] = W->qL * W->vL;
    W->GR[0] = W->qR; W->GR[1] = W->qR * uR + 0.5 * g * hR * hR; W->GR[2] = W->qR * W->vR;
    /* star-region flux of the HLL scheme */
    double d = W->SR - W->SL;
    W->Fs[0] = (W->SR * W->GL[0] - W->SL * W->GR[0] + W->SR * W->SL * (hR - hL)) / d;
    W->Fs[1] = (W->SR * W->GL[1] - W->SL * W->GR[1] + W->SR * W->SL * (W->qR - W->qL)) / d;
}

static void flux_hllc(double g, double eps, const double UL[3], const double UR[3], double F[3])
{
    wave_fan W;
    wave_speeds(g, eps, UL, UR, &W);
    if (W.dry) { F[0] = F[1] = F[2] = 0.0; return; }
    if (W.SL >= 0.0) { F[0] = W.GL[0]; F[1] = W.GL[1]; F[2] = W.GL[2]; return; }
    if (W.SR <= 0.0) { F[0] = W.GR[0]; F[1] = W.GR[1]; F[2] = W.GR[2]; return; }
    F[0] = W.Fs[0];
    F[1] = W.Fs[1];
    F[2] = F[0] * (W.Ss >= 0.0 ? W.vL : W.vR);
}

/* ------------------------------------------------------------------------
 * WAF flux (Sec. 6.2.2, TVD weights and eq. eq:superbee).
 * Reading: Toro's TVD form  w_L = (1 + sgn(c_L) A_L)/2,
 * w_LR = (sgn(c_R) A_R - sgn(c_L) A_L)/2, w_R = (1 - sgn(c_R) A_R)/2,
 * w_L* / w_R* = (1 +/- sgn(c*) A*)/2, A_k = A(r_k, c_k); with A = |c| these
 * are the unlimited weights, with A = 1 the scheme is HLLC.  c = S dt/dx with
 * dx the distance between the two cell centroids.  r_k = upwind change over
 * local change; zero local change, or a missing upwind cell, gives r = 0.
 * q = eta = h + b for the L and R waves (h on a flat bed), q = v (tangential
 * velocity) for the * wave; upwind values are means over the two upwind
 * cells.
 * ---------------------------------------------------------------------- */
static double superbee_A(double r, double c)
{
    double ac = fabs(c);
    if (r <= 0.0) return 1.0;
    if (r <= 0.5) return 1.0 - 2.0 * (1.0 - ac) * r;
    if (r <= 1.0) return ac;
    if (r <= 2.0) return 1.0 - (1.0 - ac) * r;
    return 2.0 * ac - 1.0;
}

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

typedef struct {
    double qL, qR;            /* local values of the limited quantity */
    double qLu, qRu;          /* upwind values */
    int hasLu, hasRu;
} waf_ratio_in;

static double waf_ratio(double S, const waf_ratio_in *w)
{
    double dloc = w->qR - w->qL;
    if (dloc == 0.0) return 0.0;
    if (S >= 0.0) {
        if (!w->hasLu) return 0.0;
        return (w->qL - w->qLu) / dloc;
    }
    if (!w->hasRu) return 0.0;
    return (w->qRu - w->qR) / dloc;
}

static double waf_A(int mode, double r, double c)
{
    if (mode == OR_WAF_GODUNOV) return 1.0;
    if (mode == OR_WAF_UNLIMITED) return fabs(c);
    return superbee_A(r, c);
}

static void flux_waf(double g, double eps, int mode, double dt_dx, const double UL[3],
                     const double UR[3], const waf_ratio_in *rh, const waf_ratio_in *rv,
                     double F[3])
{
    wave_fan W;
    wave_speeds(g, eps, UL, UR, &W);
    if (W.dry) { F[0] = F[1] = F[2] = 0.0; return; }
    double cL = W.SL * dt_dx, cR = W.SR * dt_dx, cs = W.Ss * dt_dx;
    double AL = waf_A(mode, waf_ratio(W.SL, rh), cL);
    double AR = waf_A(mode, waf_ratio(W.SR, rh), cR);
    double As = waf_A(mode, waf_ratio(W.Ss, rv), cs);
    double wL = 0.5 * (1.0 + sgn(cL) * AL);
    double wLR = 0.5 * (sgn(cR) * AR - sgn(cL) * AL);
    double wR = 0.5 * (1.0 - sgn(cR) * AR);
    for (int i = 0; i < 2; ++i) F[i] = wL * W.GL[i] + wLR * W.Fs[i] + wR * W.GR[i];
    double wLs = 0.5 * (1.0 + sgn(cs) * As), wRs = 0.5 * (1.0 - sgn(cs) * As);
    F[2] = (wLs * W.vL + wRs * W.vR) * F[0];
}

/* Positivity of WAF's depths (reading 10).  Over one step an edge may take
 * from the cell it drains at most the share L / P of that cell's water (L
 * the edge length, P the perimeter): a mass flux of at most
 * h |Omega| / (P dt) = h R / (2 dt), R = 2 |Omega| / P the inscribed radius.
 * Summed over its three edges no cell then loses more water than it holds;
 * the bound is taken at 99% of that share so that rounding cannot take the
 * last drop.  Where WAF's mass flux leaves these bounds (L's for a flux
 * from L to R, R's for the reverse) the flux is blended towards the
 * first-order HLLC flux of the same states, F = F_hllc + theta (F_waf -
 * F_hllc), with the largest theta in [0, 1] that meets the bound, and the
 * mass flux is set to the bound itself (exact).  If HLLC's own mass flux
 * is beyond the bound the edge keeps whichever of the two is nearer. */
static void waf_positivity(double g, double eps, const double UL[3], const double UR[3],
                           double hL, double RL, double hR, double RR, double dt, double F[3])
{
    double hi = 0.99 * hL * RL / (2.0 * dt), lo = -(0.99 * hR * RR / (2.0 * dt));
    if (F[0] <= hi && F[0] >= lo) return;
    double bound = F[0] > hi ? hi : lo;
    double Fh[3];
    flux_hllc(g, eps, UL, UR, Fh);
    double theta = (bound - Fh[0]) / (F[0] - Fh[0]);
    if (!(theta > 0.0)) {                      /* HLLC is beyond the bound too */
        for (int i = 0; i < 3; ++i) F[i] = Fh[i];
    } else if (theta < 1.0) {
        for (int i = 1; i < 3; ++i) F[i] = Fh[i] + theta * (F[i] - Fh[i]);
        F[0] = bound;
    }
}

/* ------------------------------------------------------------------------
 * Slope limiters of the MUSCL scheme (Sec. 6.2.3).  sb is the slope towards
 * the upwind side, sf the slope across the edge; the branch is taken on the
 * sign of the jump across the edge as printed; a zero jump gives zero.
 * beta = 1 is MINBEE (minmod), beta = 2 SUPERBEE.  Van Albada is the
 * classical smooth limiter sb*sf*(sb+sf)/(sb^2+sf^2) for sb*sf > 0.
 * ---------------------------------------------------------------------- */
static double limit_beta(double beta, double sb, double sf)
{
    if (sf > 0.0) return dmax(0.0, dmax(dmin(beta * sb, sf), dmin(sb, beta * sf)));
    if (sf < 0.0) return dmin(0.0, dmin(dmax(beta * sb, sf), dmax(sb, beta * sf)));
    return 0.0;
}

/* The learned slope kept inside the second-order TVD region of the
 * backward and forward slopes (Sweby's bound 0 <= slope / s <= 2 with
 * s the smaller of the two): zero unless both have the same sign, else the
 * sign of the forward slope and at most twice the smaller magnitude.  With
 * phi = 1 this is the monotonized central limiter on the central slope. */
static double tvd_clip(double s, double sb, double sf)
{
    if (!(sb * sf > 0.0)) return 0.0;
    double lim = 2.0 * fmin(fabs(sb), fabs(sf));
    return copysign(fmin(fabs(s), lim), sf);
}

static double limit_vanalbada(double sb, double sf)
{
    if (sb * sf > 0.0) return sb * sf * (sb + sf) / (sb * sb + sf * sf);
    return 0.0;
}

/* ---------------- learned limiter network, FP64 (MLP 14-32-32-1) -------- */
typedef struct { const double *W1, *b1, *W2, *b2, *W3, *b3; } mlp_view;

static mlp_view mlp_unpack(const double *p)
{
    mlp_view v;
    v.W1 = p; p += MLP_H * MLP_IN;
    v.b1 = p; p += MLP_H;
    v.W2 = p; p += MLP_H * MLP_H;
    v.b2 = p; p += MLP_H;
    v.W3 = p; p += MLP_H;
    v.b3 = p;
    return v;
}

/* Round to the nearest bfloat16 (ties to even), returned as a double. */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* Forward pass. ReLU hidden layers, sigmoid output.  When bf16 != 0 the
 * input of every layer is rounded to bfloat16 first (the operand precision of
 * the matrix-core kernels); arithmetic stays in double. */
static double mlp_forward(const mlp_view *v, const double x[MLP_IN], int bf16, double a1[MLP_H],
                          double a2[MLP_H], double *z3)
{
    double xin[MLP_IN];
    for (int i = 0; i < MLP_IN; ++i) xin[i] = bf16 ? to_bf16(x[i]) : x[i];
    for (int j = 0; j < MLP_H; ++j) {
        double s = v->b1[j];
        for (int i = 0; i < MLP_IN; ++i) s += v->W1[j * MLP_IN + i] * xin[i];
        a1[j] = s > 0.0 ? s : 0.0;
    }
    double a1r[MLP_H];
    for (int j = 0; j < MLP_H; ++j) a1r[j] = bf16 ? to_bf16(a1[j]) : a1[j];
    for (int j = 0; j < MLP_H; ++j) {
        double s = v->b2[j];
        for (int i = 0; i < MLP_H; ++i) s += v->W2[j * MLP_H + i] * a1r[i];
        a2[j] = s > 0.0 ? s : 0.0;
    }
    double s = v->b3[0];
    for (int i = 0; i < MLP_H; ++i) s += v->W3[i] * (bf16 ? to_bf16(a2[i]) : a2[i]);
    *z3 = s;
    return 1.0 / (1.0 + exp(-s));
}

/* Batched forward: phi[n] for features x[n][14]. */
int or_mlp_forward(const double *params, int n, const double *x, int bf16, double *phi)
{
    mlp_view v = mlp_unpack(params);
    double a1[MLP_H], a2[MLP_H], z;
    for (int i = 0; i < n; ++i) phi[i] = mlp_forward(&v, x + (size_t)MLP_IN * i, bf16, a1, a2, &z);
    return 0;
}

/* Loss of the limiter training: mean over n half-edges of
 *   sum_v wv[v] * (q_v + d * clip(phi * s_v, sb_v, sf_v) - t_v)^2,
 * v in {h, eta, u_n, u_t}, i.e. the squared misfit against the refined-mesh
 * target of the value the solver reconstructs with this phi (the central
 * slope s scaled by phi, kept in the TVD region of the backward and forward
 * slopes sb, sf by tvd_clip), at distance d from the centroid.  The clip
 * passes phi * s through where sb and sf agree in sign and |phi s| is below
 * the bound; elsewhere the value does not depend on phi.  Returns the loss
 * and accumulates dLoss/dparams. */
double or_mlp_loss_grad(const double *params, int n, const double *x, const double *q,
                        const double *s, const double *sb, const double *sf, const double *d,
                        const double *t, const double *wv, double *grad)
{
    mlp_view v = mlp_unpack(params);
    mlp_view gv = mlp_unpack(grad);
    double *gW1 = (double *)gv.W1, *gb1 = (double *)gv.b1, *gW2 = (double *)gv.W2;
    double *gb2 = (double *)gv.b2, *gW3 = (double *)gv.W3, *gb3 = (double *)gv.b3;
    memset(grad, 0, sizeof(double) * MLP_NPAR);
    double loss = 0.0;
    for (int e = 0; e < n; ++e) {
        const double *xe = x + (size_t)MLP_IN * e;
        double a1[MLP_H], a2[MLP_H], z;
        double phi = mlp_forward(&v, xe, 0, a1, a2, &z);
        double dphi = 0.0;
        for (int k = 0; k < 4; ++k) {
            double sk = s[4 * e + k], b = sb[4 * e + k], f = sf[4 * e + k];
            double r = q[4 * e + k] + d[e] * tvd_clip(phi * sk, b, f) - t[4 * e + k];
            loss += wv[k] * r * r;
            int passes = b * f > 0.0 && fabs(phi * sk) < 2.0 * fmin(fabs(b), fabs(f));
            if (passes) dphi += 2.0 * wv[k] * r * d[e] * copysign(fabs(sk), f);
        }
        double dz = dphi * phi * (1.0 - phi) / n;
        gb3[0] += dz;
        double da2[MLP_H];
        for (int i = 0; i < MLP_H; ++i) {
            gW3[i] += dz * a2[i];
            da2[i] = a2[i] > 0.0 ? dz * v.W3[i] : 0.0;
        }
        double da1[MLP_H];
        for (int i = 0; i < MLP_H; ++i) da1[i] = 0.0;
        for (int j = 0; j < MLP_H; ++j) {
            gb2[j] += da2[j];
            for (int i = 0; i < MLP_H; ++i) {
                gW2[j * MLP_H + i] += da2[j] * a1[i];
                da1[i] += da2[j] * v.W2[j * MLP_H + i];
            }
        }
        for (int j = 0; j < MLP_H; ++j) {
            double dj = a1[j] > 0.0 ? da1[j] : 0.0;
            gb1[j] += dj;
            for (int i = 0; i < MLP_IN; ++i) gW1[j * MLP_IN + i] += dj * xe[i];
        }
    }
    return loss / n;
}

/* ------------------------------------------------------------------------
 * Features of one half-edge for the learned limiter.  For each of h, q_n, q_t
 * (discharges in the edge frame) and b: tanh of the upwind and cross-edge
 * increments over the distance to the edge midpoint (slope times d_mid)
 * made dimensionless with the variable's scale (for q_t, whose sign flips
 * in a mirror image, their magnitudes), and the clipped ratio of the two
 * increments (regularized at 1% of the scale); then the cell Froude number
 * and the relative depth jump.
 * scale: h and b -> h_c + 0.01 m; q_n, q_t -> h_c * sqrt(g h_c) + 0.01 m^2/s.
 * ---------------------------------------------------------------------- */
static void halfedge_features(double g, const double qc[4], const double qu[4],
                              const double qf[4], double du, double df, double dm, double hc,
                              double uc, double vc, double hk, double f[MLP_IN])
{
    double sh = hc + 0.01, sq = hc * sqrt(g * dmax(hc, 0.0)) + 0.01;
    double sc[4] = {sh, sq, sq, sh};
    for (int k = 0; k < 4; ++k) {
        /* the upwind and cross-edge increments over the distance to the edge
         * midpoint: slope times d_mid */
        double ab = (qc[k] - qu[k]) / du * dm, af = (qf[k] - qc[k]) / df * dm;
        /* q_t changes sign in a mirror image: its two increments enter by
         * magnitude (their ratio keeps the relative sign), so that the
         * features of mirror-image half-edges are equal */
        f[3 * k + 0] = tanh((k == 2 ? fabs(ab) : ab) / sc[k]);
        f[3 * k + 1] = tanh((k == 2 ? fabs(af) : af) / sc[k]);
        /* the ratio of the two increments, regularized at 1% of the
         * variable's scale: smooth where the forward increment vanishes */
        double r = ab * af / (af * af + 1e-4 * sc[k] * sc[k]);
        f[3 * k + 2] = dmax(-2.0, dmin(2.0, r));
    }
    f[12] = tanh(sqrt(uc * uc + vc * vc) / sqrt(g * dmax(hc, 1e-6)));
    f[13] = tanh((hk - hc) / (hc + 0.01));
}

/* ------------------------------------------------------------------------
 * Interface values of one side of an edge (Sec. 6.2.3, MUSCL).  The states
 * of the Riemann problem are the rotated cell states U_L = T_n U_i (Sec. 6.1,
 * eq. vlap2), so the reconstruction works on T_n U: for cell c across its
 * local edge m (n = c's outward normal there) it returns h, b- and the
 * normal and tangential velocities u_n, u_t at the edge midpoint.
 * Reconstructed variables: h, eta = h + b, u_n, u_t (velocities rather than
 * discharges: near a wet/dry front h- -> 0 and a reconstructed discharge
 * gives an unbounded hu-/h-, while a limited velocity stays in the range of
 * the stencil's velocities); b- = eta- - h-.
 * The upwind value is the mean of the two other neighbours of c (the one
 * present if the other is missing), x_upw the mean of their centroids, x_RL
 * the edge midpoint.  First order (cell values) when the scheme is not MUSCL,
 * when c has no neighbour across m, when any stencil cell is dry (h <= eps),
 * when both upwind cells are missing, or when the reconstructed depth is
 * negative.
 * ---------------------------------------------------------------------- */
typedef struct { double h, b, un, ut; int second; } iface;

static double side_limiter(const or_params *P, double sb, double sf)
{
    switch (P->limiter) {
    case OR_MINMOD: return limit_beta(1.0, sb, sf);
    case OR_SUPERBEE: return limit_beta(2.0, sb, sf);
    case OR_VANALBADA: return limit_vanalbada(sb, sf);
    case OR_ZEROSLOPE: return 0.0;
    default: return limit_beta(1.0, sb, sf);
    }
}

/* (h, eta, u_n, u_t) of cell o in the frame of normal (nx, ny) */
static void frame_state(const or_mesh *M, const double *h, const double *hu, const double *hv,
                        double eps, int o, double nx, double ny, double q[4])
{
    double u = h[o] > eps ? hu[o] / h[o] : 0.0, v = h[o] > eps ? hv[o] / h[o] : 0.0;
    q[0] = h[o];
    q[1] = h[o] + M->b[o];
    q[2] = u * nx + v * ny;
    q[3] = -u * ny + v * nx;
}

static iface reconstruct(const or_mesh *M, const or_params *P, const double *h, const double *hu,
                         const double *hv, int c, int m)
{
    double eps = P->eps, nx = M->enx[3 * c + m], ny = M->eny[3 * c + m];
    double qc[4];
    frame_state(M, h, hu, hv, eps, c, nx, ny, qc);
    iface r = {h[c], M->b[c], qc[2], qc[3], 0};
    if (P->scheme != OR_MUSCL) return r;
    int k = M->nbr[3 * c + m];
    if (k < 0) return r;
    int a = M->nbr[3 * c + (m + 1) % 3], bb = M->nbr[3 * c + (m + 2) % 3];
    if (h[c] <= eps || h[k] <= eps) return r;
    if (a >= 0 && h[a] <= eps) return r;
    if (bb >= 0 && h[bb] <= eps) return r;
    if (a < 0 && bb < 0) return r;
    double qk[4], qu[4], xu, yu, bu, qnu, qtu;
    frame_state(M, h, hu, hv, eps, k, nx, ny, qk);
    if (a >= 0 && bb >= 0) {
        double qa[4], qb[4];
        frame_state(M, h, hu, hv, eps, a, nx, ny, qa);
        frame_state(M, h, hu, hv, eps, bb, nx, ny, qb);
        for (int i = 0; i < 4; ++i) qu[i] = 0.5 * (qa[i] + qb[i]);
        xu = 0.5 * (M->cx[a] + M->cx[bb]);
        yu = 0.5 * (M->cy[a] + M->cy[bb]);
        bu = 0.5 * (M->b[a] + M->b[bb]);
        qnu = 0.5 * ((hu[a] * nx + hv[a] * ny) + (hu[bb] * nx + hv[bb] * ny));
        qtu = 0.5 * ((-hu[a] * ny + hv[a] * nx) + (-hu[bb] * ny + hv[bb] * nx));
    } else {
        int o = a >= 0 ? a : bb;
        frame_state(M, h, hu, hv, eps, o, nx, ny, qu);
        xu = M->cx[o]; yu = M->cy[o];
        bu = M->b[o];
        qnu = hu[o] * nx + hv[o] * ny;
        qtu = -hu[o] * ny + hv[o] * nx;
    }
    double du = hypot(M->cx[c] - xu, M->cy[c] - yu);
    double df = hypot(M->cx[k] - M->cx[c], M->cy[k] - M->cy[c]);
    double dm = hypot(M->emx[3 * c + m] - M->cx[c], M->emy[3 * c + m] - M->cy[c]);
    double out[4];
    int learned_ok = 0;
    (void)bu; (void)qnu; (void)qtu;
    if (P->limiter == OR_LEARNED && P->mlp) {
        /* slope = phi * central slope (U_R - U_Lupw)/|x_R - x_Lupw|, with the
         * phi of this half-edge evaluated once per step from the state the
         * step starts from (step_phi) */
        double phi = M->phi[3 * c + m];
        if (phi >= 0.0 && phi <= 1.0) { /* NaN fails both tests */
            double dc = hypot(M->cx[k] - xu, M->cy[k] - yu);
            for (int i = 0; i < 4; ++i) {
                double sb = (qc[i] - qu[i]) / du, sf = (qk[i] - qc[i]) / df;
                out[i] = qc[i] + dm * tvd_clip(phi * ((qk[i] - qu[i]) / dc), sb, sf);
            }
            learned_ok = out[0] >= 0.0;
        }
    }
    if (!learned_ok) { /* classic limiter; the learned limiter falls back to minmod */
        for (int i = 0; i < 4; ++i) {
            double sb = (qc[i] - qu[i]) / du, sf = (qk[i] - qc[i]) / df;
            out[i] = qc[i] + dm * side_limiter(P, sb, sf);
        }
    }
    if (out[0] < 0.0) return r;
    r.h = out[0]; r.b = out[1] - out[0]; r.un = out[2]; r.ut = out[3];
    r.second = 1;
    return r;
}

/* Inputs of the learned limiter for every half-edge (test access): for
 * half-edge e = 3c+m, out[32*e ..]: features[14], cell values (h, eta, u_n,
 * u_t)[4] in c's edge frame, central slopes (U_R - U_Lupw)/|x_R - x_Lupw|[4],
 * d_mid, eligibility (1: reconstructed to second order by MUSCL, 0: first
 * order), backward slopes (q_c - q_upw)/d_up [4] and forward slopes
 * (q_R - q_c)/d_fwd [4] (zero where not eligible); phi[e] = network output
 * (bf16 layer inputs if P->mlp_bf16), NaN where not eligible. */
static void halfedge_inputs(const or_mesh *M, const or_params *P, const double *h,
                            const double *hu, const double *hv, int c, int m, double o[32],
                            double *phi)
{
    double eps = P->eps;
    int e = 3 * c + m;
    for (int i = 0; i < 32; ++i) o[i] = 0.0;
    *phi = NAN;                               /* not evaluated */
    double nx = M->enx[e], ny = M->eny[e];
    double qc[4];
    frame_state(M, h, hu, hv, eps, c, nx, ny, qc);
    for (int i = 0; i < 4; ++i) o[14 + i] = qc[i];
    double dm = hypot(M->emx[e] - M->cx[c], M->emy[e] - M->cy[c]);
    o[22] = dm;
    int k = M->nbr[e];
    if (k < 0) return;
    int a = M->nbr[3 * c + (m + 1) % 3], bb = M->nbr[3 * c + (m + 2) % 3];
    if (h[c] <= eps || h[k] <= eps) return;
    if ((a >= 0 && h[a] <= eps) || (bb >= 0 && h[bb] <= eps) || (a < 0 && bb < 0)) return;
    double qk[4], qu[4], xu, yu, bu, qnu, qtu;
    frame_state(M, h, hu, hv, eps, k, nx, ny, qk);
    if (a >= 0 && bb >= 0) {
        double qa[4], qb[4];
        frame_state(M, h, hu, hv, eps, a, nx, ny, qa);
        frame_state(M, h, hu, hv, eps, bb, nx, ny, qb);
        for (int i = 0; i < 4; ++i) qu[i] = 0.5 * (qa[i] + qb[i]);
        xu = 0.5 * (M->cx[a] + M->cx[bb]); yu = 0.5 * (M->cy[a] + M->cy[bb]);
        bu = 0.5 * (M->b[a] + M->b[bb]);
        qnu = 0.5 * ((hu[a] * nx + hv[a] * ny) + (hu[bb] * nx + hv[bb] * ny));
        qtu = 0.5 * ((-hu[a] * ny + hv[a] * nx) + (-hu[bb] * ny + hv[bb] * nx));
    } else {
        int oo = a >= 0 ? a : bb;
        frame_state(M, h, hu, hv, eps, oo, nx, ny, qu);
        xu = M->cx[oo]; yu = M->cy[oo]; bu = M->b[oo];
        qnu = hu[oo] * nx + hv[oo] * ny;
        qtu = -hu[oo] * ny + hv[oo] * nx;
    }
    double du = hypot(M->cx[c] - xu, M->cy[c] - yu);
    double df = hypot(M->cx[k] - M->cx[c], M->cy[k] - M->cy[c]);
    double dc = hypot(M->cx[k] - xu, M->cy[k] - yu);
    double qcb[4] = {h[c], hu[c] * nx + hv[c] * ny, -hu[c] * ny + hv[c] * nx, M->b[c]};
    double qub[4] = {qu[0], qnu, qtu, bu};
    double qkb[4] = {h[k], hu[k] * nx + hv[k] * ny, -hu[k] * ny + hv[k] * nx, M->b[k]};
    halfedge_features(P->g, qcb, qub, qkb, du, df, dm, h[c], qc[2], qc[3], h[k], o);
    for (int i = 0; i < 4; ++i) {
        o[18 + i] = (qk[i] - qu[i]) / dc;
        o[24 + i] = (qc[i] - qu[i]) / du;
        o[28 + i] = (qk[i] - qc[i]) / df;
    }
    o[23] = 1.0;
    if (P->mlp) {
        mlp_view v = mlp_unpack(P->mlp);
        double a1[MLP_H], a2[MLP_H], z;
        *phi = mlp_forward(&v, o, P->mlp_bf16, a1, a2, &z);
    }
}

int or_limiter_inputs(const or_mesh *M, const or_params *P, const double *h, const double *hu,
                      const double *hv, double *out, double *phi)
{
    for (int c = 0; c < M->nc; ++c)
        for (int m = 0; m < 3; ++m)
            halfedge_inputs(M, P, h, hu, hv, c, m, out + 32 * (size_t)(3 * c + m), &phi[3 * c + m]);
    return 0;
}

/* The learned limiter's phi of every half-edge, evaluated once per time step
 * from the state the step starts from and used by both RK2 stages.  Where
 * that state does not reconstruct the half-edge to second order phi is not
 * evaluated (NaN); a stage that does reconstruct it there (its own state
 * decides) falls back to minmod, as for a network output outside [0, 1]. */
static void step_phi(or_mesh *M, const or_params *P, const double *h, const double *hu,
                     const double *hv)
{
    if (P->limiter != OR_LEARNED || !P->mlp || P->scheme != OR_MUSCL) return;
    double o[32];
    for (int c = 0; c < M->nc; ++c)
        for (int m = 0; m < 3; ++m) halfedge_inputs(M, P, h, hu, hv, c, m, o, &M->phi[3 * c + m]);
}

/* rotation T_n of Sec. 6.1 and its inverse */
static void rot(double nx, double ny, double h, double hu, double hv, double U[3])
{
    U[0] = h; U[1] = hu * nx + hv * ny; U[2] = -hu * ny + hv * nx;
}

static void unrot(double nx, double ny, const double F[3], double G[3])
{
    G[0] = F[0]; G[1] = F[1] * nx - F[2] * ny; G[2] = F[1] * ny + F[2] * nx;
}

static double inflow_at(const or_params *P, double t)
{
    if (P->n_series <= 0) return P->inflow_q;
    const double *T = P->series_t, *Q = P->series_q;
    int n = P->n_series;
    if (t <= T[0]) return Q[0];
    if (t >= T[n - 1]) return Q[n - 1];
    for (int i = 0; i + 1 < n; ++i)
        if (t <= T[i + 1]) return Q[i] + (Q[i + 1] - Q[i]) * (t - T[i]) / (T[i + 1] - T[i]);
    return Q[n - 1];
}

/* ------------------------------------------------------------------------
 * Boundary fluxes (Sec. 6.1): transmissive = Riemann problem with U_R = U_L;
 * inflow (Q, Q^2/h_l + g h_l^2/2, 0) with Q the inward discharge per unit
 * width (total discharge over the total inflow length, h_l floored at 1 mm in
 * Q^2/h_l); wall (0, g h_l^2/2, 0); fixed-stage outflow = Riemann problem
 * against a ghost at the prescribed stage with the cell's velocity.
 * Sub-domain cut edges (outermost ghost layer) are transmissive.
 * ---------------------------------------------------------------------- */
static void boundary_flux(const or_mesh *M, const or_params *P, int tag, int c, int m,
                          double hc, double huc, double hvc, double t, double G[3])
{
    double nx = M->enx[3 * c + m], ny = M->eny[3 * c + m], g = P->g, eps = P->eps;
    double U[3], F[3];
    rot(nx, ny, hc, huc, hvc, U);
    if (tag == BC_WALL) {
        F[0] = 0.0; F[1] = 0.5 * g * hc * hc; F[2] = 0.0;
    } else if (tag == BC_INFLOW) {
        double q = inflow_at(P, t) / P->inflow_len;
        double hl = dmax(hc, 1e-3);
        F[0] = -q; F[1] = q * q / hl + 0.5 * g * hc * hc; F[2] = 0.0;
    } else if (tag == BC_OUTFLOW) {
        double hg = dmax(0.0, P->outflow_stage - M->b[c]);
        double un = hc > eps ? U[1] / hc : 0.0, ut = hc > eps ? U[2] / hc : 0.0;
        double UG[3] = {hg, hg * un, hg * ut};
        flux_hllc(g, eps, U, UG, F);
    } else { /* transmissive or sub-domain cut */
        flux_hllc(g, eps, U, U, F);
    }
    unrot(nx, ny, F, G);
}

/* ------------------------------------------------------------------------
 * One explicit stage (Sec. 6.1, eq. vlap2):
 *   U* = U + dt * R(U),
 *   R_i = -(1/|Omega_i|) sum_j L_ij [ T^-1 G~(U*_L, U*_R) + c_ij + s_ij ],
 * with the hydrostatic reconstruction (Audusse et al.) of the interface
 * states: b_e = max(b_L-, b_R-), h*_k = max(0, eta_k- - b_e),
 * U*_k = h*_k (1, u_k, v_k); side correction c = (0, g/2 (h-^2 - h*^2) n);
 * centred bed term s = (0, g/2 (h- + h_i)(b- - b_i) n).  Each interior edge
 * flux is computed once with L = the cell of smaller global id and L's
 * outward normal; the cell sums run over local edges 0, 1, 2 in order.
 * Then Manning friction, point-implicit with this stage's dt, and the
 * wet/dry cleanup (velocities zero where h <= eps).
 * ---------------------------------------------------------------------- */
static void stage(or_mesh *M, const or_params *P, const double *h, const double *hu,
                  const double *hv, double dt, double t, double *oh, double *ohu, double *ohv,
                  int *flags)
{
    int nc = M->nc;
    double g = P->g, eps = P->eps;
    /* interface values, both sides of every edge */
    for (int c = 0; c < nc; ++c)
        for (int m = 0; m < 3; ++m) {
            iface r = reconstruct(M, P, h, hu, hv, c, m);
            M->rh[3 * c + m] = r.h; M->rb[3 * c + m] = r.b;
            M->run[3 * c + m] = r.un; M->rut[3 * c + m] = r.ut;
        }
    /* edge fluxes */
    for (int c = 0; c < nc; ++c)
        for (int m = 0; m < 3; ++m) {
            int k = M->nbr[3 * c + m], e = 3 * c + m;
            if (k < 0) {
                double G[3];
                boundary_flux(M, P, k, c, m, h[c], hu[c], hv[c], t, G);
                M->fx0[e] = G[0]; M->fx1[e] = G[1]; M->fx2[e] = G[2];
                continue;
            }
            if (!(M->gid[c] < M->gid[k])) continue; /* computed from the other side */
            int L = c, R = k, mR = M->nbr_edge[e], eR = 3 * R + mR;
            double nx = M->enx[e], ny = M->eny[e];
            /* hydrostatic reconstruction */
            double hL = M->rh[e], hR = M->rh[eR];
            double bL = M->rb[e], bR = M->rb[eR];
            double be = dmax(bL, bR);
            double hsL = dmax(0.0, hL + bL - be), hsR = dmax(0.0, hR + bR - be);
            /* normal-frame states; R's values are in its own frame (-n, -t) */
            double UL[3] = {hsL, hsL * M->run[e], hsL * M->rut[e]};
            double UR[3] = {hsR, -(hsR * M->run[eR]), -(hsR * M->rut[eR])};
            double F[3], G[3];
            if (P->scheme == OR_WAF) {
                /* upwind cells of L and R: their two other neighbours */
                int La = M->nbr[3 * L + (m + 1) % 3], Lb = M->nbr[3 * L + (m + 2) % 3];
                int Ra = M->nbr[3 * R + (mR + 1) % 3], Rb = M->nbr[3 * R + (mR + 2) % 3];
                waf_ratio_in rh_, rv_;
                double vt[4];
                int ids[4] = {La, Lb, Ra, Rb};
                /* a dry upwind cell counts as missing (first order there, as
                 * for the MUSCL stencil) */
                for (int i = 0; i < 4; ++i)
                    if (ids[i] >= 0 && h[ids[i]] <= eps) ids[i] = -1;
                La = ids[0]; Lb = ids[1]; Ra = ids[2]; Rb = ids[3];
                for (int i = 0; i < 4; ++i) {
                    int o = ids[i];
                    vt[i] = o >= 0 ? (-hu[o] * ny + hv[o] * nx) / h[o] : 0.0;
                }
                /* q = eta = h + b for the L and R waves (equal to h up to a
                 * constant on the flat beds of the paper; keeps the limiter
                 * inactive over bathymetry at rest) */
                rh_.qL = h[L] + M->b[L]; rh_.qR = h[R] + M->b[R];
                rv_.qL = h[L] > eps ? (-hu[L] * ny + hv[L] * nx) / h[L] : 0.0;
                rv_.qR = h[R] > eps ? (-hu[R] * ny + hv[R] * nx) / h[R] : 0.0;
                rh_.hasLu = rv_.hasLu = (La >= 0 || Lb >= 0);
                rh_.hasRu = rv_.hasRu = (Ra >= 0 || Rb >= 0);
                double et[4];
                for (int i = 0; i < 4; ++i) et[i] = ids[i] >= 0 ? h[ids[i]] + M->b[ids[i]] : 0.0;
                if (La >= 0 && Lb >= 0) { rh_.qLu = 0.5 * (et[0] + et[1]); rv_.qLu = 0.5 * (vt[0] + vt[1]); }
                else if (La >= 0) { rh_.qLu = et[0]; rv_.qLu = vt[0]; }
                else if (Lb >= 0) { rh_.qLu = et[1]; rv_.qLu = vt[1]; }
                if (Ra >= 0 && Rb >= 0) { rh_.qRu = 0.5 * (et[2] + et[3]); rv_.qRu = 0.5 * (vt[2] + vt[3]); }
                else if (Ra >= 0) { rh_.qRu = et[2]; rv_.qRu = vt[2]; }
                else if (Rb >= 0) { rh_.qRu = et[3]; rv_.qRu = vt[3]; }
                double dx = hypot(M->cx[R] - M->cx[L], M->cy[R] - M->cy[L]);
                flux_waf(g, eps, P->waf_limiter, dt / dx, UL, UR, &rh_, &rv_, F);
                if (P->waf_pos)
                    waf_positivity(g, eps, UL, UR, h[L], M->inr[L], h[R], M->inr[R], dt, F);
            } else {
                flux_hllc(g, eps, UL, UR, F);
            }
            unrot(nx, ny, F, G);
            double pL = 0.5 * g * (hL * hL - hsL * hsL), pR = 0.5 * g * (hR * hR - hsR * hsR);
            M->fx0[e] = G[0]; M->fx1[e] = G[1] + pL * nx; M->fx2[e] = G[2] + pL * ny;
            /* R's outward normal is -n */
            M->fx0[eR] = -G[0]; M->fx1[eR] = -G[1] - pR * nx; M->fx2[eR] = -G[2] - pR * ny;
        }
    /* cell sums, update, friction, cleanup */
    for (int c = 0; c < nc; ++c) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int m = 0; m < 3; ++m) {
            int e = 3 * c + m;
            double L = M->elen[e], nx = M->enx[e], ny = M->eny[e];
            double s = 0.5 * g * (M->rh[e] + h[c]) * (M->rb[e] - M->b[c]);
            a0 += L * M->fx0[e];
            a1 += L * (M->fx1[e] + s * nx);
            a2 += L * (M->fx2[e] + s * ny);
        }
        double nh = h[c] - dt * a0 / M->area[c];
        double nu = hu[c] - dt * a1 / M->area[c];
        double nv = hv[c] - dt * a2 / M->area[c];
        if (!(isfinite(nh) && isfinite(nu) && isfinite(nv))) *flags |= FL_NONFINITE;
        if (nh < 0.0) {
            *flags |= (nh < -eps) ? FL_NEGDEPTH : FL_CLIPPED;
            nh = 0.0;
        }
        if (nh <= eps) {
            nu = 0.0; nv = 0.0;
        } else if (M->man[c] > 0.0) {
            double sp = sqrt(nu * nu + nv * nv) / nh;
            double f = 1.0 + dt * g * M->man[c] * M->man[c] * sp * pow(nh, -4.0 / 3.0);
            nu /= f; nv /= f;
        }
        oh[c] = nh; ohu[c] = nu; ohv[c] = nv;
    }
}

/* ------------------------------------------------------------------------
 * CFL time step (Sec. 6.1, CFL condition with d = R_L, the inscribed radius).
 * Reading: per-cell minimum of R_i / (|u_i| + sqrt(g h_i)) over wet owned
 * cells (cfl_rule 0), or the printed global form min R / max speed
 * (cfl_rule 1).  No wet cell: dt_max.  dt is capped by dt_max when > 0.
 * ---------------------------------------------------------------------- */
int or_dt(const or_mesh *M, const or_params *P, const double *h, const double *hu,
          const double *hv, double *dt_out)
{
    double best = INFINITY, rmin = INFINITY, lmax = 0.0;
    int wet = 0;
    for (int c = 0; c < M->n_owned; ++c) {
        if (h[c] <= P->eps) continue;
        double u = hu[c] / h[c], v = hv[c] / h[c];
        double lam = sqrt(u * u + v * v) + sqrt(P->g * h[c]);
        wet = 1;
        best = dmin(best, M->inr[c] / lam);
        rmin = dmin(rmin, M->inr[c]);
        lmax = dmax(lmax, lam);
    }
    double dt;
    if (!wet) {
        if (!(P->dt_max > 0.0)) return -1;
        dt = P->dt_max;
    } else {
        dt = P->cfl_rule == 1 ? P->cfl * rmin / lmax : P->cfl * best;
        if (P->dt_max > 0.0) dt = dmin(dt, P->dt_max);
    }
    *dt_out = dt;
    return 0;
}

/* ------------------------------------------------------------------------
 * Time integration (Sec. 6.1): explicit Euler; MUSCL is run with the two-
 * stage SSP Runge-Kutta (Heun) form U1 = E(U^n), U2 = E(U1),
 * U^{n+1} = (U^n + U2)/2 with the same dt for both stages, then the wet/dry
 * cleanup.  dt_fixed > 0 overrides the CFL step.
 * ---------------------------------------------------------------------- */
int or_run(or_mesh *M, const or_params *P, double *h, double *hu, double *hv, int nsteps,
           double dt_fixed, double *t, int *flags)
{
    int nc = M->nc;
    for (int s = 0; s < nsteps; ++s) {
        double dt;
        if (dt_fixed > 0.0) dt = dt_fixed;
        else if (or_dt(M, P, h, hu, hv, &dt) != 0) return -1;
        if (P->phi_every <= 1 || s % P->phi_every == 0) step_phi(M, P, h, hu, hv);
        if (P->integrator == OR_RK2) {
            stage(M, P, h, hu, hv, dt, *t, M->u0h, M->u0u, M->u0v, flags);
            stage(M, P, M->u0h, M->u0u, M->u0v, dt, *t + dt, M->u1h, M->u1u, M->u1v, flags);
            for (int c = 0; c < nc; ++c) {
                double nh = 0.5 * (h[c] + M->u1h[c]);
                double nu = 0.5 * (hu[c] + M->u1u[c]);
                double nv = 0.5 * (hv[c] + M->u1v[c]);
                if (nh <= P->eps) { nu = 0.0; nv = 0.0; }
                h[c] = nh; hu[c] = nu; hv[c] = nv;
            }
        } else {
            stage(M, P, h, hu, hv, dt, *t, M->u0h, M->u0u, M->u0v, flags);
            memcpy(h, M->u0h, sizeof(double) * nc);
            memcpy(hu, M->u0u, sizeof(double) * nc);
            memcpy(hv, M->u0v, sizeof(double) * nc);
        }
        *t += dt;
    }
    return 0;
}

/* Interface values (h-, b-, u_n-, u_t- in the half-edge's own outward-normal
 * frame) and the "second order" flag of every
 * half-edge for the given state (exposed for tests and feature extraction). */
int or_interfaces(or_mesh *M, const or_params *P, const double *h, const double *hu,
                  const double *hv, double *rh, double *rb, double *run, double *rut, int *second)
{
    step_phi(M, P, h, hu, hv);
    for (int c = 0; c < M->nc; ++c)
        for (int m = 0; m < 3; ++m) {
            iface r = reconstruct(M, P, h, hu, hv, c, m);
            int e = 3 * c + m;
            rh[e] = r.h; rb[e] = r.b; run[e] = r.un; rut[e] = r.ut; second[e] = r.second;
        }
    return 0;
}

/* The positivity blend of WAF on one edge (tests): F (in/out) is a flux in
 * the normal frame for the states UL, UR. */
int or_waf_positivity(const or_params *P, const double *UL, const double *UR, double hL,
                      double RL, double hR, double RR, double dt, double *F)
{
    waf_positivity(P->g, P->eps, UL, UR, hL, RL, hR, RR, dt, F);
    return 0;
}

/* Flux of one Riemann problem in the normal frame (tests). */
int or_riemann(const or_params *P, int scheme, const double *UL, const double *UR, double dt_dx,
               const double *ratio_in /* qL,qR,qLu,qRu for h then v; NULL = none */,
               double *F)
{
    if (scheme == OR_WAF) {
        waf_ratio_in rh = {0, 0, 0, 0, 0, 0}, rv = {0, 0, 0, 0, 0, 0};
        if (ratio_in) {
            rh.qL = ratio_in[0]; rh.qR = ratio_in[1]; rh.qLu = ratio_in[2]; rh.qRu = ratio_in[3];
            rv.qL = ratio_in[4]; rv.qR = ratio_in[5]; rv.qLu = ratio_in[6]; rv.qRu = ratio_in[7];
            rh.hasLu = rh.hasRu = rv.hasLu = rv.hasRu = 1;
        }
        flux_waf(P->g, P->eps, P->waf_limiter, dt_dx, UL, UR, &rh, &rv, F);
    } else {
        flux_hllc(P->g, P->eps, UL, UR, F);
    }
    return 0;
}

double or_limiter(int kind, double sb, double sf)
{
    if (kind == OR_MINMOD) return limit_beta(1.0, sb, sf);
    if (kind == OR_SUPERBEE) return limit_beta(2.0, sb, sf);
    if (kind == OR_VANALBADA) return limit_vanalbada(sb, sf);
    return 0.0;
}

double or_superbee_A(double r, double c) { return superbee_A(r, c); }

double or_bf16(double x) { return to_bf16(x); }
