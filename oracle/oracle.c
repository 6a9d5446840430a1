/*
 * oracle.c -- plain FP64 CPU reference of the MAP EGLM-MHD block update.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for readability, not
 * speed: every quantity is computed where the paper defines it, with
 * temporary arrays instead of fusion, and in the order the equations are
 * printed.  Build with -O2 -ffp-contract=off and no fast-math.
 *
 * Section references are to the paper (Jiang, Fang & Chen, MAP):
 *   Sec. 2  EGLM-MHD equations (MHD-1..MHD-5), c_h and c_p
 *   Sec. 3  conservative update (Equ:basic), MMC, LF (Equ:LFFlux,
 *           limiter1/limiter2, minmod), resistivity, multi-D and dt
 *   Sec. 4.3 boundary procedure: restriction, reflux, exchange, conservative
 *           prolongation (Matsumoto's minmod interpolation)
 *   Sec. 4.5 regrid error estimator
 *   Sec. 5  error norms
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, BX = 4, BY = 5, BZ = 6, EN = 7, PSI = 8 };
#define NVMAX 9

/* ------------------------------------------------------------------ */
/* tile geometry                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    int nd;
    int n[3], g[3], p[3];
    long s[3];  /* strides of x, y, z in the padded tile */
    long P;     /* cells per variable in the padded tile */
    long I;     /* interior cells per variable */
} geo;

static geo mkgeo(int nd, const int n_in[3])
{
    geo G;
    G.nd = nd;
    for (int d = 0; d < 3; d++) {
        G.n[d] = (d < nd) ? n_in[d] : 1;
        G.g[d] = (d < nd) ? 2 : 0;
        G.p[d] = G.n[d] + 2 * G.g[d];
    }
    G.s[0] = 1;
    G.s[1] = G.p[0];
    G.s[2] = (long)G.p[0] * G.p[1];
    G.P = (long)G.p[0] * G.p[1] * G.p[2];
    G.I = (long)G.n[0] * G.n[1] * G.n[2];
    return G;
}

static long at(const geo *G, int x, int y, int z)
{
    return ((long)(z + G->g[2]) * G->p[1] + (y + G->g[1])) * G->p[0] + (x + G->g[0]);
}

static long interior_index(const geo *G, int x, int y, int z)
{
    return ((long)z * G->n[1] + y) * G->n[0] + x;
}

/* ------------------------------------------------------------------ */
/* pointwise physics                                                   */
/* ------------------------------------------------------------------ */
int orc_nvar(const orc_params *p) { return p->physics == ORC_MHD ? 9 : 1; }

/* Threads of the block-tree loops (orc_amr_*).  Each block's arithmetic is
 * the same whichever thread runs it and no reduction order depends on the
 * thread count (maxima are exact, the totals stay serial), so every result
 * is bit for bit the one-thread result.  Default 1. */
static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return g_threads; }

/* p = (gamma-1)(e - rho v^2/2 - B^2/2)   (Sec. 2, below MHD-04) */
double orc_pressure(const orc_params *p, const double *u)
{
    double ir = 1.0 / u[RHO];
    double vx = u[MX] * ir, vy = u[MY] * ir, vz = u[MZ] * ir;
    double ke = 0.5 * (u[MX] * vx + u[MY] * vy + u[MZ] * vz);
    double me = 0.5 * (u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ]);
    return (p->gamma - 1.0) * (u[EN] - ke - me);
}

/* flux of the EGLM-MHD system in direction `dim` (MHD-1..MHD-5):
 * mass m_d; momentum m_j v_d - B_j B_d + delta_jd (p + B^2/2);
 * induction B_j v_d - B_d v_j plus psi on the normal component;
 * energy (e + p + B^2/2) v_d - B_d (v.B); psi: c_h^2 B_d. */
void orc_flux(const orc_params *p, const double *u, int d, double ch, double *f)
{
    if (p->physics == ORC_SCALAR) {
        f[0] = p->adv[d] * u[0];
        return;
    }
    double ir = 1.0 / u[RHO];
    double v[3] = {u[MX] * ir, u[MY] * ir, u[MZ] * ir};
    const double *B = u + BX;
    double ke = 0.5 * (u[MX] * v[0] + u[MY] * v[1] + u[MZ] * v[2]);
    double me = 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    double pr = (p->gamma - 1.0) * (u[EN] - ke - me);
    double pt = pr + me;
    double vd = v[d], Bd = B[d];
    double vb = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
    f[RHO] = u[MX + d];
    for (int j = 0; j < 3; j++)
        f[MX + j] = u[MX + j] * vd - B[j] * Bd;
    f[MX + d] = f[MX + d] + pt;
    for (int j = 0; j < 3; j++)
        f[BX + j] = B[j] * vd - Bd * v[j];
    f[BX + d] = u[PSI];
    f[EN] = (u[EN] + pt) * vd - Bd * vb;
    f[PSI] = ch * ch * Bd;
}

/* fast magnetosonic speed along d */
static double fast_speed(const orc_params *p, const double *u, int d)
{
    double ir = 1.0 / u[RHO];
    double pr = orc_pressure(p, u);
    double a2 = p->gamma * pr * ir;
    double bb = u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ];
    double b2 = bb * ir;
    double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * (u[BX + d] * u[BX + d]) * ir;
    if (disc < 0.0)
        disc = 0.0;
    double cf2 = 0.5 * (s + sqrt(disc));
    if (cf2 < 0.0)
        cf2 = 0.0;
    return sqrt(cf2);
}

/* |v_d| + fast magnetosonic speed along d: the local largest eigenvalue of
 * the MHD part (Sec. 3.1-3.2); the GLM speed c_h is handled separately. */
double orc_speed(const orc_params *p, const double *u, int d)
{
    if (p->physics == ORC_SCALAR)
        return fabs(p->adv[d]);
    double ir = 1.0 / u[RHO];
    double pr = orc_pressure(p, u);
    double a2 = p->gamma * pr * ir;
    double bb = u[BX] * u[BX] + u[BY] * u[BY] + u[BZ] * u[BZ];
    double b2 = bb * ir;
    double s = a2 + b2;
    double disc = s * s - 4.0 * a2 * (u[BX + d] * u[BX + d]) * ir;
    if (disc < 0.0)
        disc = 0.0;
    double cf2 = 0.5 * (s + sqrt(disc));
    if (cf2 < 0.0)
        cf2 = 0.0;
    return fabs(u[MX + d] * ir) + sqrt(cf2);
}

static double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

/* minmod(a,b) = sgn(a) max(0, min(|a|, sgn(a) b))   (eq. minmod)
 * van Leer:      (ab + |ab|)/(a + b)
 * literal flux limiter of Sec. 3.1 in ratio-free form: phi(a/b) b. */
double orc_limiter(int kind, double a, double b)
{
    if (kind == ORC_MINMOD) {
        double s = sgn(a);
        double m = fabs(a);
        double t = s * b;
        if (t < m)
            m = t;
        if (m < 0.0)
            m = 0.0;
        return s * m;
    }
    if (kind == ORC_VANLEER) {
        double ab = a * b;
        if (ab <= 0.0)
            return 0.0;
        return (ab + fabs(ab)) / (a + b);
    }
    /* ORC_PAPER_PHI: phi(r) = r for |r| <= 1, 1 otherwise, r = a/b */
    return (fabs(a) <= fabs(b)) ? a : b;
}

static int admissible(const orc_params *p, const double *u)
{
    if (p->physics == ORC_SCALAR)
        return 1;
    if (!(u[RHO] > 0.0))
        return 0;
    return orc_pressure(p, u) > 0.0;
}

/* the GLM pair (B_d, psi) is transported at speed c_h */
static int glm_component(const orc_params *p, int k, int d)
{
    return p->physics == ORC_MHD && (k == BX + d || k == PSI);
}

/* primitive (rho, v, B, p, psi) -> conserved (rho, rho v, B, e, psi);
 * w is [9][ncell].  e = p/(gamma-1) + rho v^2/2 + B^2/2 (Sec. 2). */
void orc_prim_to_cons(const orc_params *p, double *w, long nc)
{
    if (p->physics == ORC_SCALAR)
        return;
    for (long c = 0; c < nc; c++) {
        double r = w[RHO * nc + c];
        double vx = w[MX * nc + c], vy = w[MY * nc + c], vz = w[MZ * nc + c];
        double bx = w[BX * nc + c], by = w[BY * nc + c], bz = w[BZ * nc + c];
        double pr = w[EN * nc + c];
        double e = pr / (p->gamma - 1.0) + 0.5 * r * (vx * vx + vy * vy + vz * vz)
                   + 0.5 * (bx * bx + by * by + bz * bz);
        w[MX * nc + c] = r * vx;
        w[MY * nc + c] = r * vy;
        w[MZ * nc + c] = r * vz;
        w[EN * nc + c] = e;
    }
}

/* ------------------------------------------------------------------ */
/* one padded tile                                                     */
/* ------------------------------------------------------------------ */
static void load(const double *u, long P, int nv, long c, double *out)
{
    for (int k = 0; k < nv; k++)
        out[k] = u[k * P + c];
}

/* the (n+2)^d region E: one ring outside the interior */
static void e_range(const geo *G, int lo[3], int hi[3])
{
    for (int d = 0; d < 3; d++) {
        lo[d] = (d < G->nd) ? -1 : 0;
        hi[d] = (d < G->nd) ? G->n[d] + 1 : G->n[d];
    }
}

/* LF predictor (limiter1 + the half-step formula): per cell of E,
 * slopes from the old-time differences, fall-back to zero slopes if a face
 * state is not admissible, then u~ = u - dt/(2dx) sum_d [f(u+D/2) - f(u-D/2)]. */
static void lf_predict(const orc_params *p, const geo *G, const double *u,
                       const double hdt[3], double ch, double *ut, double *sl,
                       long *cnt)
{
    int nv = orc_nvar(p), nd = G->nd;
    long P = G->P;
    int lo[3], hi[3];
    e_range(G, lo, hi);
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(G, x, y, z);
                double uc[NVMAX], s[3][NVMAX];
                load(u, P, nv, c, uc);
                for (int d = 0; d < nd; d++)
                    for (int k = 0; k < nv; k++) {
                        double a = uc[k] - u[k * P + c - G->s[d]];
                        double b = u[k * P + c + G->s[d]] - uc[k];
                        s[d][k] = orc_limiter(p->limiter, a, b);
                    }
                int ok = 1;
                for (int d = 0; d < nd; d++) {
                    double up[NVMAX], um[NVMAX];
                    for (int k = 0; k < nv; k++) {
                        up[k] = uc[k] + 0.5 * s[d][k];
                        um[k] = uc[k] - 0.5 * s[d][k];
                    }
                    if (!admissible(p, up) || !admissible(p, um))
                        ok = 0;
                }
                if (!ok) {
                    memset(s, 0, sizeof(s));
                    cnt[0]++;
                }
                double acc[NVMAX] = {0};
                for (int d = 0; d < nd; d++) {
                    double up[NVMAX], um[NVMAX], fp[NVMAX], fm[NVMAX];
                    for (int k = 0; k < nv; k++) {
                        up[k] = uc[k] + 0.5 * s[d][k];
                        um[k] = uc[k] - 0.5 * s[d][k];
                    }
                    orc_flux(p, up, d, ch, fp);
                    orc_flux(p, um, d, ch, fm);
                    for (int k = 0; k < nv; k++)
                        acc[k] += hdt[d] * (fp[k] - fm[k]);
                }
                for (int k = 0; k < nv; k++) {
                    ut[k * P + c] = uc[k] - acc[k];
                    for (int d = 0; d < nd; d++)
                        sl[((long)d * nv + k) * P + c] = s[d][k];
                }
            }
}

/* Rusanov flux (Equ:LFFlux): alpha = the larger fast speed |v_d| + c_f of
 * the two states for the MHD components, c_h for the GLM pair (B_d, psi),
 * which makes the pair's flux Dedner's exact upwind flux of its linear
 * system. */
static void rusanov_flux(const orc_params *p, const double *L, const double *R, int d, double ch,
                         double *f)
{
    int nv = orc_nvar(p);
    double FL[NVMAX], FR[NVMAX];
    orc_flux(p, L, d, ch, FL);
    orc_flux(p, R, d, ch, FR);
    double aL = orc_speed(p, L, d), aR = orc_speed(p, R, d);
    double a = aL > aR ? aL : aR;
    for (int k = 0; k < nv; k++) {
        double al = glm_component(p, k, d) ? ch : a;
        f[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * al * (R[k] - L[k]);
    }
}

/* HLLC flux (the paper names the HLLC solver of Gurski for MHD without
 * printing it; this is that construction with the intermediate states of
 * Li's HLLC for MHD), across a face normal to d:
 *  1. The GLM pair (B_d, psi) is a linear system with speeds +-c_h; its
 *     exact interface values are B_m = (B_dL + B_dR)/2 - (psi_R - psi_L)/(2 c_h)
 *     and psi_m = (psi_L + psi_R)/2 - c_h (B_dR - B_dL)/2, with fluxes psi_m
 *     and c_h^2 B_m.  (c_h = 0: B_m is the mean, the flux of B_d is the mean
 *     of psi and that of psi is zero.)
 *  2. Both states take B_d = B_m, so the normal field is continuous, and the
 *     other seven components get the HLLC fan: outer speeds
 *     S_L = min(v_L, v_R) - max(c_fL, c_fR), S_R = max(v_L, v_R) + max(c_fL, c_fR)
 *     (v = v_d, c_f the fast speeds); the HLL mean state
 *     U_hll = (S_R U_R - S_L U_L - F_R + F_L) / (S_R - S_L);
 *     the contact speed S_M = (rho v_d)_hll / rho_hll; the total pressure
 *     of the star region p* = rho_K (S_K - v_K)(S_M - v_K) + p_T,K (the
 *     same from both sides; their mean is used); on side K the star state
 *       rho* = rho_K (S_K - v_K) / (S_K - S_M),  (rho v_d)* = rho* S_M,
 *       (rho v_t)* = [rho_K v_t,K (S_K - v_K) - B_m (B_t,hll - B_t,K)] / (S_K - S_M),
 *       B_t* = B_t,hll,
 *       e* = [e_K (S_K - v_K) - p_T,K v_K + p* S_M + B_m (v_K.B_K - v_hll.B_hll)] / (S_K - S_M),
 *     with v_hll = (rho v)_hll / rho_hll; the flux is F_L (S_L >= 0),
 *     F_L + S_L (U*_L - U_L) (S_L < 0 <= S_M), F_R + S_R (U*_R - U_R)
 *     (S_M < 0 < S_R) or F_R (S_R <= 0). */
typedef struct {
    double Bm, psim;          /* interface values of the GLM pair */
    double S[3];              /* S_L, S_M, S_R */
    double U[2][NVMAX];       /* the two states with B_d = B_m */
    double F[2][NVMAX];       /* their physical fluxes */
    double Us[2][NVMAX];      /* star states (rho, momentum, B, e; psi unused) */
} hllc_fan;

static void hllc_fan_of(const orc_params *p, const double *L0, const double *R0, int d, double ch,
                        hllc_fan *h)
{
    if (ch > 0.0) {
        h->Bm = 0.5 * (L0[BX + d] + R0[BX + d]) - (R0[PSI] - L0[PSI]) / (2.0 * ch);
        h->psim = 0.5 * (L0[PSI] + R0[PSI]) - 0.5 * ch * (R0[BX + d] - L0[BX + d]);
    } else {
        h->Bm = 0.5 * (L0[BX + d] + R0[BX + d]);
        h->psim = 0.5 * (L0[PSI] + R0[PSI]);
    }
    double v[2], pt[2], cf[2], vb[2];
    for (int s = 0; s < 2; s++) {
        const double *u0 = s ? R0 : L0;
        double *U = h->U[s];
        for (int k = 0; k < 9; k++)
            U[k] = u0[k];
        U[BX + d] = h->Bm;
        orc_flux(p, U, d, ch, h->F[s]);
        double ir = 1.0 / U[RHO];
        v[s] = U[MX + d] * ir;
        double bb = U[BX] * U[BX] + U[BY] * U[BY] + U[BZ] * U[BZ];
        pt[s] = orc_pressure(p, U) + 0.5 * bb;
        cf[s] = fast_speed(p, U, d);
        vb[s] = (U[MX] * U[BX] + U[MY] * U[BY] + U[MZ] * U[BZ]) * ir;
    }
    double cmax = cf[0] > cf[1] ? cf[0] : cf[1];
    double SL = (v[0] < v[1] ? v[0] : v[1]) - cmax;
    double SR = (v[0] > v[1] ? v[0] : v[1]) + cmax;
    /* HLL mean state */
    double hll[NVMAX];
    for (int k = 0; k < 9; k++)
        hll[k] = (SR * h->U[1][k] - SL * h->U[0][k] - h->F[1][k] + h->F[0][k]) / (SR - SL);
    hll[BX + d] = h->Bm;
    double vh[3];
    for (int j = 0; j < 3; j++)
        vh[j] = hll[MX + j] / hll[RHO];
    double SM = vh[d];
    double vbh = vh[0] * hll[BX] + vh[1] * hll[BY] + vh[2] * hll[BZ];
    double ps[2];
    for (int s = 0; s < 2; s++) {
        double S = s ? SR : SL;
        ps[s] = h->U[s][RHO] * (S - v[s]) * (SM - v[s]) + pt[s];
    }
    double pst = 0.5 * (ps[0] + ps[1]);
    for (int s = 0; s < 2; s++) {
        const double *U = h->U[s];
        double *st = h->Us[s];
        double S = s ? SR : SL;
        double den = S - SM;
        double sv = S - v[s];
        st[RHO] = U[RHO] * sv / den;
        for (int j = 0; j < 3; j++) {
            if (j == d) {
                st[MX + j] = st[RHO] * SM;
                st[BX + j] = h->Bm;
            } else {
                st[MX + j] = (U[MX + j] * sv - h->Bm * (hll[BX + j] - U[BX + j])) / den;
                st[BX + j] = hll[BX + j];
            }
        }
        st[EN] = (U[EN] * sv - pt[s] * v[s] + pst * SM + h->Bm * (vb[s] - vbh)) / den;
        st[PSI] = 0.0;
    }
    h->S[0] = SL;
    h->S[1] = SM;
    h->S[2] = SR;
}

static void hllc_flux(const orc_params *p, const double *L0, const double *R0, int d, double ch,
                      double *f)
{
    hllc_fan h;
    hllc_fan_of(p, L0, R0, d, ch, &h);
    double SL = h.S[0], SM = h.S[1], SR = h.S[2];
    if (SL >= 0.0 || SR <= 0.0) {
        const double *F = h.F[SL >= 0.0 ? 0 : 1];
        for (int k = 0; k < 8; k++)
            f[k] = F[k];
    } else {
        int s = SM >= 0.0 ? 0 : 1;
        double S = s ? SR : SL;
        for (int k = 0; k < 8; k++)
            f[k] = h.F[s][k] + S * (h.Us[s][k] - h.U[s][k]);
    }
    /* the GLM pair */
    f[BX + d] = h.psim;
    f[PSI] = ch * ch * h.Bm;
}

void orc_hllc_fan(const orc_params *p, const double *L, const double *R, int d, double ch,
                  double S[3], double UsL[9], double UsR[9])
{
    hllc_fan h;
    hllc_fan_of(p, L, R, d, ch, &h);
    for (int k = 0; k < 3; k++)
        S[k] = h.S[k];
    for (int k = 0; k < 9; k++) {
        UsL[k] = h.Us[0][k];
        UsR[k] = h.Us[1][k];
    }
}

void orc_face_flux(const orc_params *p, const double *L, const double *R, int d, double ch,
                   double *f)
{
    if (p->physics == ORC_MHD && p->riemann == ORC_HLLC)
        hllc_flux(p, L, R, d, ch, f);
    else
        rusanov_flux(p, L, R, d, ch, f);
}

/* LF corrector fluxes (limiter2 + Equ:LFFlux) on every face of dimension d
 * that bounds an interior cell; the face c+1/2 is stored at index c. */
static void lf_faces(const orc_params *p, const geo *G, const double *ut,
                     const double *sl, int d, double ch, double *fh, long *cnt,
                     double *lr)
{
    int nv = orc_nvar(p);
    long P = G->P;
    int lo[3] = {0, 0, 0}, hi[3] = {G->n[0], G->n[1], G->n[2]};
    lo[d] = -1;
    hi[d] = G->n[d];
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(G, x, y, z), cn = c + G->s[d];
                double L[NVMAX], R[NVMAX];
                for (int k = 0; k < nv; k++) {
                    L[k] = ut[k * P + c] + 0.5 * sl[((long)d * nv + k) * P + c];
                    R[k] = ut[k * P + cn] - 0.5 * sl[((long)d * nv + k) * P + cn];
                }
                if (!admissible(p, L)) {
                    load(ut, P, nv, c, L);
                    cnt[1]++;
                }
                if (!admissible(p, R)) {
                    load(ut, P, nv, cn, R);
                    cnt[1]++;
                }
                if (lr)  /* the two states the face flux receives */
                    for (int k = 0; k < nv; k++) {
                        lr[k * P + c] = L[k];
                        lr[((long)nv + k) * P + c] = R[k];
                    }
                double fc[NVMAX];
                orc_face_flux(p, L, R, d, ch, fc);
                for (int k = 0; k < nv; k++)
                    fh[k * P + c] = fc[k];
            }
}

/* WENO (Sec. 3.3, component-wise, third order): the states either side of
 * a face from the three cells around each of them, with the smoothness
 * weights a = 1 / (eps + (difference)^2)^2, eps = 1e-12.  The printed
 * denominator of u+ repeats a_{i-1/2}; the weights 1 and 2 of its numerator
 * are read as the denominator a_{i+1/2} + 2 a_{i-1/2}. */
#define WENO_EPS 1e-12
static double sq(double a) { return a * a; }

/* u^-_{i+1/2} from u_{i-1}, u_i, u_{i+1} */
static double weno_minus(double um, double u0, double up)
{
    double ap = 1.0 / sq(WENO_EPS + sq(up - u0));
    double am = 1.0 / sq(WENO_EPS + sq(u0 - um));
    double w = 0.5 * (u0 + up);
    double v = 0.5 * (3.0 * u0 - um);
    return (2.0 * ap * w + am * v) / (2.0 * ap + am);
}

/* u^+_{i-1/2} from u_{i-1}, u_i, u_{i+1} */
static double weno_plus(double um, double u0, double up)
{
    double ap = 1.0 / sq(WENO_EPS + sq(up - u0));
    double am = 1.0 / sq(WENO_EPS + sq(u0 - um));
    double w = 0.5 * (3.0 * u0 - up);
    double v = 0.5 * (u0 + um);
    return (ap * w + 2.0 * am * v) / (ap + 2.0 * am);
}

double orc_weno_face(double um, double u0, double up, int side)
{
    return side ? weno_plus(um, u0, up) : weno_minus(um, u0, up);
}

/* Rusanov flux (Equ:LFFlux) at every face i+1/2 along d from the WENO
 * states; a face state with rho <= 0 or p <= 0 falls back to its cell's
 * value (the same fall-back as the LF scheme). */
static void weno_faces(const orc_params *p, const geo *G, const double *u, int d, double ch,
                       double *fh, long *cnt)
{
    int nv = orc_nvar(p);
    long P = G->P, s = G->s[d];
    int lo[3] = {0, 0, 0}, hi[3] = {G->n[0], G->n[1], G->n[2]};
    lo[d] = -1;
    hi[d] = G->n[d];
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(G, x, y, z), cn = c + s;
                double L[NVMAX], R[NVMAX];
                for (int k = 0; k < nv; k++) {
                    const double *q = u + k * P;
                    L[k] = weno_minus(q[c - s], q[c], q[cn]);
                    R[k] = weno_plus(q[c], q[cn], q[cn + s]);
                }
                if (!admissible(p, L)) {
                    load(u, P, nv, c, L);
                    cnt[1]++;
                }
                if (!admissible(p, R)) {
                    load(u, P, nv, cn, R);
                    cnt[1]++;
                }
                double fc[NVMAX];
                orc_face_flux(p, L, R, d, ch, fc);
                for (int k = 0; k < nv; k++)
                    fh[k * P + c] = fc[k];
            }
}

/* MMC (Sec. 3.1): Lax-Friedrichs splitting f+- = (f +- alpha u)/2 with the
 * global alpha (c_h on the GLM pair), predictor with h = f+_i + f-_{i+1},
 * and the flux-limited correction with g+ and g- built from u~. */
static void mmc_fluxes(const orc_params *p, const geo *G, const double *u,
                       const double dtdx[3], const orc_dtrec *dt, double *fh[3])
{
    int nv = orc_nvar(p), nd = G->nd;
    long P = G->P;
    double *fp[3], *fm[3], *ftp[3], *ftm[3];
    double *ut = calloc((size_t)nv * P, sizeof(double));
    for (int d = 0; d < nd; d++) {
        fp[d] = calloc((size_t)nv * P, sizeof(double));
        fm[d] = calloc((size_t)nv * P, sizeof(double));
        ftp[d] = calloc((size_t)nv * P, sizeof(double));
        ftm[d] = calloc((size_t)nv * P, sizeof(double));
    }
    /* split fluxes of u on the whole padded tile */
    for (int z = -G->g[2]; z < G->n[2] + G->g[2]; z++)
        for (int y = -G->g[1]; y < G->n[1] + G->g[1]; y++)
            for (int x = -G->g[0]; x < G->n[0] + G->g[0]; x++) {
                long c = at(G, x, y, z);
                double uc[NVMAX], F[NVMAX];
                load(u, P, nv, c, uc);
                for (int d = 0; d < nd; d++) {
                    orc_flux(p, uc, d, dt->ch, F);
                    for (int k = 0; k < nv; k++) {
                        double al = glm_component(p, k, d) ? dt->ch : dt->alpha;
                        fp[d][k * P + c] = 0.5 * (F[k] + al * uc[k]);
                        fm[d][k * P + c] = 0.5 * (F[k] - al * uc[k]);
                    }
                }
            }
    /* predictor u~ on E */
    int lo[3], hi[3];
    e_range(G, lo, hi);
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(G, x, y, z);
                for (int k = 0; k < nv; k++) {
                    double acc = 0.0;
                    for (int d = 0; d < nd; d++) {
                        long s = G->s[d];
                        double hp = fp[d][k * P + c] + fm[d][k * P + c + s];
                        double hm = fp[d][k * P + c - s] + fm[d][k * P + c];
                        acc += dtdx[d] * (hp - hm);
                    }
                    ut[k * P + c] = u[k * P + c] - acc;
                }
                double uc[NVMAX], F[NVMAX];
                load(ut, P, nv, c, uc);
                for (int d = 0; d < nd; d++) {
                    orc_flux(p, uc, d, dt->ch, F);
                    for (int k = 0; k < nv; k++) {
                        double al = glm_component(p, k, d) ? dt->ch : dt->alpha;
                        ftp[d][k * P + c] = 0.5 * (F[k] + al * uc[k]);
                        ftm[d][k * P + c] = 0.5 * (F[k] - al * uc[k]);
                    }
                }
            }
    /* limited fluxes on the faces bounding interior cells */
    for (int d = 0; d < nd; d++) {
        int flo[3] = {0, 0, 0}, fhi[3] = {G->n[0], G->n[1], G->n[2]};
        flo[d] = -1;
        fhi[d] = G->n[d];
        long s = G->s[d];
        for (int z = flo[2]; z < fhi[2]; z++)
            for (int y = flo[1]; y < fhi[1]; y++)
                for (int x = flo[0]; x < fhi[0]; x++) {
                    long c = at(G, x, y, z);
                    for (int k = 0; k < nv; k++) {
                        long o = (long)k * P;
                        double h = fp[d][o + c] + fm[d][o + c + s];
                        double gp_m = ftp[d][o + c] - fp[d][o + c - s];     /* g+ at i-1/2 */
                        double gp_p = ftp[d][o + c + s] - fp[d][o + c];     /* g+ at i+1/2 */
                        double gm_p = fm[d][o + c + s] - ftm[d][o + c];     /* g- at i+1/2 */
                        double gm_pp = fm[d][o + c + 2 * s] - ftm[d][o + c + s]; /* g- at i+3/2 */
                        fh[d][o + c] = h + 0.5 * (orc_limiter(p->limiter, gp_m, gp_p)
                                                  - orc_limiter(p->limiter, gm_pp, gm_p));
                    }
                }
    }
    free(ut);
    for (int d = 0; d < nd; d++) {
        free(fp[d]);
        free(fm[d]);
        free(ftp[d]);
        free(ftm[d]);
    }
}

/* central difference along d of array a (stride per variable implied) */
static double cdiff(const double *a, long c, long s, double inv2dx)
{
    return (a[c + s] - a[c - s]) * inv2dx;
}

void orc_eglm_source(const orc_params *p, const double dx[3], const double *u,
                     const int n_in[3], double *out)
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p);
    long P = G.P;
    memset(out, 0, sizeof(double) * nv * G.I);
    if (p->physics != ORC_MHD)
        return;
    double inv2dx[3];
    for (int d = 0; d < G.nd; d++)
        inv2dx[d] = 0.5 / dx[d];
    for (int z = 0; z < G.n[2]; z++)
        for (int y = 0; y < G.n[1]; y++)
            for (int x = 0; x < G.n[0]; x++) {
                long c = at(&G, x, y, z), ic = interior_index(&G, x, y, z);
                double divb = 0.0, bgp = 0.0;
                for (int d = 0; d < G.nd; d++)
                    divb += cdiff(u + (BX + d) * P, c, G.s[d], inv2dx[d]);
                for (int d = 0; d < G.nd; d++)
                    bgp += u[(BX + d) * P + c] * cdiff(u + PSI * P, c, G.s[d], inv2dx[d]);
                for (int j = 0; j < 3; j++)
                    out[(MX + j) * G.I + ic] = -(divb * u[(BX + j) * P + c]);
                out[EN * G.I + ic] = -bgp;
            }
}

void orc_resistive(const orc_params *p, const double dx[3], const double *u,
                   const int n_in[3], double *out)
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p), nd = G.nd;
    long P = G.P;
    memset(out, 0, sizeof(double) * nv * G.I);
    if (p->physics != ORC_MHD)
        return;
    double h[3];
    for (int d = 0; d < nd; d++)
        h[d] = 0.5 / dx[d];
    const double *Bx = u + BX * P, *By = u + BY * P, *Bz = u + BZ * P;
    double *J = calloc((size_t)3 * P, sizeof(double));  /* eta J */
    double *Q = calloc((size_t)3 * P, sizeof(double));  /* eta (J x B) rows of R_e */
    int lo[3], hi[3];
    e_range(&G, lo, hi);
    double eta = p->eta;
    /* J = curl B by central differences; z-derivatives vanish in 2-D */
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(&G, x, y, z);
                double jx, jy, jz;
                if (nd == 3) {
                    jx = cdiff(Bz, c, G.s[1], h[1]) - cdiff(By, c, G.s[2], h[2]);
                    jy = cdiff(Bx, c, G.s[2], h[2]) - cdiff(Bz, c, G.s[0], h[0]);
                } else {
                    jx = cdiff(Bz, c, G.s[1], h[1]);
                    jy = -cdiff(Bz, c, G.s[0], h[0]);
                }
                jz = cdiff(By, c, G.s[0], h[0]) - cdiff(Bx, c, G.s[1], h[1]);
                J[0 * P + c] = eta * jx;
                J[1 * P + c] = eta * jy;
                J[2 * P + c] = eta * jz;
                Q[0 * P + c] = eta * (jz * By[c] - jy * Bz[c]);
                Q[1 * P + c] = eta * (jx * Bz[c] - jz * Bx[c]);
                Q[2 * P + c] = eta * (jy * Bx[c] - jx * By[c]);
            }
    for (int z = 0; z < G.n[2]; z++)
        for (int y = 0; y < G.n[1]; y++)
            for (int x = 0; x < G.n[0]; x++) {
                long c = at(&G, x, y, z), ic = interior_index(&G, x, y, z);
                const double *Jx = J, *Jy = J + P, *Jz = J + 2 * P;
                double rx, ry, rz, re;
                if (nd == 3) {
                    rx = cdiff(Jy, c, G.s[2], h[2]) - cdiff(Jz, c, G.s[1], h[1]);
                    ry = cdiff(Jz, c, G.s[0], h[0]) - cdiff(Jx, c, G.s[2], h[2]);
                } else {
                    rx = -cdiff(Jz, c, G.s[1], h[1]);
                    ry = cdiff(Jz, c, G.s[0], h[0]);
                }
                rz = cdiff(Jx, c, G.s[1], h[1]) - cdiff(Jy, c, G.s[0], h[0]);
                re = cdiff(Q, c, G.s[0], h[0]) + cdiff(Q + P, c, G.s[1], h[1]);
                if (nd == 3)
                    re = re + cdiff(Q + 2 * P, c, G.s[2], h[2]);
                out[BX * G.I + ic] = rx;
                out[BY * G.I + ic] = ry;
                out[BZ * G.I + ic] = rz;
                out[EN * G.I + ic] = re;
            }
    free(J);
    free(Q);
}

void orc_step_tile(const orc_params *p, const double dx[3], const double *u,
                   const int n_in[3], const orc_dtrec *dt, double *unew,
                   double *ff, long *cnt)
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p), nd = G.nd;
    long P = G.P;
    long dummy[4] = {0, 0, 0, 0};
    if (!cnt)
        cnt = dummy;
    double dtdx[3] = {0, 0, 0}, hdt[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) {
        dtdx[d] = dt->dt / dx[d];
        hdt[d] = 0.5 * dtdx[d];
    }
    double *fh[3] = {NULL, NULL, NULL};
    for (int d = 0; d < nd; d++)
        fh[d] = calloc((size_t)nv * P, sizeof(double));

    if (p->scheme == ORC_LF) {
        double *ut = calloc((size_t)nv * P, sizeof(double));
        double *sl = calloc((size_t)nd * nv * P, sizeof(double));
        lf_predict(p, &G, u, hdt, dt->ch, ut, sl, cnt);
        for (int d = 0; d < nd; d++)
            lf_faces(p, &G, ut, sl, d, dt->ch, fh[d], cnt, NULL);
        free(ut);
        free(sl);
    } else if (p->scheme == ORC_WENO) {
        /* one Euler stage: the fluxes of every direction from the same u */
        for (int d = 0; d < nd; d++)
            weno_faces(p, &G, u, d, dt->ch, fh[d], cnt);
    } else {
        mmc_fluxes(p, &G, u, dtdx, dt, fh);
    }

    double *src = NULL, *res = NULL;
    if (p->physics == ORC_MHD && p->eglm_sources) {
        src = malloc(sizeof(double) * nv * G.I);
        orc_eglm_source(p, dx, u, n_in, src);
    }
    if (p->physics == ORC_MHD && p->eta > 0.0) {
        res = malloc(sizeof(double) * nv * G.I);
        orc_resistive(p, dx, u, n_in, res);
    }

    /* conservative update (Equ:basic), all directions together */
    for (int z = 0; z < G.n[2]; z++)
        for (int y = 0; y < G.n[1]; y++)
            for (int x = 0; x < G.n[0]; x++) {
                long c = at(&G, x, y, z), ic = interior_index(&G, x, y, z);
                double v[NVMAX];
                for (int k = 0; k < nv; k++) {
                    double acc = 0.0;
                    for (int d = 0; d < nd; d++)
                        acc += dtdx[d] * (fh[d][k * P + c] - fh[d][k * P + c - G.s[d]]);
                    v[k] = u[k * P + c] - acc;
                }
                if (p->physics == ORC_MHD) {
                    if (src) {
                        for (int j = 0; j < 3; j++)
                            v[MX + j] = v[MX + j] + dt->dt * src[(MX + j) * G.I + ic];
                        v[EN] = v[EN] + dt->dt * src[EN * G.I + ic];
                    }
                    if (res) {
                        for (int j = 0; j < 3; j++)
                            v[BX + j] = v[BX + j] + dt->dt * res[(BX + j) * G.I + ic];
                        v[EN] = v[EN] + dt->dt * res[EN * G.I + ic];
                    }
                    /* MHD-5 damping term integrated exactly over dt (for WENO
                     * once per step, after the second Runge-Kutta stage) */
                    if (p->scheme != ORC_WENO)
                        v[PSI] = v[PSI] * dt->damp;
                }
                for (int k = 0; k < nv; k++)
                    unew[k * G.I + ic] = v[k];
            }

    /* fluxes of the block faces, for refluxing */
    if (ff) {
        long off = 0;
        for (int d = 0; d < nd; d++) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            long T = (long)G.n[t1] * G.n[t2];
            for (int side = 0; side < 2; side++) {
                int cd = side ? G.n[d] - 1 : -1;
                for (int k = 0; k < nv; k++)
                    for (int b = 0; b < G.n[t2]; b++)
                        for (int a = 0; a < G.n[t1]; a++) {
                            int xyz[3];
                            xyz[d] = cd;
                            xyz[t1] = a;
                            xyz[t2] = b;
                            ff[off + k * T + (long)b * G.n[t1] + a] =
                                fh[d][k * P + at(&G, xyz[0], xyz[1], xyz[2])];
                        }
                off += (long)nv * T;
            }
        }
    }
    free(src);
    free(res);
    for (int d = 0; d < nd; d++)
        free(fh[d]);
}

/* The intermediate states of the LF scheme on one padded tile (for the
 * tests of the positivity fall-back, Sec. 3.2): the predicted state u~ and
 * the limited slopes on the whole padded tile (zero outside the region the
 * predictor covers), and, per dimension, the left and right states that the
 * face flux of each face receives after the fall-back, face c+1/2 stored at
 * cell c.  Layouts: ut[nvar][P], sl[ndim][nvar][P], lr[ndim][2][nvar][P]. */
void orc_lf_states(const orc_params *p, const double dx[3], const double *u,
                   const int n_in[3], const orc_dtrec *dt, double *ut, double *sl,
                   double *lr, long *cnt)
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p), nd = G.nd;
    long P = G.P;
    double hdt[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++)
        hdt[d] = 0.5 * dt->dt / dx[d];
    memset(ut, 0, sizeof(double) * nv * P);
    memset(sl, 0, sizeof(double) * nd * nv * P);
    memset(lr, 0, sizeof(double) * nd * 2 * nv * P);
    double *fh = calloc((size_t)nv * P, sizeof(double));
    lf_predict(p, &G, u, hdt, dt->ch, ut, sl, cnt);
    for (int d = 0; d < nd; d++)
        lf_faces(p, &G, ut, sl, d, dt->ch, fh, cnt, lr + (size_t)d * 2 * nv * P);
    free(fh);
}

double orc_tile_maxspeed(const orc_params *p, const double *u, const int n_in[3])
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p);
    double m = 0.0;
    for (int z = 0; z < G.n[2]; z++)
        for (int y = 0; y < G.n[1]; y++)
            for (int x = 0; x < G.n[0]; x++) {
                double uc[NVMAX];
                load(u, G.P, nv, at(&G, x, y, z), uc);
                for (int d = 0; d < G.nd; d++) {
                    double s = orc_speed(p, uc, d);
                    if (s > m)
                        m = s;
                }
            }
    return m;
}

/* dt = c_cfl min(dx)/(n_dim alpha_g) (Sec. 3.7); resistive limit by analogy
 * with the conduction step of Sec. 3.4; c_h and the psi factor per GLM mode (Sec. 2).
 * Conduction (Sec. 3.4): the sub-step limit dt_c = c_cfl min(dx)^2 /
 * (n_dim max(kappa T/p)) with kmax = max(kappa T/p); the step is capped at
 * cond_max_sub dt_c, and split into nsub = ceil(dt/dt_c) equal sub-steps. */
void orc_make_dtrec(const orc_params *p, double alpha, double dxmin, double kmax, orc_dtrec *o)
{
    int nd = p->ndim;
    double dt = p->cfl * dxmin / (nd * alpha);
    if (p->physics == ORC_MHD && p->eta > 0.0) {
        double dr = p->cfl * dxmin * dxmin / (nd * p->eta);
        if (dr < dt)
            dt = dr;
    }
    o->dt_sub = 0.0;
    o->nsub = 0;
    o->reserved = 0;
    if (p->physics == ORC_MHD && p->cond_mode != ORC_COND_OFF && kmax > 0.0) {
        double dtc = p->cfl * dxmin * dxmin / (nd * kmax);
        double cap = p->cond_max_sub * dtc;
        if (cap < dt)
            dt = cap;
        double ns = ceil(dt / dtc);
        int nsub = ns < 1.0 ? 1 : (ns > p->cond_max_sub ? p->cond_max_sub : (int)ns);
        o->nsub = nsub;
        o->dt_sub = dt / nsub;
    }
    o->dt = dt;
    o->alpha = alpha;
    if (p->glm_mode == ORC_GLM_PAPER) {
        o->ch = p->cfl * dxmin / dt;
        o->damp = p->cd;
    } else {
        o->ch = alpha;
        o->damp = exp(-dt * o->ch / p->cr);
    }
}

/* ------------------------------------------------------------------ */
/* thermal conduction sub-step (Sec. 3.4)                              */
/* ------------------------------------------------------------------ */
/* temperature T = p / rho (code units) */
static double temperature(const orc_params *p, const double *u, long P, long c)
{
    double uc[NVMAX];
    load(u, P, 9, c, uc);
    return orc_pressure(p, uc) / uc[RHO];
}

/* kappa = kappa0 T^n for n a multiple of 1/2: whole powers by repeated
 * multiplication, then one square root for the half */
static double kappa_of(const orc_params *p, double T)
{
    int k = (int)lround(2.0 * p->kappa_exp);
    double q = 1.0;
    for (int i = 0; i < k / 2; i++)
        q = q * T;
    if (k & 1)
        q = q * sqrt(T);
    return p->kappa0 * q;
}

double orc_tile_cond_rate(const orc_params *p, const double *u, const int n_in[3])
{
    if (p->physics != ORC_MHD || p->cond_mode == ORC_COND_OFF)
        return 0.0;
    geo G = mkgeo(p->ndim, n_in);
    double m = 0.0;
    for (int z = 0; z < G.n[2]; z++)
        for (int y = 0; y < G.n[1]; y++)
            for (int x = 0; x < G.n[0]; x++) {
                long c = at(&G, x, y, z);
                double T = temperature(p, u, G.P, c);
                /* kappa T / p = kappa / rho */
                double r = kappa_of(p, T) / u[RHO * G.P + c];
                if (r > m)
                    m = r;
            }
    return m;
}

/* energy flux along +d across the face between the cells c and cn = c + s_d,
 * F = -(kappa grad T)_d, in the conservative form de/dt + div F = 0 that the
 * reflux of Sec. 4.3 corrects.
 * Isotropic (the scheme of Sec. 3.4): -sqrt(kappa_c kappa_cn)(T_cn - T_c)/dx_d.
 * Along the field (the form of the conduction test, Sec. 5): the same face
 * kappa times b_d (b . grad T) with b = B_f/|B_f|, B_f the mean of the two
 * cells' fields; grad T at the face: the difference across it along d and,
 * along each other dimension e, the mean of the two cells' central
 * differences; zero where B_f = 0. */
static double cond_face(const orc_params *p, const geo *G, const double *Tc, const double *Kc,
                        const double *u, long c, int d, const double dx[3])
{
    long cn = c + G->s[d];
    double kf = sqrt(Kc[c] * Kc[cn]);
    double gd = (Tc[cn] - Tc[c]) / dx[d];
    if (p->cond_mode == ORC_COND_ISO)
        return -(kf * gd);
    double Bf[3], bb = 0.0;
    for (int j = 0; j < 3; j++) {
        Bf[j] = 0.5 * (u[(BX + j) * G->P + c] + u[(BX + j) * G->P + cn]);
        bb += Bf[j] * Bf[j];
    }
    if (!(bb > 0.0))
        return 0.0;
    double bg = 0.0;
    for (int e = 0; e < 3; e++) {
        double g;
        if (e == d) {
            g = gd;
        } else if (e < G->nd) {
            long s = G->s[e];
            g = ((Tc[c + s] - Tc[c - s]) + (Tc[cn + s] - Tc[cn - s])) / (4.0 * dx[e]);
        } else {
            g = 0.0;
        }
        bg += Bf[e] * g;
    }
    return -(kf * Bf[d] * bg / bb);
}

void orc_conduct_tile(const orc_params *p, const double dx[3], const double *u,
                      const int n_in[3], double dt_sub, double *enew, double *ff)
{
    geo G = mkgeo(p->ndim, n_in);
    int nd = G.nd, nv = orc_nvar(p);
    double *Tc = calloc(G.P, sizeof(double)), *Kc = calloc(G.P, sizeof(double));
    /* T and kappa on the interior and the first ghost ring (edges and
     * corners included) */
    int lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        lo[d] = d < nd ? -1 : 0;
        hi[d] = d < nd ? G.n[d] + 1 : 1;
    }
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(&G, x, y, z);
                Tc[c] = temperature(p, u, G.P, c);
                Kc[c] = kappa_of(p, Tc[c]);
            }
    for (int z = 0; z < G.n[2]; z++)
        for (int y = 0; y < G.n[1]; y++)
            for (int x = 0; x < G.n[0]; x++) {
                long c = at(&G, x, y, z);
                double acc = 0.0;
                for (int d = 0; d < nd; d++) {
                    double fp = cond_face(p, &G, Tc, Kc, u, c, d, dx);
                    double fm = cond_face(p, &G, Tc, Kc, u, c - G.s[d], d, dx);
                    acc += (fp - fm) / dx[d];
                }
                enew[interior_index(&G, x, y, z)] = u[EN * G.P + c] - dt_sub * acc;
            }
    if (ff) {
        long off = 0;
        for (int d = 0; d < nd; d++) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            long T = (long)G.n[t1] * G.n[t2];
            for (int side = 0; side < 2; side++) {
                int cd = side ? G.n[d] - 1 : -1;
                for (int k = 0; k < nv; k++)
                    for (int b = 0; b < G.n[t2]; b++)
                        for (int a = 0; a < G.n[t1]; a++) {
                            int xyz[3];
                            xyz[d] = cd;
                            xyz[t1] = a;
                            xyz[t2] = b;
                            double q = 0.0;
                            if (k == EN)
                                q = cond_face(p, &G, Tc, Kc, u, at(&G, xyz[0], xyz[1], xyz[2]), d, dx);
                            ff[off + k * T + (long)b * G.n[t1] + a] = q;
                        }
                off += (long)nv * T;
            }
        }
    }
    free(Tc);
    free(Kc);
}

/* ------------------------------------------------------------------ */
/* monolithic uniform grid                                             */
/* ------------------------------------------------------------------ */
static int map_index(int G, int N, int bclo, int bchi)
{
    if (G < 0) {
        if (bclo == ORC_BC_PERIODIC)
            return ((G % N) + N) % N;
        return 0;
    }
    if (G >= N) {
        if (bchi == ORC_BC_PERIODIC)
            return G % N;
        return N - 1;
    }
    return G;
}

void orc_grid_fill(const orc_params *p, double *u, const int n_in[3], const int bc[3][2])
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p);
    for (int z = -G.g[2]; z < G.n[2] + G.g[2]; z++)
        for (int y = -G.g[1]; y < G.n[1] + G.g[1]; y++)
            for (int x = -G.g[0]; x < G.n[0] + G.g[0]; x++) {
                int xyz[3] = {x, y, z}, src[3];
                int inside = 1;
                for (int d = 0; d < 3; d++) {
                    if (xyz[d] < 0 || xyz[d] >= G.n[d])
                        inside = 0;
                    src[d] = map_index(xyz[d], G.n[d], bc[d][0], bc[d][1]);
                }
                if (inside)
                    continue;
                long c = at(&G, x, y, z), s = at(&G, src[0], src[1], src[2]);
                for (int k = 0; k < nv; k++)
                    u[k * G.P + c] = u[k * G.P + s];
            }
}

void orc_grid_run(const orc_params *p, const double dx[3], double *u, const int n_in[3],
                  const int bc[3][2], int nsteps, double *dt_trace, long *cnt)
{
    geo G = mkgeo(p->ndim, n_in);
    int nv = orc_nvar(p);
    double *unew = malloc(sizeof(double) * nv * G.I);
    double dxmin = dx[0];
    for (int d = 1; d < G.nd; d++)
        if (dx[d] < dxmin)
            dxmin = dx[d];
    for (int it = 0; it < nsteps; it++) {
        orc_grid_fill(p, u, n_in, bc);
        orc_dtrec r;
        orc_make_dtrec(p, orc_tile_maxspeed(p, u, n_in), dxmin, orc_tile_cond_rate(p, u, n_in), &r);
        if (dt_trace)
            dt_trace[it] = r.dt;
        orc_step_tile(p, dx, u, n_in, &r, unew, NULL, cnt);
        if (p->scheme == ORC_WENO) {
            /* TVD Runge-Kutta 2: u1 = u + dt L(u); u = (u + u1 + dt L(u1)) / 2 */
            double *u1 = malloc(sizeof(double) * nv * G.P);
            memcpy(u1, u, sizeof(double) * nv * G.P);
            for (int z = 0; z < G.n[2]; z++)
                for (int y = 0; y < G.n[1]; y++)
                    for (int x = 0; x < G.n[0]; x++)
                        for (int k = 0; k < nv; k++)
                            u1[k * G.P + at(&G, x, y, z)] =
                                unew[k * G.I + interior_index(&G, x, y, z)];
            orc_grid_fill(p, u1, n_in, bc);
            orc_step_tile(p, dx, u1, n_in, &r, unew, NULL, cnt);
            free(u1);
            for (int z = 0; z < G.n[2]; z++)
                for (int y = 0; y < G.n[1]; y++)
                    for (int x = 0; x < G.n[0]; x++) {
                        long c = at(&G, x, y, z), ic = interior_index(&G, x, y, z);
                        for (int k = 0; k < nv; k++)
                            u[k * G.P + c] = 0.5 * (u[k * G.P + c] + unew[k * G.I + ic]);
                        if (p->physics == ORC_MHD)
                            u[PSI * G.P + c] = u[PSI * G.P + c] * r.damp;
                    }
        } else {
            for (int z = 0; z < G.n[2]; z++)
                for (int y = 0; y < G.n[1]; y++)
                    for (int x = 0; x < G.n[0]; x++)
                        for (int k = 0; k < nv; k++)
                            u[k * G.P + at(&G, x, y, z)] =
                                unew[k * G.I + interior_index(&G, x, y, z)];
        }
        /* conduction subcycle (Sec. 3.4): only the energy changes; each
         * sub-step sees boundaries refreshed from the previous one */
        for (int i = 0; i < r.nsub; i++) {
            orc_grid_fill(p, u, n_in, bc);
            orc_conduct_tile(p, dx, u, n_in, r.dt_sub, unew, NULL);
            for (int z = 0; z < G.n[2]; z++)
                for (int y = 0; y < G.n[1]; y++)
                    for (int x = 0; x < G.n[0]; x++)
                        u[EN * G.P + at(&G, x, y, z)] = unew[interior_index(&G, x, y, z)];
        }
    }
    orc_grid_fill(p, u, n_in, bc);
    free(unew);
}

/* ------------------------------------------------------------------ */
/* block tree                                                          */
/* ------------------------------------------------------------------ */
struct orc_amr {
    orc_params p;
    int n, nv, nd, nsims, nb, lmax;
    orc_sim *sims;
    orc_key *keys;
    int *order;   /* block indices sorted by key */
    int *parent;  /* -1 for base blocks */
    int *haskids;
    geo G;
    long T;       /* cells of one block face */
    double *U;    /* [nb][nv][P] */
    double *ff;   /* [nb][2 nd][nv][T] */
    long cnt[4];
};

static const orc_key *g_sort_keys;

static int key_cmp(const orc_key *a, const orc_key *b)
{
    if (a->sim != b->sim) return a->sim < b->sim ? -1 : 1;
    if (a->level != b->level) return a->level < b->level ? -1 : 1;
    if (a->iz != b->iz) return a->iz < b->iz ? -1 : 1;
    if (a->iy != b->iy) return a->iy < b->iy ? -1 : 1;
    if (a->ix != b->ix) return a->ix < b->ix ? -1 : 1;
    return 0;
}

static int idx_cmp(const void *a, const void *b)
{
    return key_cmp(&g_sort_keys[*(const int *)a], &g_sort_keys[*(const int *)b]);
}

static int lookup(const orc_amr *A, int sim, int level, int ix, int iy, int iz)
{
    orc_key k = {sim, level, ix, iy, iz};
    int lo = 0, hi = A->nb - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        int c = key_cmp(&A->keys[A->order[mid]], &k);
        if (c == 0)
            return A->order[mid];
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

static int cells_at_level(const orc_amr *A, int sim, int d, int level)
{
    return A->sims[sim].nbase[d] * A->n << (level - 1);
}

static void block_dx(const orc_amr *A, int b, double dx[3])
{
    const orc_key *k = &A->keys[b];
    for (int d = 0; d < 3; d++) {
        if (d < A->nd) {
            const orc_sim *s = &A->sims[k->sim];
            dx[d] = (s->hi[d] - s->lo[d]) / cells_at_level(A, k->sim, d, k->level);
        } else {
            dx[d] = 1.0;
        }
    }
}

static void key_coords(const orc_key *k, int c[3])
{
    c[0] = k->ix;
    c[1] = k->iy;
    c[2] = k->iz;
}

orc_amr *orc_amr_new(const orc_params *p, int n, int nsims, const orc_sim *sims,
                     int nb, const orc_key *keys)
{
    orc_amr *A = calloc(1, sizeof(orc_amr));
    A->p = *p;
    A->n = n;
    A->nv = orc_nvar(p);
    A->nd = p->ndim;
    A->nsims = nsims;
    A->nb = nb;
    A->sims = malloc(sizeof(orc_sim) * nsims);
    memcpy(A->sims, sims, sizeof(orc_sim) * nsims);
    A->keys = malloc(sizeof(orc_key) * nb);
    memcpy(A->keys, keys, sizeof(orc_key) * nb);
    A->order = malloc(sizeof(int) * nb);
    for (int i = 0; i < nb; i++)
        A->order[i] = i;
    g_sort_keys = A->keys;
    qsort(A->order, nb, sizeof(int), idx_cmp);
    int nn[3] = {n, n, n};
    A->G = mkgeo(A->nd, nn);
    A->T = (A->nd == 3) ? (long)n * n : n;
    A->parent = malloc(sizeof(int) * nb);
    A->haskids = calloc(nb, sizeof(int));
    A->lmax = 1;
    for (int b = 0; b < nb; b++) {
        const orc_key *k = &A->keys[b];
        if (k->level > A->lmax)
            A->lmax = k->level;
        A->parent[b] = -1;
        if (k->level > 1) {
            int pb = lookup(A, k->sim, k->level - 1, k->ix >> 1, k->iy >> 1, k->iz >> 1);
            A->parent[b] = pb;
            if (pb >= 0)
                A->haskids[pb] = 1;
        }
    }
    A->U = calloc((size_t)nb * A->nv * A->G.P, sizeof(double));
    A->ff = calloc((size_t)nb * 2 * A->nd * A->nv * A->T, sizeof(double));
    return A;
}

void orc_amr_free(orc_amr *A)
{
    if (!A)
        return;
    free(A->sims);
    free(A->keys);
    free(A->order);
    free(A->parent);
    free(A->haskids);
    free(A->U);
    free(A->ff);
    free(A);
}

double *orc_amr_state(orc_amr *A) { return A->U; }
int orc_amr_tile_cells(const orc_amr *A) { return (int)A->G.P; }
int orc_amr_is_leaf(const orc_amr *A, int b) { return !A->haskids[b]; }

void orc_amr_counters(const orc_amr *A, long out[4])
{
    for (int i = 0; i < 4; i++)
        out[i] = A->cnt[i];
}

static double *tile(orc_amr *A, int b) { return A->U + (size_t)b * A->nv * A->G.P; }

void orc_amr_prim_to_cons(orc_amr *A)
{
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int b = 0; b < A->nb; b++)
        orc_prim_to_cons(&A->p, tile(A, b), A->G.P);
}

/* conservative minmod-limited linear interpolation from the parent's padded
 * tile (Sec. 4.3, step 6) at fine padded cell (x,y,z) of block b */
static void prolong_cell(orc_amr *A, int b, int x, int y, int z, double *out)
{
    const orc_key *k = &A->keys[b];
    int pb = A->parent[b];
    const double *pu = tile(A, pb);
    int kc[3], loc[3] = {x, y, z}, ci[3], off[3];
    key_coords(k, kc);
    for (int d = 0; d < 3; d++) {
        if (d < A->nd) {
            int f = (kc[d] & 1) * A->n + loc[d];  /* fine index relative to the parent origin */
            int c = (f >= 0) ? f / 2 : -((-f + 1) / 2);
            ci[d] = c;
            off[d] = f - 2 * c;
        } else {
            ci[d] = 0;
            off[d] = 0;
        }
    }
    long c = at(&A->G, ci[0], ci[1], ci[2]);
    for (int kv = 0; kv < A->nv; kv++) {
        const double *q = pu + (long)kv * A->G.P;
        double v = q[c];
        for (int d = 0; d < A->nd; d++) {
            long s = A->G.s[d];
            double slope = orc_limiter(ORC_MINMOD, q[c + s] - q[c], q[c] - q[c - s]);
            double w = off[d] ? 0.25 : -0.25;
            v = v + slope * w;
        }
        out[kv] = v;
    }
}

/* the same-level source of ghost cell (x, y, z) of block b (Sec. 4.3 steps
 * 3-5): the global index at b's level after periodic wrap or outflow
 * clamping, split into the block that holds it (-1 if no block of b's level
 * does) and the cell inside that block (lc) */
static int ghost_source(const orc_amr *A, int b, int x, int y, int z, int lc[3])
{
    const orc_key *k = &A->keys[b];
    const orc_sim *S = &A->sims[k->sim];
    int kc[3], loc[3] = {x, y, z}, bc3[3] = {0, 0, 0};
    key_coords(k, kc);
    lc[0] = lc[1] = lc[2] = 0;
    for (int d = 0; d < A->nd; d++) {
        int N = cells_at_level(A, k->sim, d, k->level);
        int g = map_index(kc[d] * A->n + loc[d], N, S->bc[d][0], S->bc[d][1]);
        bc3[d] = g / A->n;
        lc[d] = g - bc3[d] * A->n;
    }
    return lookup(A, k->sim, k->level, bc3[0], bc3[1], bc3[2]);
}

static int is_interior(const geo *G, int x, int y, int z)
{
    return x >= 0 && x < G->n[0] && y >= 0 && y < G->n[1] && z >= 0 && z < G->n[2];
}

/* ghost cells of every block: copies of the same-level source's interior
 * cells, then, level by level from coarse to fine (so that a parent's own
 * prolonged ghosts are in place), prolongation from the parent where no
 * same-level source exists */
void orc_amr_fill(orc_amr *A)
{
    geo *G = &A->G;
    int nv = A->nv;
#pragma omp parallel for schedule(dynamic, 8) num_threads(g_threads)
    for (int b = 0; b < A->nb; b++) {
        double *u = tile(A, b);
        for (int z = -G->g[2]; z < G->n[2] + G->g[2]; z++)
            for (int y = -G->g[1]; y < G->n[1] + G->g[1]; y++)
                for (int x = -G->g[0]; x < G->n[0] + G->g[0]; x++) {
                    if (is_interior(G, x, y, z))
                        continue;
                    int lc[3];
                    int src = ghost_source(A, b, x, y, z, lc);
                    if (src < 0)
                        continue;
                    const double *su = tile(A, src);
                    long c = at(G, x, y, z), sc = at(G, lc[0], lc[1], lc[2]);
                    for (int kv = 0; kv < nv; kv++)
                        u[kv * G->P + c] = su[kv * G->P + sc];
                }
    }
    for (int lv = 2; lv <= A->lmax; lv++) {
#pragma omp parallel for schedule(dynamic, 8) num_threads(g_threads)
        for (int b = 0; b < A->nb; b++) {
            if (A->keys[b].level != lv)
                continue;
            double *u = tile(A, b);
            for (int z = -G->g[2]; z < G->n[2] + G->g[2]; z++)
                for (int y = -G->g[1]; y < G->n[1] + G->g[1]; y++)
                    for (int x = -G->g[0]; x < G->n[0] + G->g[0]; x++) {
                        if (is_interior(G, x, y, z))
                            continue;
                        int lc[3];
                        if (ghost_source(A, b, x, y, z, lc) >= 0)
                            continue;
                        double v[NVMAX];
                        prolong_cell(A, b, x, y, z, v);
                        long c = at(G, x, y, z);
                        for (int kv = 0; kv < nv; kv++)
                            u[kv * G->P + c] = v[kv];
                    }
        }
    }
}

void orc_amr_prolong_block(orc_amr *A, int b)
{
    geo *G = &A->G;
    double *u = tile(A, b);
    for (int z = 0; z < G->n[2]; z++)
        for (int y = 0; y < G->n[1]; y++)
            for (int x = 0; x < G->n[0]; x++) {
                double v[NVMAX];
                prolong_cell(A, b, x, y, z, v);
                for (int kv = 0; kv < A->nv; kv++)
                    u[kv * G->P + at(G, x, y, z)] = v[kv];
            }
}

/* parent = average of its 2^d children's cells (Sec. 4.2, 4.3 step 1),
 * summed in pairs so that equal inputs give the same value back */
void orc_amr_restrict(orc_amr *A)
{
    geo *G = &A->G;
    int n = A->n, nd = A->nd;
    for (int lv = A->lmax - 1; lv >= 1; lv--) {
#pragma omp parallel for schedule(dynamic, 8) num_threads(g_threads)
        for (int b = 0; b < A->nb; b++) {
            const orc_key *k = &A->keys[b];
            if (k->level != lv || !A->haskids[b])
                continue;
            double *u = tile(A, b);
            int kc[3];
            key_coords(k, kc);
            for (int z = 0; z < G->n[2]; z++)
                for (int y = 0; y < G->n[1]; y++)
                    for (int x = 0; x < G->n[0]; x++) {
                        int loc[3] = {x, y, z};
                        double f[8][NVMAX];
                        int nf = 1 << nd;
                        for (int o = 0; o < nf; o++) {
                            int cc[3] = {0, 0, 0}, lc[3] = {0, 0, 0};
                            for (int d = 0; d < nd; d++) {
                                int fg = 2 * (kc[d] * n + loc[d]) + ((o >> d) & 1);
                                cc[d] = fg / n;
                                lc[d] = fg - cc[d] * n;
                            }
                            int cb = lookup(A, k->sim, lv + 1, cc[0], cc[1], cc[2]);
                            load(tile(A, cb), G->P, A->nv, at(G, lc[0], lc[1], lc[2]), f[o]);
                        }
                        long c = at(G, x, y, z);
                        for (int kv = 0; kv < A->nv; kv++) {
                            double v;
                            if (nd == 2)
                                v = ((f[0][kv] + f[1][kv]) + (f[2][kv] + f[3][kv])) * 0.25;
                            else
                                v = (((f[0][kv] + f[1][kv]) + (f[2][kv] + f[3][kv]))
                                     + ((f[4][kv] + f[5][kv]) + (f[6][kv] + f[7][kv]))) * 0.125;
                            u[kv * G->P + c] = v;
                        }
                    }
        }
    }
}

static void sim_dxmin(const orc_amr *A, int sim, double *dxmin)
{
    double m = 0.0;
    int first = 1;
    for (int b = 0; b < A->nb; b++) {
        if (A->keys[b].sim != sim || A->haskids[b])
            continue;
        double dx[3];
        block_dx(A, b, dx);
        for (int d = 0; d < A->nd; d++)
            if (first || dx[d] < m) {
                m = dx[d];
                first = 0;
            }
    }
    *dxmin = m;
}

void orc_amr_cfl(orc_amr *A, orc_dtrec *out)
{
    int nn[3] = {A->n, A->n, A->n};
    for (int s = 0; s < A->nsims; s++) {
        double alpha = 0.0, dxmin;
#pragma omp parallel for schedule(dynamic, 8) reduction(max : alpha) num_threads(g_threads)
        for (int b = 0; b < A->nb; b++) {
            if (A->keys[b].sim != s || A->haskids[b])
                continue;
            double m = orc_tile_maxspeed(&A->p, tile(A, b), nn);
            if (m > alpha)
                alpha = m;
        }
        sim_dxmin(A, s, &dxmin);
        double kmax = 0.0;
#pragma omp parallel for schedule(dynamic, 8) reduction(max : kmax) num_threads(g_threads)
        for (int b = 0; b < A->nb; b++) {
            if (A->keys[b].sim != s || A->haskids[b])
                continue;
            double k = orc_tile_cond_rate(&A->p, tile(A, b), nn);
            if (k > kmax)
                kmax = k;
        }
        orc_make_dtrec(&A->p, alpha, dxmin, kmax, &out[s]);
    }
}

static void amr_weno_rk2(orc_amr *A, const orc_dtrec *dt);

static void add_counters(orc_amr *A, const long cnt[4])
{
    for (int i = 0; i < 4; i++) {
#pragma omp atomic
        A->cnt[i] += cnt[i];
    }
}

void orc_amr_step(orc_amr *A, const orc_dtrec *dt)
{
    if (A->p.scheme == ORC_WENO) {
        amr_weno_rk2(A, dt);
        return;
    }
    geo *G = &A->G;
    int nn[3] = {A->n, A->n, A->n};
    /* every block reads only its own padded tile, so blocks are independent */
#pragma omp parallel num_threads(g_threads)
    {
        double *unew = malloc(sizeof(double) * A->nv * G->I);
#pragma omp for schedule(dynamic, 4)
        for (int b = 0; b < A->nb; b++) {
            if (A->haskids[b])
                continue;
            double dx[3];
            block_dx(A, b, dx);
            double *u = tile(A, b);
            double *ff = A->ff + (size_t)b * 2 * A->nd * A->nv * A->T;
            long cnt[4] = {0, 0, 0, 0};
            orc_step_tile(&A->p, dx, u, nn, &dt[A->keys[b].sim], unew, ff, cnt);
            add_counters(A, cnt);
            for (int z = 0; z < G->n[2]; z++)
                for (int y = 0; y < G->n[1]; y++)
                    for (int x = 0; x < G->n[0]; x++)
                        for (int k = 0; k < A->nv; k++)
                            u[k * G->P + at(G, x, y, z)] = unew[k * G->I + interior_index(G, x, y, z)];
        }
        free(unew);
    }
}

/* WENO with TVD Runge-Kutta 2 on the tree: stage 1 on every leaf into a
 * second state, the boundary procedure (restriction, ghost exchange,
 * prolongation) on that state, stage 2 from it; psi damping once; the face
 * fluxes for reflux are the stage average (F + F1) / 2, which is the flux
 * the two stages apply in total. */
static void amr_weno_rk2(orc_amr *A, const orc_dtrec *dt)
{
    geo *G = &A->G;
    int nn[3] = {A->n, A->n, A->n};
    int nv = A->nv;
    size_t ntot = (size_t)A->nb * nv * G->P;
    size_t nff = (size_t)A->nb * 2 * A->nd * nv * A->T;
    double *U1 = malloc(sizeof(double) * ntot);
    double *ff1 = calloc(nff, sizeof(double));
    memcpy(U1, A->U, sizeof(double) * ntot);
#pragma omp parallel num_threads(g_threads)
    {
        double *unew = malloc(sizeof(double) * nv * G->I);
#pragma omp for schedule(dynamic, 4)
        for (int b = 0; b < A->nb; b++) {
            if (A->haskids[b])
                continue;
            double dx[3];
            block_dx(A, b, dx);
            long cnt[4] = {0, 0, 0, 0};
            orc_step_tile(&A->p, dx, tile(A, b), nn, &dt[A->keys[b].sim], unew,
                          ff1 + (size_t)b * 2 * A->nd * nv * A->T, cnt);
            add_counters(A, cnt);
            double *u1 = U1 + (size_t)b * nv * G->P;
            for (int z = 0; z < G->n[2]; z++)
                for (int y = 0; y < G->n[1]; y++)
                    for (int x = 0; x < G->n[0]; x++)
                        for (int k = 0; k < nv; k++)
                            u1[k * G->P + at(G, x, y, z)] = unew[k * G->I + interior_index(G, x, y, z)];
        }
        free(unew);
    }
    /* the boundary procedure on the stage state */
    double *U0 = A->U;
    A->U = U1;
    orc_amr_restrict(A);
    orc_amr_fill(A);
    A->U = U0;
#pragma omp parallel num_threads(g_threads)
    {
        double *unew = malloc(sizeof(double) * nv * G->I);
#pragma omp for schedule(dynamic, 4)
        for (int b = 0; b < A->nb; b++) {
            if (A->haskids[b])
                continue;
            double dx[3];
            block_dx(A, b, dx);
            const orc_dtrec *r = &dt[A->keys[b].sim];
            double *ff = A->ff + (size_t)b * 2 * A->nd * nv * A->T;
            long cnt[4] = {0, 0, 0, 0};
            orc_step_tile(&A->p, dx, U1 + (size_t)b * nv * G->P, nn, r, unew, ff, cnt);
            add_counters(A, cnt);
            double *u = tile(A, b);
            for (int z = 0; z < G->n[2]; z++)
                for (int y = 0; y < G->n[1]; y++)
                    for (int x = 0; x < G->n[0]; x++) {
                        long c = at(G, x, y, z), ic = interior_index(G, x, y, z);
                        for (int k = 0; k < nv; k++)
                            u[k * G->P + c] = 0.5 * (u[k * G->P + c] + unew[k * G->I + ic]);
                        if (A->p.physics == ORC_MHD)
                            u[PSI * G->P + c] = u[PSI * G->P + c] * r->damp;
                    }
            const double *f1 = ff1 + (size_t)b * 2 * A->nd * nv * A->T;
            for (size_t i = 0; i < (size_t)2 * A->nd * nv * A->T; i++)
                ff[i] = 0.5 * f1[i] + 0.5 * ff[i];
        }
        free(unew);
    }
    free(U1);
    free(ff1);
}

/* Sec. 4.3 step 2: a coarse leaf next to finer leaves replaces its own face
 * flux by the area mean of the fine face fluxes (same dt on all levels). */
void orc_amr_reflux(orc_amr *A, const orc_dtrec *dt)
{
    geo *G = &A->G;
    int n = A->n, nd = A->nd, nv = A->nv;
    long T = A->T;
    /* a coarse leaf writes only its own cells and reads fine face fluxes */
#pragma omp parallel for schedule(dynamic, 8) num_threads(g_threads)
    for (int b = 0; b < A->nb; b++) {
        if (A->haskids[b])
            continue;
        const orc_key *k = &A->keys[b];
        const orc_sim *S = &A->sims[k->sim];
        int kc[3];
        key_coords(k, kc);
        double dx[3];
        block_dx(A, b, dx);
        double *u = tile(A, b);
        for (int d = 0; d < nd; d++) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            for (int side = 0; side < 2; side++) {
                int nbk[3] = {kc[0], kc[1], kc[2]};
                int nblocks = S->nbase[d] << (k->level - 1);
                nbk[d] += side ? 1 : -1;
                if (nbk[d] < 0 || nbk[d] >= nblocks) {
                    if (S->bc[d][side] != ORC_BC_PERIODIC)
                        continue;
                    nbk[d] = (nbk[d] + nblocks) % nblocks;
                }
                int nbb = lookup(A, k->sim, k->level, nbk[0], nbk[1], nbk[2]);
                if (nbb < 0 || !A->haskids[nbb])
                    continue;
                int fside = 1 - side;
                double dtdx = dt[k->sim].dt / dx[d];
                const double *fc = A->ff + ((size_t)b * 2 * nd + 2 * d + side) * nv * T;
                int na = n, nbt = (nd == 3) ? n : 1;
                for (int tb = 0; tb < nbt; tb++)
                    for (int ta = 0; ta < na; ta++) {
                        /* the 2^(d-1) fine faces covering this coarse face */
                        double fsum[NVMAX];
                        double fv[4][NVMAX];
                        int nfine = (nd == 3) ? 4 : 2;
                        for (int o = 0; o < nfine; o++) {
                            int fk[3];
                            int lft[3];
                            fk[d] = 2 * nbk[d] + (side ? 0 : 1);
                            int ga = 2 * (kc[t1] * n + ta) + (o & 1);
                            fk[t1] = ga / n;
                            lft[t1] = ga - fk[t1] * n;
                            if (nd == 3) {
                                int gb = 2 * (kc[t2] * n + tb) + ((o >> 1) & 1);
                                fk[t2] = gb / n;
                                lft[t2] = gb - fk[t2] * n;
                            } else {
                                fk[t2] = 0;
                                lft[t2] = 0;
                            }
                            int fb = lookup(A, k->sim, k->level + 1, fk[0], fk[1], fk[2]);
                            const double *ffb = A->ff + ((size_t)fb * 2 * nd + 2 * d + fside) * nv * T;
                            long t = (long)lft[t2] * n + lft[t1];
                            for (int kv = 0; kv < nv; kv++)
                                fv[o][kv] = ffb[kv * T + t];
                        }
                        for (int kv = 0; kv < nv; kv++) {
                            if (nd == 3)
                                fsum[kv] = ((fv[0][kv] + fv[1][kv]) + (fv[2][kv] + fv[3][kv])) * 0.25;
                            else
                                fsum[kv] = (fv[0][kv] + fv[1][kv]) * 0.5;
                        }
                        int loc[3];
                        loc[d] = side ? n - 1 : 0;
                        loc[t1] = ta;
                        loc[t2] = tb;
                        long c = at(G, loc[0], loc[1], loc[2]);
                        long t = (long)tb * n + ta;
                        for (int kv = 0; kv < nv; kv++) {
                            double delta = dtdx * (fc[kv * T + t] - fsum[kv]);
                            if (side)
                                u[kv * G->P + c] = u[kv * G->P + c] + delta;
                            else
                                u[kv * G->P + c] = u[kv * G->P + c] - delta;
                        }
                    }
            }
        }
    }
}

void orc_amr_totals(const orc_amr *A, double *out)
{
    const geo *G = &A->G;
    memset(out, 0, sizeof(double) * A->nsims * A->nv);
    for (int b = 0; b < A->nb; b++) {
        if (A->haskids[b])
            continue;
        double dx[3];
        block_dx(A, b, dx);
        double vol = dx[0] * dx[1] * (A->nd == 3 ? dx[2] : 1.0);
        const double *u = A->U + (size_t)b * A->nv * G->P;
        double *o = out + (size_t)A->keys[b].sim * A->nv;
        for (int kv = 0; kv < A->nv; kv++)
            for (int z = 0; z < G->n[2]; z++)
                for (int y = 0; y < G->n[1]; y++)
                    for (int x = 0; x < G->n[0]; x++)
                        o[kv] += u[kv * G->P + at(G, x, y, z)] * vol;
    }
}

/* the conduction subcycle of one step (Sec. 3.4, Fig. 1): sub-step i
 * updates the energy of every leaf of each simulation with i < nsub, then
 * the boundary procedure for the energy: reflux with the sub-step dt,
 * restriction, exchange and prolongation (the other variables are unchanged,
 * so refilling them is harmless). */
void orc_amr_conduct(orc_amr *A, const orc_dtrec *dt)
{
    geo *G = &A->G;
    int nn[3] = {A->n, A->n, A->n};
    int maxsub = 0;
    for (int s = 0; s < A->nsims; s++)
        if (dt[s].nsub > maxsub)
            maxsub = dt[s].nsub;
    if (maxsub == 0)
        return;
    double *enew = malloc(sizeof(double) * (size_t)A->nb * G->I);
    orc_dtrec *sub = malloc(sizeof(orc_dtrec) * A->nsims);
    size_t nff = (size_t)2 * A->nd * A->nv * A->T;
    for (int i = 0; i < maxsub; i++) {
        for (int s = 0; s < A->nsims; s++) {
            sub[s] = dt[s];
            sub[s].dt = i < dt[s].nsub ? dt[s].dt_sub : 0.0;
        }
#pragma omp parallel for schedule(dynamic, 4) num_threads(g_threads)
        for (int b = 0; b < A->nb; b++) {
            double *ff = A->ff + (size_t)b * nff;
            if (A->haskids[b])
                continue;
            if (sub[A->keys[b].sim].dt == 0.0) {
                memset(ff, 0, sizeof(double) * nff);
                continue;
            }
            double dx[3];
            block_dx(A, b, dx);
            orc_conduct_tile(&A->p, dx, tile(A, b), nn, sub[A->keys[b].sim].dt,
                             enew + (size_t)b * G->I, ff);
        }
        for (int b = 0; b < A->nb; b++) {
            if (A->haskids[b] || sub[A->keys[b].sim].dt == 0.0)
                continue;
            double *u = tile(A, b);
            for (int z = 0; z < G->n[2]; z++)
                for (int y = 0; y < G->n[1]; y++)
                    for (int x = 0; x < G->n[0]; x++)
                        u[EN * G->P + at(G, x, y, z)] =
                            enew[(size_t)b * G->I + interior_index(G, x, y, z)];
        }
        orc_amr_reflux(A, sub);
        orc_amr_restrict(A);
        orc_amr_fill(A);
    }
    free(enew);
    free(sub);
}

/* one cycle per step: dt, update of all leaves, reflux, restriction, then
 * ghost exchange and prolongation (the main loop of Fig. 1 with the boundary
 * work moved after the update), then the conduction subcycle. */
void orc_amr_run(orc_amr *A, int nsteps, orc_dtrec *trace)
{
    orc_dtrec *r = malloc(sizeof(orc_dtrec) * A->nsims);
    for (int it = 0; it < nsteps; it++) {
        orc_amr_cfl(A, r);
        if (trace)
            memcpy(trace + (size_t)it * A->nsims, r, sizeof(orc_dtrec) * A->nsims);
        orc_amr_step(A, r);
        orc_amr_reflux(A, r);
        orc_amr_restrict(A);
        orc_amr_fill(A);
        orc_amr_conduct(A, r);
    }
    free(r);
}

/* ------------------------------------------------------------------ */
/* regrid error estimator (Sec. 4.5)                                   */
/* ------------------------------------------------------------------ */
static double est_value(const double *u, long P, long c, int mode, int kv)
{
    if (mode == 1) {
        double bx = u[BX * P + c], by = u[BY * P + c], bz = u[BZ * P + c];
        return sqrt(bx * bx + by * by + bz * bz);
    }
    return u[kv * P + c];
}

double orc_estimate(const orc_params *p, const double *u, const int n_in[3], int mode,
                    int kv, double eps, double filt, double bias, double ratio,
                    double xi, int level)
{
    geo G = mkgeo(p->ndim, n_in);
    int lo[3], hi[3];
    e_range(&G, lo, hi);
    double scale = pow(ratio, xi * (level - 1));
    double best = 0.0;
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                long c = at(&G, x, y, z);
                double v = est_value(u, G.P, c, mode, kv);
                double s1 = 0.0, s2 = 0.0;
                for (int d = 0; d < G.nd; d++) {
                    double vp = est_value(u, G.P, c + G.s[d], mode, kv);
                    double vm = est_value(u, G.P, c - G.s[d], mode, kv);
                    s1 += (vp - vm) * (vp - vm);
                    s2 += (vp - 2.0 * v + vm) * (vp - 2.0 * v + vm);
                }
                double d1 = 0.5 * sqrt(3.0) * sqrt(s1);
                double d2 = sqrt(s2);
                double av = fabs(v) + eps;
                double e = (bias * d1 / av + (1.0 - bias) * d2 / (d1 + filt * av)) * scale;
                if (e > best)
                    best = e;
            }
    return best;
}
