/*
 * oracle.h -- plain, slow, FP64 CPU reference of the MAP block update
 * (Jiang, Fang & Chen, "MAP: an MHD code with AMR and parallelization").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or execute this code; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.  It shares no source with the
 * HIP library: it has its own tables, its own tree search and its own
 * arithmetic, written from the paper's equations in the paper's order.
 *
 * Conventions (all arrays are C order, FP64):
 *   variables   k = 0..8 : rho, m_x, m_y, m_z, B_x, B_y, B_z, e, psi
 *               (Sec. 2, EGLM-MHD system); scalar test physics has nvar = 1.
 *   padded tile [k][z][y][x] with 2 ghost layers in every active dimension
 *               (2-D tiles have a single z plane and no z ghosts).
 *   block keys  (sim, level, ix, iy, iz); the base level is 1 (Sec. 4.1).
 */
#ifndef MAP_ORACLE_H
#define MAP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MHD = 0, ORC_SCALAR = 1 };
enum { ORC_LF = 0, ORC_MMC = 1, ORC_WENO = 2 };
enum { ORC_MINMOD = 0, ORC_VANLEER = 1, ORC_PAPER_PHI = 2 };
enum { ORC_GLM_PAPER = 0, ORC_GLM_FASTSPEED = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1 };
enum { ORC_RUSANOV = 0, ORC_HLLC = 1 };
enum { ORC_COND_OFF = 0, ORC_COND_ISO = 1, ORC_COND_FIELD = 2 };

typedef struct {
    int ndim;          /* 2 or 3 */
    int physics;       /* ORC_MHD or ORC_SCALAR */
    int scheme;        /* ORC_LF, ORC_MMC, or ORC_WENO (with TVD Runge-Kutta 2) */
    int limiter;       /* slope limiter (LF) or flux limiter (MMC) */
    int glm_mode;      /* how c_h and the psi damping factor follow from dt */
    int eglm_sources;  /* 1: EGLM source terms on, 0: plain GLM */
    int riemann;       /* face flux of LF and WENO: ORC_RUSANOV or ORC_HLLC */
    int cond_mode;     /* thermal conduction: ORC_COND_OFF, _ISO, or _FIELD (along B) */
    int cond_max_sub;  /* at most this many conduction sub-steps per step */
    double gamma, cfl, cd, cr, eta;
    double kappa0, kappa_exp;  /* kappa = kappa0 T^kappa_exp, T = p/rho; the
                                  exponent is a multiple of 1/2 in [0, 5] */
    double adv[3];     /* scalar physics: constant advection velocity */
} orc_params;

typedef struct {
    double dt, ch, damp, alpha;  /* time step, GLM speed, psi factor, max speed */
    double dt_sub;               /* conduction sub-step dt / nsub (0: no conduction) */
    int nsub, reserved;          /* conduction sub-steps in this step */
} orc_dtrec;

typedef struct {
    double lo[3], hi[3];
    int nbase[3];      /* base-level blocks per dimension */
    int bc[3][2];      /* ORC_BC_* per dimension and side */
} orc_sim;

typedef struct {
    int sim, level, ix, iy, iz;
} orc_key;

/* threads of the block-tree loops (orc_amr_*), default 1; results are the
 * same bit for bit for any count */
void   orc_set_threads(int n);
int    orc_get_threads(void);

/* ---- pointwise physics (Sec. 2, Sec. 3) ---- */
int    orc_nvar(const orc_params *p);
double orc_pressure(const orc_params *p, const double *u);
void   orc_flux(const orc_params *p, const double *u, int dim, double ch,
                double *f);
double orc_speed(const orc_params *p, const double *u, int dim);
double orc_limiter(int kind, double a, double b);
/* face flux between the states L and R across a face normal to `dim`:
 * Rusanov (Equ:LFFlux) or HLLC, as p->riemann selects */
void   orc_face_flux(const orc_params *p, const double *L, const double *R, int dim,
                     double ch, double *f);
/* the HLLC fan of a face (for tests): speeds S_L, S_M, S_R and the star
 * states of both sides, computed with B_d replaced by the GLM interface value */
void   orc_hllc_fan(const orc_params *p, const double *L, const double *R, int dim,
                    double ch, double S[3], double UsL[9], double UsR[9]);
/* WENO face state (Sec. 3.3) from the cells i-1, i, i+1: side 0 gives
 * u^-_{i+1/2} (left state of the face right of cell i), side 1 gives
 * u^+_{i-1/2} (right state of the face left of cell i). */
double orc_weno_face(double um, double u0, double up, int side);
void   orc_prim_to_cons(const orc_params *p, double *w, long ncell);

/* ---- one padded tile (any interior size n[0] x n[1] x n[2]) ----
 * unew receives the interior [nvar][n2][n1][n0]; ff (may be NULL) receives
 * the fluxes of the 2*ndim boundary faces, [2*d+side][nvar][t2][t1];
 * cnt[0] counts slope fall-backs, cnt[1] face-state fall-backs. */
void orc_step_tile(const orc_params *p, const double dx[3], const double *u,
                   const int n[3], const orc_dtrec *dt, double *unew,
                   double *ff, long *cnt);
/* LF intermediate states (positivity fall-back tests): ut[nvar][P] the
 * predicted state, sl[ndim][nvar][P] the slopes after the fall-back,
 * lr[ndim][2][nvar][P] the left/right states each face flux receives
 * (face c+1/2 at cell c); cnt as in orc_step_tile. */
void orc_lf_states(const orc_params *p, const double dx[3], const double *u,
                   const int n[3], const orc_dtrec *dt, double *ut, double *sl,
                   double *lr, long *cnt);
/* EGLM source densities -(divB)B and -B.grad(psi) on the interior,
 * out[nvar][interior] (zero for the other components). */
void orc_eglm_source(const orc_params *p, const double dx[3], const double *u,
                     const int n[3], double *out);
/* resistive terms R = -curl(eta J) and R_e = -div((eta J) x B) on the
 * interior, out[nvar][interior] (B rows and e row filled). */
void orc_resistive(const orc_params *p, const double dx[3], const double *u,
                   const int n[3], double *out);
/* max over the interior of max_d speed_d */
double orc_tile_maxspeed(const orc_params *p, const double *u, const int n[3]);
/* time-step record from a max speed and the smallest cell width */
void orc_make_dtrec(const orc_params *p, double alpha, double dxmin,
                    double kmax, orc_dtrec *out);
/* largest kappa T / p over the interior of a tile (Sec. 3.4 sub-step) */
double orc_tile_cond_rate(const orc_params *p, const double *u, const int n[3]);
/* one conduction sub-step on a padded tile (Sec. 3.4): enew receives the
 * interior energy [n2][n1][n0]; ff (may be NULL) the face fluxes as in
 * orc_step_tile (zero except the energy component) */
void orc_conduct_tile(const orc_params *p, const double dx[3], const double *u,
                      const int n[3], double dt_sub, double *enew, double *ff);

/* ---- single uniform grid (monolithic mode): one tile covering a domain ---- */
void orc_grid_fill(const orc_params *p, double *u, const int n[3],
                   const int bc[3][2]);
void orc_grid_run(const orc_params *p, const double dx[3], double *u,
                  const int n[3], const int bc[3][2], int nsteps,
                  double *dt_trace, long *cnt);

/* ---- block tree (AMR mode) ---- */
typedef struct orc_amr orc_amr;
orc_amr *orc_amr_new(const orc_params *p, int n, int nsims,
                     const orc_sim *sims, int nblocks, const orc_key *keys);
void     orc_amr_free(orc_amr *a);
double  *orc_amr_state(orc_amr *a);            /* [nblocks][nvar][P] */
int      orc_amr_tile_cells(const orc_amr *a); /* P */
int      orc_amr_is_leaf(const orc_amr *a, int b);
void     orc_amr_prim_to_cons(orc_amr *a);
void     orc_amr_fill(orc_amr *a);
void     orc_amr_restrict(orc_amr *a);
void     orc_amr_prolong_block(orc_amr *a, int b);
void     orc_amr_cfl(orc_amr *a, orc_dtrec *out /* [nsims] */);
void     orc_amr_step(orc_amr *a, const orc_dtrec *dt);
void     orc_amr_reflux(orc_amr *a, const orc_dtrec *dt);
void     orc_amr_totals(const orc_amr *a, double *out /* [nsims][nvar] */);
void     orc_amr_conduct(orc_amr *a, const orc_dtrec *dt);  /* the conduction subcycle */
void     orc_amr_run(orc_amr *a, int nsteps, orc_dtrec *trace /* [nsteps][nsims] or NULL */);
void     orc_amr_counters(const orc_amr *a, long out[4]);

/* ---- regrid error estimator (Sec. 4.5), on one padded tile ----
 * mode 0: the variable k_var itself; mode 1: |B|.  Returns the largest
 * estimate over the interior plus one ghost ring. */
double orc_estimate(const orc_params *p, const double *u, const int n[3],
                    int mode, int k_var, double eps, double filt,
                    double bias, double ratio, double xi, int level);

#ifdef __cplusplus
}
#endif
#endif
