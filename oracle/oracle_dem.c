/*
 * Plain FP64 CPU oracle of the soft-sphere DEM time step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the GPU library.  Compiled with -ffp-contract=off so that every
 * expression is evaluated exactly as written (no fused multiply-add).
 *
 * Source of every formula: Golshan et al., "Lethe-DEM: an open-source parallel
 * discrete element solver with load balancing" (arXiv 2106.09576).
 *   Sec. 2, Eqs. (main1)-(main2)   Newton-Euler equations of motion
 *   Sec. 2.1, Eq. (deltan)         normal overlap
 *   Sec. 2.1, Eq. (vecn)           contact normal, from i to j
 *   Sec. 2.1, Eq. (delta_t)        tangential overlap history update
 *   Sec. 2.1, Eq. (vrt) and the two equations after it: relative velocities
 *   Sec. 2.1, Eqs. (normal_force), (tangential_force): spring-dashpot laws
 *   Sec. 2.1, Eqs. (nonlinearkn)-(nonlinearetat) and the table of effective
 *             parameters: Hertz-Mindlin coefficients
 *   Sec. 2.1, Eq. (torque_t)       tangential torque
 *   Sec. 2.1, Eqs. (linearkn), (linearetan): linear spring-dashpot coefficients
 *   Sec. 2.1, table of rolling models: constant and viscous rolling torque
 *   Sec. 2.1, Eqs. (coulomb_overlap)-(coulomb_overlap3): Coulomb limit with
 *             truncation of the tangential overlap
 *   Sec. 2.1, last paragraph       particle-wall contacts use the same law
 *   Sec. 2.2, Eqs. (integ_EE), (halfstep), (newvv): explicit Euler and
 *             velocity Verlet
 *   Sec. 3.2                       broad search over cells and their neighbour
 *             cells listed without repetition, then a fine search that keeps
 *             pairs closer than a threshold; Sec. 3.1: searched every n steps
 *   Sec. 3.7                       moving (rotating and translating) and floating
 *                                  walls; particle-face, particle-line and
 *                                  particle-point contacts with meshed walls
 *   walls are analytic surfaces (plane, cylinder, cone) or triangle meshes
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - the undefined force F^c in the tangential torque is the tangential force;
 *     the torque on j is R_j n_ij x F^t_ij and the rolling torque on j is the
 *     negative of the one on i;
 *   - rolling torque is zero when omega_i == omega_j exactly;
 *   - the Coulomb test and the rolling torque use the full normal force
 *     (spring + damping); no truncation when |F^t| == 0;
 *   - delta_t is incremented before the force is evaluated, with no projection;
 *   - delta_t is reset to zero whenever a listed pair does not touch;
 *   - velocity Verlet evaluates forces at x^{n+1} with v^{n+1/2};
 *   - F = T = 0 before the first step;
 *   - solid spheres: m = rho (4/3) pi R^3, I = (2/5) m R^2;
 *   - search radius r_s = min(threshold, cell_factor) d_max, cell edge
 *     h = cell_factor d_max (1 + 1e-9), skin s = r_s - d_max;
 *   - a wall is a candidate when the centre-to-surface distance is below
 *     R + s and above -R; walls are bodies of infinite mass and radius: R_e =
 *     R_i, m_e = m_i, wall surface velocity at the contact point replaces the
 *     velocity of body j, the wall's angular velocity enters the rolling term;
 *     restitution, friction and rolling friction are the wall material's;
 *   - unlike particle types: restitution, friction and rolling friction are the
 *     arithmetic means of the two materials (parity unpinned: the paper fixes
 *     no mixing rule and no closed form or published value checks this one;
 *     the effective mass, radius and moduli of unlike spheres are pinned);
 *   - particles outside the domain box become inactive at a contact search;
 *   - viscous rolling torque against a wall: V_omega = R_i (omega_i -
 *     Omega_wall) x n (the particle's lever arm, spin relative to the wall's);
 *   - linear model: the tangential spring and damping constants equal the
 *     normal ones; e = 1 gives zero damping (the limit of the formula).
 *
 * Parity unpinned: trajectories of dense packings over long horizons, where
 * the dynamics are chaotic; pins and comparisons use short horizons and
 * non-chaotic scenes.
 */
#include "oracle_dem.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

typedef struct {
  int kind; /* 0 plane, 1 cylinder, 2 cone, 3 triangle mesh */
  double p[3];     /* plane point / axis point */
  double nrm[3];   /* plane normal (into the domain) / axis direction */
  int bounded;
  double u[3], vax[3], hu, hv; /* plane extent */
  double radius, smin, smax;   /* cylinder; cone: radius at s = 0 */
  double slope;                /* cone: radius grows by slope per unit s */
  int inside;
  int material;
  double omega[3]; /* angular velocity vector of the wall */
  double ax[3];    /* a point on the rotation axis */
  double t_on, t_off;
  double vel[3];   /* translational velocity: p and ax move with it */
  int64_t tri_begin, ntri; /* mesh: its triangles in the simulation's list */
} ora_wall;

/* One triangle of a mesh wall: corners at time 0 (the front side, where the
   particles are, is the side of (p1 - p0) x (p2 - p0)) and the mesh's own
   indices of the corners, which name its edges and vertices. */
typedef struct {
  double p[3][3];
  int32_t v[3];
} ora_tri;

/* The wall at time t: its point and rotation axis translated by vel t. */
static ora_wall wall_at(const ora_wall* W, double t) {
  ora_wall out = *W;
  for (int k = 0; k < 3; ++k) {
    out.p[k] = W->p[k] + W->vel[k] * t;
    out.ax[k] = W->ax[k] + W->vel[k] * t;
  }
  return out;
}

typedef struct {
  int64_t i, j; /* gid_i < gid_j */
  double dt[3]; /* tangential overlap, orientation i -> j */
  double f[3];  /* F^n + F^t on i at the last evaluation (0 when not touching) */
} ora_pair;

typedef struct {
  int64_t i;
  int32_t w;
  double dt[3];
} ora_wpair;

/* particle-triangle candidate of a mesh wall */
typedef struct {
  int64_t i;
  int32_t w;
  int64_t tri; /* index in the simulation's triangle list */
  double dt[3];
} ora_mpair;

struct ora_sim {
  ora_config cfg;
  ora_material mat[ORA_MAX_TYPES];
  int mat_set[ORA_MAX_TYPES];
  int64_t n;
  double *x, *v, *w, *R, *m, *I, *F, *T, *S, *S2, *xref;
  int32_t* type;
  uint8_t* active;
  double dmax, rs, rs2, h, skin;
  int64_t nc[3];
  int nw;
  ora_wall walls[ORA_MAX_WALLS];
  ora_pair* pairs;
  int64_t npairs;
  ora_wpair* wpairs;
  int64_t nwpairs;
  ora_tri* tris;
  int64_t ntris;
  ora_mpair* mpairs;
  int64_t nmpairs;
  int64_t step;
  int ready;
#ifdef ORA_PARALLEL
  /* timing build only: per-pair law results and the per-particle pair index */
  double* prec;           /* 11 doubles per pair: F_i, M_i, M_j, the two scales */
  int64_t prec_cap;
  int64_t *ifirst, *jfirst, *jlist;
  int64_t idx_n, idx_pairs;
  int idx_dirty;
#endif
};

/* ------------------------------------------------------------------ vectors */

static void vsub(const double* a, const double* b, double* r) {
  r[0] = a[0] - b[0];
  r[1] = a[1] - b[1];
  r[2] = a[2] - b[2];
}
static double vdot(const double* a, const double* b) {
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
static void vcross(const double* a, const double* b, double* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
static double vnorm(const double* a) { return sqrt(vdot(a, a)); }

/* --------------------------------------------------------------- materials */

/* Table of effective parameters (Sec. 2.1). */
static double eff_youngs(const ora_material* a, const ora_material* b) {
  return 1.0 / ((1.0 - a->poisson * a->poisson) / a->youngs +
                (1.0 - b->poisson * b->poisson) / b->youngs);
}
static double eff_shear(const ora_material* a, const ora_material* b) {
  return 1.0 / (2.0 * (2.0 - a->poisson) * (1.0 + a->poisson) / a->youngs +
                2.0 * (2.0 - b->poisson) * (1.0 + b->poisson) / b->youngs);
}
static double beta_of(double e) {
  double le = log(e);
  return le / sqrt(le * le + PI * PI);
}

/* Everything the contact law needs about a contact besides kinematics. */
typedef struct {
  double me, Re, Ye, Ge, e, mu, mur;
} ora_contact_props;

/*
 * The spring-dashpot contact law of Sec. 2.1 for one contact, with the
 * nonlinear (Hertz-Mindlin) or the linear spring and damping constants.
 * Inputs: overlap dn > 0, unit normal n from body i towards body j, contact
 * relative velocity vij, relative angular velocity wrel = omega_i - omega_j,
 * the rolling velocity vroll (V_omega of the table of rolling models), the
 * lever arms Ri, Rj and the tangential overlap (updated in place).
 * Outputs: the force on i (normal + tangential), the torques on i and j, and
 * two force scales: fmag[0] = |F^n + F^t| and fmag[1] = the sum of the
 * magnitudes of the four terms of Eqs. (normal_force) and (tangential_force)
 * before the Coulomb limit (spring and dashpot of each), which stays large
 * where the spring and the dashpot nearly cancel.
 */
static void contact_law(const ora_contact_props* cp, const ora_config* cfg, double dn,
                        const double* n, const double* vij, const double* wrel,
                        const double* vroll, double Ri, double Rj, double* delta_t,
                        double* Fi, double* Mi, double* Mj, double* fmag) {
  const double dt = cfg->dt;
  double vn = vdot(vij, n);
  double vrn[3] = {vn * n[0], vn * n[1], vn * n[2]};
  double vrt[3];
  vsub(vij, vrn, vrt);
  /* Eq. (delta_t): single-step accumulation, before the force is evaluated */
  for (int k = 0; k < 3; ++k) delta_t[k] = delta_t[k] + vrt[k] * dt;

  double kn, kt, etan, etat;
  if (cfg->contact_model == 0) {
    double beta = beta_of(cp->e);
    double q = sqrt(cp->Re * dn);
    kn = 4.0 / 3.0 * cp->Ye * q;                /* Eq. (nonlinearkn) */
    kt = 8.0 * cp->Ge * q;                      /* Eq. (nonlinearkt) */
    double Sn = 2.0 * cp->Ye * q;               /* S_n */
    double St = 8.0 * cp->Ge * q;               /* S_t */
    etan = -2.0 * sqrt(5.0 / 6.0) * beta * sqrt(Sn * cp->me); /* Eq. (nonlinearetan) */
    etat = -2.0 * sqrt(5.0 / 6.0) * beta * sqrt(St * cp->me); /* Eq. (nonlinearetat) */
  } else {
    /* linear model, Eqs. (linearkn), (linearetan); the tangential constants
       are the same; e = 1 (ln e = 0) is the undamped limit */
    double V = cfg->characteristic_velocity;
    double sr = sqrt(cp->Re);
    kn = 16.0 / 15.0 * sr * cp->Ye * pow(15.0 * cp->me * V * V / (16.0 * sr * cp->Ye), 0.2);
    double le = log(cp->e);
    etan = 0.0;
    if (le != 0.0) {
      double pl = PI / le;
      etan = sqrt(4.0 * cp->me * kn / (1.0 + pl * pl));
    }
    kt = kn;
    etat = etan;
  }

  double Fn[3], Ft[3];
  for (int k = 0; k < 3; ++k) {
    Fn[k] = -(kn * dn) * n[k] - etan * vrn[k];       /* Eq. (normal_force) */
    Ft[k] = -(kt * delta_t[k]) - etat * vrt[k];      /* Eq. (tangential_force) */
  }
  double fn = vnorm(Fn);
  double ft = vnorm(Ft);
  const double terms = kn * dn + fabs(etan) * fabs(vn) + kt * vnorm(delta_t) +
                       fabs(etat) * vnorm(vrt);
  /* Coulomb criterion, Eqs. (coulomb_overlap)-(coulomb_overlap3) */
  if (ft >= cp->mu * fn && ft > 0.0) {
    for (int k = 0; k < 3; ++k) {
      double fhat = cp->mu * fn * Ft[k] / ft;          /* limited force */
      double ftilde = fhat + etat * vrt[k];            /* limited elastic force */
      delta_t[k] = ftilde / (-kt);                     /* limited overlap */
      Ft[k] = fhat;
    }
  }
  /* Eq. (torque_t) with F^c read as F^t; the torque on j acts at -R_j n */
  double nxft[3];
  vcross(n, Ft, nxft);
  double Mr[3] = {0.0, 0.0, 0.0};
  if (cfg->rolling_model == 1) {
    /* constant rolling torque, first row of the rolling-model table */
    double wn = vnorm(wrel);
    if (wn > 0.0) {
      for (int k = 0; k < 3; ++k) Mr[k] = -cp->mur * cp->Re * fn * (wrel[k] / wn);
    }
  } else if (cfg->rolling_model == 2) {
    /* viscous rolling torque, second row: scaled by |V_omega| */
    double wn = vnorm(wrel);
    double vr = vnorm(vroll);
    if (wn > 0.0) {
      for (int k = 0; k < 3; ++k) Mr[k] = -cp->mur * cp->Re * fn * vr * (wrel[k] / wn);
    }
  }
  double Fsum[3];
  for (int k = 0; k < 3; ++k) {
    Fsum[k] = Fn[k] + Ft[k];
    Fi[k] = Fsum[k];
    Mi[k] = Ri * nxft[k] + Mr[k];
    Mj[k] = Rj * nxft[k] - Mr[k];
  }
  fmag[0] = vnorm(Fsum);
  fmag[1] = terms;
}

static void pp_props(const ora_sim* s, int ti, int tj, double mi, double mj, double Ri,
                     double Rj, ora_contact_props* cp) {
  const ora_material* a = &s->mat[ti];
  const ora_material* b = &s->mat[tj];
  cp->me = 1.0 / (1.0 / mi + 1.0 / mj);
  cp->Re = 1.0 / (1.0 / Ri + 1.0 / Rj);
  cp->Ye = eff_youngs(a, b);
  cp->Ge = eff_shear(a, b);
  if (ti == tj) {
    cp->e = a->restitution;
    cp->mu = a->friction;
    cp->mur = a->rolling_friction;
  } else {
    cp->e = 0.5 * (a->restitution + b->restitution);
    cp->mu = 0.5 * (a->friction + b->friction);
    cp->mur = 0.5 * (a->rolling_friction + b->rolling_friction);
  }
}

/* Particle-particle contact (i, j).  Returns 1 when the pair touches. */
static int pp_contact(const ora_sim* s, const double* xi, const double* xj,
                      const double* vi, const double* vj, const double* wi,
                      const double* wj, double Ri, double Rj, double mi, double mj,
                      int ti, int tj, double* delta_t, double* Fi, double* Mi,
                      double* Mj, double* fmag) {
  double dx[3];
  vsub(xj, xi, dx);
  double d2 = vdot(dx, dx);
  double rsum = Ri + Rj;
  for (int k = 0; k < 3; ++k) Fi[k] = Mi[k] = Mj[k] = 0.0;
  fmag[0] = fmag[1] = 0.0;
  if (!(d2 < rsum * rsum)) {
    delta_t[0] = delta_t[1] = delta_t[2] = 0.0; /* contact ended */
    return 0;
  }
  double d = sqrt(d2);
  double dn = rsum - d; /* Eq. (deltan) */
  if (dn < 0.0) dn = 0.0;
  double n[3] = {dx[0] / d, dx[1] / d, dx[2] / d}; /* Eq. (vecn) */
  double rw[3] = {Ri * wi[0] + Rj * wj[0], Ri * wi[1] + Rj * wj[1],
                  Ri * wi[2] + Rj * wj[2]};
  double rwxn[3];
  vcross(rw, n, rwxn);
  double vij[3], wrel[3];
  for (int k = 0; k < 3; ++k) {
    vij[k] = (vi[k] - vj[k]) + rwxn[k];
    wrel[k] = wi[k] - wj[k];
  }
  ora_contact_props cp;
  pp_props(s, ti, tj, mi, mj, Ri, Rj, &cp);
  /* V_omega = omega_i x R_i n_ij - omega_j x R_j n_ji = (R_i w_i + R_j w_j) x n */
  contact_law(&cp, &s->cfg, dn, n, vij, wrel, rwxn, Ri, Rj, delta_t, Fi, Mi, Mj, fmag);
  return 1;
}

/* ------------------------------------------------------------------- walls */

/* Geometry of particle centre x against wall W.  Fills the candidate and
   touching predicates (evaluated without square roots) and, when touching, the
   normal from the particle to the wall, the overlap and the contact point. */
typedef struct {
  int candidate, touching;
  double n[3], dn, xc[3];
} ora_wgeo;

/* Cone (frustum) around the axis through p along nrm: at axial coordinate s
   the surface lies at distance r(s) = radius + slope s from the axis.  A
   particle whose centre has s in [smin, smax] and lies at rho from the axis
   is at distance (r(s) - rho) / q from the surface line of its meridian
   (inside; rho - r(s) for outside), q = sqrt(1 + slope^2).  The predicates
   compare rho^2 with squared bounds, as for the cylinder.  The outward
   surface normal of the meridian is (e_rho - slope nrm) / q. */
static void cone_geometry(const ora_wall* W, const double* x, const double* rel, double R,
                          double skin, ora_wgeo* g) {
  double sax = vdot(rel, W->nrm);
  if (!(sax >= W->smin && sax <= W->smax)) return;
  double r[3] = {rel[0] - sax * W->nrm[0], rel[1] - sax * W->nrm[1],
                 rel[2] - sax * W->nrm[2]};
  double rho2 = vdot(r, r);
  if (!(rho2 > 0.0)) return;
  double q = sqrt(1.0 + W->slope * W->slope);
  double rs = W->radius + W->slope * sax;
  if (W->inside) {
    /* candidate: r(s) - (R + s) q < rho < r(s) + R q; touching: rho > r(s) - R q */
    double lo = rs - (R + skin) * q;
    double hi = rs + R * q;
    int above_lo = (lo <= 0.0) || (rho2 > lo * lo);
    g->candidate = above_lo && (hi > 0.0) && (rho2 < hi * hi);
    double lt = rs - R * q;
    g->touching = (lt <= 0.0) || (rho2 > lt * lt);
  } else {
    /* candidate: r(s) - R q < rho < r(s) + (R + s) q; touching: rho < r(s) + R q */
    double hi = rs + (R + skin) * q;
    double lo = rs - R * q;
    int above_lo = (lo <= 0.0) || (rho2 > lo * lo);
    g->candidate = above_lo && (hi > 0.0) && (rho2 < hi * hi);
    double lt = rs + R * q;
    g->touching = (lt > 0.0) && (rho2 < lt * lt);
  }
  if (g->touching) {
    double rho = sqrt(rho2);
    double er[3] = {r[0] / rho, r[1] / rho, r[2] / rho};
    double m[3] = {(er[0] - W->slope * W->nrm[0]) / q, (er[1] - W->slope * W->nrm[1]) / q,
                   (er[2] - W->slope * W->nrm[2]) / q};
    double dist = W->inside ? (rs - rho) / q : (rho - rs) / q;
    g->dn = R - dist;
    for (int k = 0; k < 3; ++k) {
      g->n[k] = W->inside ? m[k] : -m[k];
      g->xc[k] = x[k] + dist * g->n[k];
    }
  }
}

static void wall_geometry(const ora_wall* W, const double* x, double R, double skin,
                          ora_wgeo* g) {
  g->candidate = g->touching = 0;
  double rel[3];
  vsub(x, W->p, rel);
  if (W->kind == 0) {
    double dist = vdot(rel, W->nrm);
    if (W->bounded) {
      double a = vdot(rel, W->u), b = vdot(rel, W->vax);
      if (!(fabs(a) <= W->hu && fabs(b) <= W->hv)) return;
    }
    g->candidate = (dist < R + skin) && (dist > -R);
    g->touching = dist < R;
    if (g->touching) {
      for (int k = 0; k < 3; ++k) {
        g->n[k] = -W->nrm[k];
        g->xc[k] = x[k] - dist * W->nrm[k];
      }
      g->dn = R - dist;
    }
    return;
  }
  if (W->kind == 2) {
    cone_geometry(W, x, rel, R, skin, g);
    return;
  }
  /* cylinder */
  double sax = vdot(rel, W->nrm);
  if (!(sax >= W->smin && sax <= W->smax)) return;
  double r[3] = {rel[0] - sax * W->nrm[0], rel[1] - sax * W->nrm[1],
                 rel[2] - sax * W->nrm[2]};
  double rho2 = vdot(r, r);
  if (!(rho2 > 0.0)) return; /* centre on the axis: no defined normal */
  double Rc = W->radius;
  if (W->inside) {
    /* dist = Rc - rho; candidate: -R < dist < R + s; touching: dist < R */
    double lo = Rc - (R + skin);
    double hi = Rc + R;
    int above_lo = (lo <= 0.0) || (rho2 > lo * lo);
    g->candidate = above_lo && (rho2 < hi * hi);
    double lt = Rc - R;
    g->touching = (lt <= 0.0) || (rho2 > lt * lt);
  } else {
    /* dist = rho - Rc; candidate: -R < dist < R + s; touching: dist < R */
    double hi = Rc + R + skin;
    double lo = Rc - R;
    int above_lo = (lo <= 0.0) || (rho2 > lo * lo);
    g->candidate = above_lo && (rho2 < hi * hi);
    double lt = Rc + R;
    g->touching = rho2 < lt * lt;
  }
  if (g->touching) {
    double rho = sqrt(rho2);
    double er[3] = {r[0] / rho, r[1] / rho, r[2] / rho};
    double dist = W->inside ? (Rc - rho) : (rho - Rc);
    g->dn = R - dist;
    for (int k = 0; k < 3; ++k) {
      g->n[k] = W->inside ? er[k] : -er[k];
      g->xc[k] = W->p[k] + sax * W->nrm[k] + Rc * er[k];
    }
  }
}

static int wall_enabled(const ora_wall* W, double t) { return t >= W->t_on && t < W->t_off; }

/* The contact law against a wall (W at the current time) touching with unit
   normal n (from the particle to the wall), overlap dn and contact point xc. */
static void wall_law(const ora_sim* s, const ora_wall* W, const double* v, const double* w,
                     double R, double m, int ti, const double* n, double dn_geo,
                     const double* xc, double* delta_t, double* Fi, double* Mi, double* fmag) {
  ora_wgeo g;
  for (int k = 0; k < 3; ++k) {
    g.n[k] = n[k];
    g.xc[k] = xc[k];
  }
  double dn = dn_geo < 0.0 ? 0.0 : dn_geo;
  /* velocity of the wall surface at the contact point:
     v_wall + Omega x (x_c - axis point) */
  double arm[3], vw[3];
  vsub(g.xc, W->ax, arm);
  vcross(W->omega, arm, vw);
  for (int k = 0; k < 3; ++k) vw[k] = W->vel[k] + vw[k];
  double rw[3] = {R * w[0], R * w[1], R * w[2]};
  double rwxn[3];
  vcross(rw, g.n, rwxn);
  double vij[3], wrel[3];
  for (int k = 0; k < 3; ++k) {
    vij[k] = (v[k] - vw[k]) + rwxn[k];
    wrel[k] = w[k] - W->omega[k];
  }
  const ora_material* a = &s->mat[ti];
  const ora_material* b = &s->mat[W->material];
  ora_contact_props cp;
  cp.me = m;
  cp.Re = R;
  cp.Ye = eff_youngs(a, b);
  cp.Ge = eff_shear(a, b);
  cp.e = b->restitution;
  cp.mu = b->friction;
  cp.mur = b->rolling_friction;
  /* V_omega against a wall: the particle's lever arm with the spin relative
     to the wall's, R (omega - Omega_wall) x n */
  double rrel[3] = {R * wrel[0], R * wrel[1], R * wrel[2]};
  double vroll[3];
  vcross(rrel, g.n, vroll);
  double Mj[3];
  contact_law(&cp, &s->cfg, dn, g.n, vij, wrel, vroll, R, 0.0, delta_t, Fi, Mi, Mj, fmag);
}

/* Particle-wall contact, same law with the wall as body j. */
static int pw_contact(const ora_sim* s, const ora_wall* W, double t, const double* x,
                      const double* v, const double* w, double R, double m, int ti,
                      double* delta_t, double* Fi, double* Mi, double* fmag) {
  for (int k = 0; k < 3; ++k) Fi[k] = Mi[k] = 0.0;
  fmag[0] = fmag[1] = 0.0;
  const ora_wall Wt = wall_at(W, t);
  W = &Wt;
  ora_wgeo g;
  wall_geometry(W, x, R, s->skin, &g);
  if (!wall_enabled(W, t) || !g.touching) {
    delta_t[0] = delta_t[1] = delta_t[2] = 0.0;
    return 0;
  }
  wall_law(s, W, v, w, R, m, ti, g.n, g.dn, g.xc, delta_t, Fi, Mi, fmag);
  return 1;
}

/* ----------------------------------------------------------- mesh walls

   A mesh wall is a rigid surface of triangles (Sec. 3.7: particles collide
   with boundary faces, lines and points).  The closest point of a closed
   triangle to a particle centre x is the projection of x onto the
   triangle's plane when that projection lies strictly inside all three
   edges (a face contact), else the closest of the three edges' closest
   points (the projection onto the edge line clamped to the edge), which is
   an edge when the projection falls strictly inside the edge and a corner
   otherwise (line and point contacts). */
typedef struct {
  int feature;  /* 0 face, 1 edge, 2 vertex */
  int a, b;     /* edge: its corners a, a + 1 (mod 3); vertex: corner a */
  double s;     /* signed distance of x from the plane, along the unit normal */
  double d2;    /* squared distance from x to the closest point */
  double q[3];  /* the closest point */
  double n[3];  /* unit normal of the triangle (front side) */
} ora_trigeo;

/* T's corners move with the wall: at time t they are at p + vel t; the
   normal and the edge vectors are those of the corners at time 0. */
static void triangle_closest(const ora_tri* T, const double* vel, double t, const double* x,
                             ora_trigeo* g) {
  double P[3][3];
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 3; ++k) P[c][k] = T->p[c][k] + vel[k] * t;
  double e01[3], e02[3], N[3];
  vsub(T->p[1], T->p[0], e01);
  vsub(T->p[2], T->p[0], e02);
  vcross(e01, e02, N);
  const double len = vnorm(N);
  for (int k = 0; k < 3; ++k) g->n[k] = N[k] / len;
  double rel[3];
  vsub(x, P[0], rel);
  g->s = vdot(rel, g->n);
  /* inside: x lies on the inner side of every edge, strictly */
  int inside = 1;
  for (int c = 0; c < 3; ++c) {
    double E[3], r[3], cr[3];
    vsub(T->p[(c + 1) % 3], T->p[c], E);
    vsub(x, P[c], r);
    vcross(E, r, cr);
    if (!(vdot(cr, g->n) > 0.0)) inside = 0;
  }
  if (inside) {
    g->feature = 0;
    g->a = g->b = 0;
    for (int k = 0; k < 3; ++k) g->q[k] = x[k] - g->s * g->n[k];
    g->d2 = g->s * g->s;
    return;
  }
  g->d2 = INFINITY;
  for (int c = 0; c < 3; ++c) {
    double E[3], r[3], q[3], dq[3];
    vsub(T->p[(c + 1) % 3], T->p[c], E);
    vsub(x, P[c], r);
    const double u = vdot(r, E) / vdot(E, E);
    const double uc = u <= 0.0 ? 0.0 : (u >= 1.0 ? 1.0 : u);
    for (int k = 0; k < 3; ++k) q[k] = P[c][k] + uc * E[k];
    vsub(x, q, dq);
    const double d2 = vdot(dq, dq);
    if (d2 < g->d2) {
      g->d2 = d2;
      for (int k = 0; k < 3; ++k) g->q[k] = q[k];
      if (u <= 0.0) {
        g->feature = 2;
        g->a = g->b = c;
      } else if (u >= 1.0) {
        g->feature = 2;
        g->a = g->b = (c + 1) % 3;
      } else {
        g->feature = 1;
        g->a = c;
        g->b = (c + 1) % 3;
      }
    }
  }
}

/* A triangle is a candidate of a particle when the centre is less than R
   behind its plane and closer than R + skin to the closed triangle. */
static int triangle_candidate(const ora_trigeo* g, double R, double skin) {
  const double m = R + skin;
  return g->s > -R && g->d2 < m * m;
}

/* Identity of a triangle's closest feature within its mesh: faces by
   triangle, edges by their two corner indices (smaller first), vertices by
   corner index. */
typedef struct {
  int kind;
  int64_t a, b;
} ora_feature;

static ora_feature feature_of(const ora_tri* T, int64_t tri, const ora_trigeo* g) {
  ora_feature f;
  f.kind = g->feature;
  if (g->feature == 0) {
    f.a = tri;
    f.b = -1;
  } else if (g->feature == 1) {
    const int64_t va = T->v[g->a], vb = T->v[g->b];
    f.a = va < vb ? va : vb;
    f.b = va < vb ? vb : va;
  } else {
    f.a = T->v[g->a];
    f.b = -1;
  }
  return f;
}

static int tri_has_vertex(const ora_tri* T, int64_t v) {
  return T->v[0] == v || T->v[1] == v || T->v[2] == v;
}

/* Contacts of particle i with one mesh wall, from its candidate triangles
   M[0..m) (ascending): the points of the surface where the distance from
   the centre has a local minimum closer than R.  Every candidate reports
   its closest point and the feature it lies on.  A face is in contact when
   the centre is less than R above its plane.  The distance restricted to
   one triangle is convex, so a point on an edge or a vertex is a local
   minimum of the surface exactly when every triangle around it has it as
   its own closest point: an edge or vertex counts when every candidate
   triangle that contains it reports it, once, evaluated by the first
   candidate that reports it, whose slot keeps the tangential overlap.  All
   other slots start over from zero. */
static void mesh_contacts(ora_sim* s, const ora_wall* W0, double t, ora_mpair* M, int64_t m) {
  const int64_t i = M[0].i;
  const double* x = &s->x[3 * i];
  const double R = s->R[i];
  const ora_wall Wt = wall_at(W0, t);
  const int on = wall_enabled(&Wt, t);
  ora_trigeo* G = (ora_trigeo*)malloc(sizeof(ora_trigeo) * (size_t)m);
  ora_feature* Fe = (ora_feature*)malloc(sizeof(ora_feature) * (size_t)m);
  for (int64_t k = 0; k < m; ++k) {
    triangle_closest(&s->tris[M[k].tri], W0->vel, t, x, &G[k]);
    Fe[k] = feature_of(&s->tris[M[k].tri], M[k].tri, &G[k]);
  }
  for (int64_t k = 0; k < m; ++k) {
    int contact = 0;
    if (on) {
      if (Fe[k].kind == 0) {
        contact = G[k].s < R;
      } else {
        int dropped = 0, owner = 1;
        for (int64_t j = 0; j < m && !dropped; ++j) {
          const ora_tri* Tj = &s->tris[M[j].tri];
          const int same = Fe[j].kind == Fe[k].kind && Fe[j].a == Fe[k].a && Fe[j].b == Fe[k].b;
          const int contains = tri_has_vertex(Tj, Fe[k].a) &&
                               (Fe[k].kind == 2 || tri_has_vertex(Tj, Fe[k].b));
          if (contains && !same) dropped = 1;
          if (j < k && same) owner = 0;
        }
        contact = !dropped && owner && G[k].d2 < R * R && G[k].d2 > 0.0;
      }
    }
    if (!contact) {
      M[k].dt[0] = M[k].dt[1] = M[k].dt[2] = 0.0;
      continue;
    }
    double n[3], dn;
    if (Fe[k].kind == 0) {
      for (int c = 0; c < 3; ++c) n[c] = -G[k].n[c];
      dn = R - G[k].s;
    } else {
      const double dist = sqrt(G[k].d2);
      for (int c = 0; c < 3; ++c) n[c] = (G[k].q[c] - x[c]) / dist;
      dn = R - dist;
    }
    double Fi[3], Mi[3], fm[2];
    wall_law(s, &Wt, &s->v[3 * i], &s->w[3 * i], R, s->m[i], s->type[i], n, dn, G[k].q,
             M[k].dt, Fi, Mi, fm);
    for (int c = 0; c < 3; ++c) {
      s->F[3 * i + c] += Fi[c];
      s->T[3 * i + c] += Mi[c];
    }
    s->S[i] += fm[0];
    s->S2[i] += fm[1];
  }
  free(G);
  free(Fe);
}

/* ------------------------------------------------------------------ search */

static int cmp_pair(const void* a, const void* b) {
  const ora_pair* p = (const ora_pair*)a;
  const ora_pair* q = (const ora_pair*)b;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  if (p->j != q->j) return p->j < q->j ? -1 : 1;
  return 0;
}

static int64_t cell_coord(double x, double lo, double h) { return (int64_t)floor((x - lo) / h); }

static int inside_domain(const ora_sim* s, const double* x) {
  for (int k = 0; k < 3; ++k)
    if (!(x[k] >= s->cfg.domain_lo[k] && x[k] < s->cfg.domain_hi[k])) return 0;
  return 1;
}

/* Broad search over cells + fine search (Sec. 3.2).  Each cell is paired with
   itself and with the 13 neighbour cells that follow it, so every pair of
   neighbouring cells is visited once ("neighbour lists without repetition").
   The cell lists are a list of (cell id, gid) sorted by cell, so memory stays
   proportional to the number of particles whatever the domain size. */
typedef struct {
  int64_t cell, gid;
} ora_cell_entry;

static int cmp_cell_entry(const void* a, const void* b) {
  const ora_cell_entry* p = (const ora_cell_entry*)a;
  const ora_cell_entry* q = (const ora_cell_entry*)b;
  if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
  if (p->gid != q->gid) return p->gid < q->gid ? -1 : 1;
  return 0;
}

/* first index in E[0..m) whose cell is >= c */
static int64_t lower_bound_cell(const ora_cell_entry* E, int64_t m, int64_t c) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (E[mid].cell < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

static int build_candidates(ora_sim* s, ora_pair** out, int64_t* nout) {
  int64_t n = s->n;
  ora_cell_entry* E = (ora_cell_entry*)malloc(sizeof(ora_cell_entry) * (size_t)(n > 0 ? n : 1));
  if (!E) return ORA_ENOMEM;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!s->active[i]) continue;
    int64_t c[3];
    for (int k = 0; k < 3; ++k) {
      c[k] = cell_coord(s->x[3 * i + k], s->cfg.domain_lo[k], s->h);
      if (c[k] < 0) c[k] = 0;
      if (c[k] >= s->nc[k]) c[k] = s->nc[k] - 1;
    }
    E[m].cell = (c[2] * s->nc[1] + c[1]) * s->nc[0] + c[0];
    E[m].gid = i;
    ++m;
  }
  qsort(E, (size_t)m, sizeof(ora_cell_entry), cmp_cell_entry);
  int64_t cap = 1024, cnt = 0;
  ora_pair* P = (ora_pair*)malloc(sizeof(ora_pair) * (size_t)cap);
  if (!P) {
    free(E);
    return ORA_ENOMEM;
  }
  static const int half[13][3] = {{1, 0, 0},  {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},
                                  {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {-1, 0, 1},
                                  {0, 0, 1},  {1, 0, 1},  {-1, 1, 1}, {0, 1, 1},
                                  {1, 1, 1}};
  int64_t c0start = 0;
  while (c0start < m) {
    int64_t c0 = E[c0start].cell;
    int64_t c0end = c0start;
    while (c0end < m && E[c0end].cell == c0) ++c0end;
    int64_t cx = c0 % s->nc[0], cy = (c0 / s->nc[0]) % s->nc[1], cz = c0 / (s->nc[0] * s->nc[1]);
    for (int o = -1; o < 13; ++o) {
      int64_t b_lo, b_hi;
      if (o < 0) {
        b_lo = c0start;
        b_hi = c0end;
      } else {
        int64_t ox = cx + half[o][0], oy = cy + half[o][1], oz = cz + half[o][2];
        if (ox < 0 || oy < 0 || oz < 0 || ox >= s->nc[0] || oy >= s->nc[1] || oz >= s->nc[2])
          continue;
        int64_t c1 = (oz * s->nc[1] + oy) * s->nc[0] + ox;
        b_lo = lower_bound_cell(E, m, c1);
        b_hi = lower_bound_cell(E, m, c1 + 1);
      }
      for (int64_t ea = c0start; ea < c0end; ++ea) {
        int64_t a = E[ea].gid;
        for (int64_t eb = (o < 0 ? ea + 1 : b_lo); eb < b_hi; ++eb) {
          int64_t b = E[eb].gid;
          double dx[3];
          vsub(&s->x[3 * b], &s->x[3 * a], dx);
          double d2 = vdot(dx, dx);
          if (d2 < s->rs2) { /* fine search */
            if (cnt == cap) {
              cap *= 2;
              ora_pair* Q = (ora_pair*)realloc(P, sizeof(ora_pair) * (size_t)cap);
              if (!Q) {
                free(P);
                free(E);
                return ORA_ENOMEM;
              }
              P = Q;
            }
            P[cnt].i = a < b ? a : b;
            P[cnt].j = a < b ? b : a;
            P[cnt].dt[0] = P[cnt].dt[1] = P[cnt].dt[2] = 0.0;
            P[cnt].f[0] = P[cnt].f[1] = P[cnt].f[2] = 0.0;
            ++cnt;
          }
        }
      }
    }
    c0start = c0end;
  }
  free(E);
  qsort(P, (size_t)cnt, sizeof(ora_pair), cmp_pair);
  *out = P;
  *nout = cnt;
  return ORA_OK;
}

/* Contact search step: deactivate escaped particles, rebuild the particle-pair
   and particle-wall lists and carry the tangential overlap of pairs present in
   both the old and the new list. */
static int rebuild(ora_sim* s) {
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->active[i]) continue;
    for (int k = 0; k < 3; ++k)
      if (!isfinite(s->x[3 * i + k]) || !isfinite(s->v[3 * i + k]) ||
          !isfinite(s->w[3 * i + k]))
        return ORA_EUNSTABLE;
  }
  if (s->ready) {
    /* a contact can only be missed if a particle moved more than s/2 */
    double lim = 0.5 * s->skin;
    for (int64_t i = 0; i < s->n; ++i) {
      if (!s->active[i]) continue;
      double d[3];
      vsub(&s->x[3 * i], &s->xref[3 * i], d);
      if (vdot(d, d) > lim * lim) return ORA_EUNSTABLE;
    }
  }
  for (int64_t i = 0; i < s->n; ++i)
    if (s->active[i] && !inside_domain(s, &s->x[3 * i])) s->active[i] = 0;
  memcpy(s->xref, s->x, sizeof(double) * 3 * (size_t)s->n);

  ora_pair* np = NULL;
  int64_t nn = 0;
  int rc = build_candidates(s, &np, &nn);
  if (rc) return rc;
  /* merge: both lists sorted by (i, j) */
  int64_t a = 0;
  for (int64_t b = 0; b < nn; ++b) {
    while (a < s->npairs && cmp_pair(&s->pairs[a], &np[b]) < 0) ++a;
    if (a < s->npairs && cmp_pair(&s->pairs[a], &np[b]) == 0)
      memcpy(np[b].dt, s->pairs[a].dt, sizeof(double) * 3);
  }
  free(s->pairs);
  s->pairs = np;
  s->npairs = nn;
#ifdef ORA_PARALLEL
  s->idx_dirty = 1;
#endif

  /* particle-wall candidates, in (gid, wall id) order */
  int64_t cap = 64, cnt = 0;
  ora_wpair* W = (ora_wpair*)malloc(sizeof(ora_wpair) * (size_t)cap);
  if (!W) return ORA_ENOMEM;
  int64_t old = 0;
  const double t_search = (double)s->step * s->cfg.dt; /* walls where they are now */
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->active[i]) continue;
    for (int w = 0; w < s->nw; ++w) {
      if (s->walls[w].kind == 3) continue;
      ora_wgeo g;
      const ora_wall Wt = wall_at(&s->walls[w], t_search);
      wall_geometry(&Wt, &s->x[3 * i], s->R[i], s->skin, &g);
      if (!g.candidate) continue;
      if (cnt == cap) {
        cap *= 2;
        ora_wpair* Q = (ora_wpair*)realloc(W, sizeof(ora_wpair) * (size_t)cap);
        if (!Q) {
          free(W);
          return ORA_ENOMEM;
        }
        W = Q;
      }
      W[cnt].i = i;
      W[cnt].w = w;
      W[cnt].dt[0] = W[cnt].dt[1] = W[cnt].dt[2] = 0.0;
      while (old < s->nwpairs && (s->wpairs[old].i < i ||
                                  (s->wpairs[old].i == i && s->wpairs[old].w < w)))
        ++old;
      if (old < s->nwpairs && s->wpairs[old].i == i && s->wpairs[old].w == w)
        memcpy(W[cnt].dt, s->wpairs[old].dt, sizeof(double) * 3);
      ++cnt;
    }
  }
  free(s->wpairs);
  s->wpairs = W;
  s->nwpairs = cnt;

  /* particle-triangle candidates of mesh walls, in (gid, wall, triangle)
     order, every triangle of the mesh tested */
  int64_t mcap = 64, mcnt = 0, mold = 0;
  ora_mpair* Mp = (ora_mpair*)malloc(sizeof(ora_mpair) * (size_t)mcap);
  if (!Mp) return ORA_ENOMEM;
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->active[i]) continue;
    for (int w = 0; w < s->nw; ++w) {
      const ora_wall* Wm = &s->walls[w];
      if (Wm->kind != 3) continue;
      for (int64_t tr = Wm->tri_begin; tr < Wm->tri_begin + Wm->ntri; ++tr) {
        ora_trigeo g;
        triangle_closest(&s->tris[tr], Wm->vel, t_search, &s->x[3 * i], &g);
        if (!triangle_candidate(&g, s->R[i], s->skin)) continue;
        if (mcnt == mcap) {
          mcap *= 2;
          ora_mpair* Q = (ora_mpair*)realloc(Mp, sizeof(ora_mpair) * (size_t)mcap);
          if (!Q) {
            free(Mp);
            return ORA_ENOMEM;
          }
          Mp = Q;
        }
        Mp[mcnt].i = i;
        Mp[mcnt].w = w;
        Mp[mcnt].tri = tr;
        Mp[mcnt].dt[0] = Mp[mcnt].dt[1] = Mp[mcnt].dt[2] = 0.0;
        /* triangles are numbered in wall order, so (i, tri) orders the list */
        while (mold < s->nmpairs && (s->mpairs[mold].i < i ||
                                     (s->mpairs[mold].i == i && s->mpairs[mold].tri < tr)))
          ++mold;
        if (mold < s->nmpairs && s->mpairs[mold].i == i && s->mpairs[mold].tri == tr)
          memcpy(Mp[mcnt].dt, s->mpairs[mold].dt, sizeof(double) * 3);
        ++mcnt;
      }
    }
  }
  free(s->mpairs);
  s->mpairs = Mp;
  s->nmpairs = mcnt;
  return ORA_OK;
}

/* ------------------------------------------------------------------ forces */

#ifdef ORA_PARALLEL
/* Timing build (benchmark CPU baseline, not the parity oracle): the law of
   every pair runs in parallel into a per-pair record, then every particle
   sums its records, first those where it is the pair's first particle, then
   those where it is the second, each in list order.  That order does not
   depend on the number of threads, so the result is deterministic; it
   differs from the serial oracle's by summation order only. */
static int par_index(ora_sim* s) {
  const int64_t n = s->n, np = s->npairs;
  if (!s->idx_dirty && s->idx_n == n && s->idx_pairs == np) return ORA_OK;
  free(s->ifirst);
  free(s->jfirst);
  free(s->jlist);
  s->ifirst = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  s->jfirst = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  s->jlist = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
  if (!s->ifirst || !s->jfirst || !s->jlist) return ORA_ENOMEM;
  for (int64_t p = 0; p < np; ++p) {
    s->ifirst[s->pairs[p].i + 1] += 1;
    s->jfirst[s->pairs[p].j + 1] += 1;
  }
  for (int64_t q = 0; q < n; ++q) {
    s->ifirst[q + 1] += s->ifirst[q];
    s->jfirst[q + 1] += s->jfirst[q];
  }
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) return ORA_ENOMEM;
  memcpy(fill, s->jfirst, sizeof(int64_t) * (size_t)n);
  for (int64_t p = 0; p < np; ++p) s->jlist[fill[s->pairs[p].j]++] = p;
  free(fill);
  if (s->prec_cap < np) {
    free(s->prec);
    s->prec = (double*)malloc(sizeof(double) * 11 * (size_t)np);
    if (!s->prec) return ORA_ENOMEM;
    s->prec_cap = np;
  }
  s->idx_n = n;
  s->idx_pairs = np;
  s->idx_dirty = 0;
  return ORA_OK;
}

static void par_pair_forces(ora_sim* s) {
  const int64_t np = s->npairs, n = s->n;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < np; ++p) {
    int64_t i = s->pairs[p].i, j = s->pairs[p].j;
    double* r = &s->prec[11 * p];
    pp_contact(s, &s->x[3 * i], &s->x[3 * j], &s->v[3 * i], &s->v[3 * j], &s->w[3 * i],
               &s->w[3 * j], s->R[i], s->R[j], s->m[i], s->m[j], s->type[i], s->type[j],
               s->pairs[p].dt, r, r + 3, r + 6, r + 9);
    memcpy(s->pairs[p].f, r, sizeof(double) * 3);
  }
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n; ++q) {
    for (int64_t p = s->ifirst[q]; p < s->ifirst[q + 1]; ++p) {
      const double* r = &s->prec[11 * p];
      for (int k = 0; k < 3; ++k) {
        s->F[3 * q + k] += r[k];
        s->T[3 * q + k] += r[3 + k];
      }
      s->S[q] += r[9];
      s->S2[q] += r[10];
    }
    for (int64_t m = s->jfirst[q]; m < s->jfirst[q + 1]; ++m) {
      const double* r = &s->prec[11 * s->jlist[m]];
      for (int k = 0; k < 3; ++k) {
        s->F[3 * q + k] -= r[k];
        s->T[3 * q + k] += r[6 + k];
      }
      s->S[q] += r[9];
      s->S2[q] += r[10];
    }
  }
}
#endif

static void compute_forces(ora_sim* s, double t) {
  size_t n3 = 3 * (size_t)s->n;
  memset(s->F, 0, sizeof(double) * n3);
  memset(s->T, 0, sizeof(double) * n3);
  memset(s->S, 0, sizeof(double) * (size_t)s->n);
  memset(s->S2, 0, sizeof(double) * (size_t)s->n);
#ifdef ORA_PARALLEL
  const int64_t serial_pairs = par_index(s) == ORA_OK ? 0 : s->npairs;
  if (serial_pairs == 0) par_pair_forces(s);
  for (int64_t p = 0; p < serial_pairs; ++p) {
#else
  for (int64_t p = 0; p < s->npairs; ++p) {
#endif
    int64_t i = s->pairs[p].i, j = s->pairs[p].j;
    double Fi[3], Mi[3], Mj[3], fm[2];
    pp_contact(s, &s->x[3 * i], &s->x[3 * j], &s->v[3 * i], &s->v[3 * j], &s->w[3 * i],
               &s->w[3 * j], s->R[i], s->R[j], s->m[i], s->m[j], s->type[i], s->type[j],
               s->pairs[p].dt, Fi, Mi, Mj, fm);
    memcpy(s->pairs[p].f, Fi, sizeof(Fi));
    for (int k = 0; k < 3; ++k) {
      s->F[3 * i + k] += Fi[k];
      s->F[3 * j + k] -= Fi[k];
      s->T[3 * i + k] += Mi[k];
      s->T[3 * j + k] += Mj[k];
    }
    s->S[i] += fm[0];
    s->S[j] += fm[0];
    s->S2[i] += fm[1];
    s->S2[j] += fm[1];
  }
  for (int64_t p = 0; p < s->nwpairs; ++p) {
    int64_t i = s->wpairs[p].i;
    double Fi[3], Mi[3], fm[2];
    pw_contact(s, &s->walls[s->wpairs[p].w], t, &s->x[3 * i], &s->v[3 * i], &s->w[3 * i],
               s->R[i], s->m[i], s->type[i], s->wpairs[p].dt, Fi, Mi, fm);
    for (int k = 0; k < 3; ++k) {
      s->F[3 * i + k] += Fi[k];
      s->T[3 * i + k] += Mi[k];
    }
    s->S[i] += fm[0];
    s->S2[i] += fm[1];
  }
  /* mesh walls: the candidates of one particle and one mesh together */
  for (int64_t p = 0; p < s->nmpairs;) {
    int64_t q = p + 1;
    while (q < s->nmpairs && s->mpairs[q].i == s->mpairs[p].i &&
           s->mpairs[q].w == s->mpairs[p].w)
      ++q;
    mesh_contacts(s, &s->walls[s->mpairs[p].w], t, &s->mpairs[p], q - p);
    p = q;
  }
}

/* ------------------------------------------------------------------- steps */

static void kick(ora_sim* s, double h) {
#ifdef ORA_PARALLEL
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->active[i]) continue;
    for (int k = 0; k < 3; ++k) {
      double a = s->F[3 * i + k] / s->m[i] + s->cfg.gravity[k];
      s->v[3 * i + k] = s->v[3 * i + k] + a * h;
      s->w[3 * i + k] = s->w[3 * i + k] + (s->T[3 * i + k] / s->I[i]) * h;
    }
  }
}

static void drift(ora_sim* s, double dt) {
#ifdef ORA_PARALLEL
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->active[i]) continue;
    for (int k = 0; k < 3; ++k) s->x[3 * i + k] = s->x[3 * i + k] + s->v[3 * i + k] * dt;
  }
}

static int one_step(ora_sim* s) {
  double dt = s->cfg.dt;
  int K = s->cfg.rebuild_interval;
  if (s->cfg.integrator == 0) {
    /* velocity Verlet, Eqs. (halfstep)-(newvv) */
    double h = 0.5 * dt;
    kick(s, h);
    drift(s, dt);
    s->step += 1;
    if (s->step % K == 0) {
      int rc = rebuild(s);
      if (rc) return rc;
    }
    compute_forces(s, (double)s->step * dt);
    kick(s, h);
  } else {
    /* explicit Euler, Eq. (integ_EE): forces at step n, then x with v^n */
    compute_forces(s, (double)s->step * dt);
    for (int64_t i = 0; i < s->n; ++i) {
      if (!s->active[i]) continue;
      for (int k = 0; k < 3; ++k) {
        double a = s->F[3 * i + k] / s->m[i] + s->cfg.gravity[k];
        s->x[3 * i + k] = s->x[3 * i + k] + s->v[3 * i + k] * dt;
        s->v[3 * i + k] = s->v[3 * i + k] + a * dt;
        s->w[3 * i + k] = s->w[3 * i + k] + (s->T[3 * i + k] / s->I[i]) * dt;
      }
    }
    s->step += 1;
    if (s->step % K == 0) {
      int rc = rebuild(s);
      if (rc) return rc;
    }
  }
  return ORA_OK;
}

/* --------------------------------------------------------------- interface */

int ora_create(const ora_config* cfg, ora_sim** out) {
  if (!cfg || !out) return ORA_EINVAL;
  if (!(cfg->dt > 0.0) || cfg->rebuild_interval < 1 || cfg->integrator < 0 ||
      cfg->integrator > 1 || cfg->rolling_model < 0 || cfg->rolling_model > 2 ||
      cfg->contact_model < 0 || cfg->contact_model > 1)
    return ORA_EINVAL;
  if (cfg->contact_model == 1 && !(cfg->characteristic_velocity > 0.0)) return ORA_EINVAL;
  if (!(cfg->neighbor_threshold >= 1.0)) return ORA_EINVAL;
  if (!(cfg->cell_factor >= 1.0)) return ORA_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!(cfg->domain_hi[k] > cfg->domain_lo[k])) return ORA_EINVAL;
  ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
  if (!s) return ORA_ENOMEM;
  s->cfg = *cfg;
  *out = s;
  return ORA_OK;
}

static void free_particles(ora_sim* s) {
  free(s->x); free(s->v); free(s->w); free(s->R); free(s->m); free(s->I);
  free(s->F); free(s->T); free(s->S); free(s->S2); free(s->xref); free(s->type); free(s->active);
  free(s->pairs); free(s->wpairs); free(s->mpairs);
  s->x = s->v = s->w = s->R = s->m = s->I = s->F = s->T = s->S = s->S2 = s->xref = NULL;
  s->type = NULL; s->active = NULL; s->pairs = NULL; s->wpairs = NULL; s->mpairs = NULL;
  s->npairs = s->nwpairs = s->nmpairs = 0;
#ifdef ORA_PARALLEL
  free(s->prec); free(s->ifirst); free(s->jfirst); free(s->jlist);
  s->prec = NULL; s->ifirst = s->jfirst = s->jlist = NULL;
  s->prec_cap = 0;
  s->idx_dirty = 1;
#endif
}

void ora_destroy(ora_sim* s) {
  if (!s) return;
  free_particles(s);
  free(s->tris);
  free(s);
}

int ora_set_material(ora_sim* s, int32_t type, const ora_material* m) {
  if (!s || !m || type < 0 || type >= ORA_MAX_TYPES) return ORA_EINVAL;
  if (!(m->density > 0.0) || !(m->youngs > 0.0) || !(m->poisson > -1.0 && m->poisson < 0.5) ||
      !(m->restitution > 0.0 && m->restitution <= 1.0) || !(m->friction >= 0.0) ||
      !(m->rolling_friction >= 0.0))
    return ORA_EINVAL;
  s->mat[type] = *m;
  s->mat_set[type] = 1;
  return ORA_OK;
}

int ora_set_particles(ora_sim* s, int64_t n, const double* pos, const double* vel,
                      const double* omega, const double* radius, const int32_t* type) {
  if (!s || n < 0 || (n > 0 && (!pos || !radius))) return ORA_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (!(radius[i] > 0.0)) return ORA_EINVAL;
    int t = type ? type[i] : 0;
    if (t < 0 || t >= ORA_MAX_TYPES || !s->mat_set[t]) return ORA_EINVAL;
  }
  for (int w = 0; w < s->nw; ++w)
    if (!s->mat_set[s->walls[w].material]) return ORA_EINVAL;
  free_particles(s);
  size_t n3 = 3 * (size_t)(n > 0 ? n : 1), n1 = (size_t)(n > 0 ? n : 1);
  s->n = n;
  s->x = (double*)calloc(n3, sizeof(double));
  s->v = (double*)calloc(n3, sizeof(double));
  s->w = (double*)calloc(n3, sizeof(double));
  s->F = (double*)calloc(n3, sizeof(double));
  s->T = (double*)calloc(n3, sizeof(double));
  s->xref = (double*)calloc(n3, sizeof(double));
  s->R = (double*)calloc(n1, sizeof(double));
  s->m = (double*)calloc(n1, sizeof(double));
  s->I = (double*)calloc(n1, sizeof(double));
  s->S = (double*)calloc(n1, sizeof(double));
  s->S2 = (double*)calloc(n1, sizeof(double));
  s->type = (int32_t*)calloc(n1, sizeof(int32_t));
  s->active = (uint8_t*)calloc(n1, 1);
  if (!s->x || !s->v || !s->w || !s->F || !s->T || !s->xref || !s->R || !s->m || !s->I ||
      !s->S || !s->S2 || !s->type || !s->active) {
    free_particles(s);
    return ORA_ENOMEM;
  }
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      s->x[3 * i + k] = pos[3 * i + k];
      s->v[3 * i + k] = vel ? vel[3 * i + k] : 0.0;
      s->w[3 * i + k] = omega ? omega[3 * i + k] : 0.0;
    }
    s->R[i] = radius[i];
    s->type[i] = type ? type[i] : 0;
    double R = radius[i];
    s->m[i] = s->mat[s->type[i]].density * (4.0 / 3.0) * PI * R * R * R;
    s->I[i] = 0.4 * s->m[i] * R * R;
    s->active[i] = 1;
    if (R > rmax) rmax = R;
  }
  s->dmax = 2.0 * rmax;
  double f = s->cfg.neighbor_threshold < s->cfg.cell_factor ? s->cfg.neighbor_threshold
                                                            : s->cfg.cell_factor;
  s->rs = f * s->dmax;
  s->rs2 = s->rs * s->rs;
  s->h = s->cfg.cell_factor * s->dmax * (1.0 + 1e-9);
  s->skin = s->rs - s->dmax;
  for (int k = 0; k < 3; ++k) {
    double span = s->cfg.domain_hi[k] - s->cfg.domain_lo[k];
    int64_t c = (int64_t)ceil(span / (s->h > 0.0 ? s->h : 1.0));
    s->nc[k] = c < 1 ? 1 : c;
  }
  /* a moving wall may travel at most half the skin between two searches:
     with the particles' half skin, no contact is missed */
  for (int w = 0; w < s->nw; ++w) {
    double vw = vnorm(s->walls[w].vel);
    if (vw > 0.0 && !(vw * (double)s->cfg.rebuild_interval * s->cfg.dt <= 0.5 * s->skin))
      return ORA_EINVAL;
  }
  s->step = 0;
  s->ready = 0;
  int rc = rebuild(s);
  if (rc) return rc;
  s->ready = 1;
  return ORA_OK;
}

static int unit3(const double* a, double* out) {
  double nn = vnorm(a);
  if (!(nn > 0.0) || !isfinite(nn)) return ORA_EINVAL;
  for (int k = 0; k < 3; ++k) out[k] = a[k] / nn;
  return ORA_OK;
}

int ora_add_plane(ora_sim* s, const double point[3], const double normal[3],
                  const double* extent, int32_t material, const double axis_point[3],
                  const double omega[3], double t_on, double t_off, int32_t* wall_id) {
  if (!s || !point || !normal || s->nw >= ORA_MAX_WALLS) return ORA_EINVAL;
  if (material < 0 || material >= ORA_MAX_TYPES || !s->mat_set[material]) return ORA_EINVAL;
  if (s->n > 0) return ORA_ESTATE; /* walls are added before the particles */
  ora_wall W;
  memset(&W, 0, sizeof(W));
  W.kind = 0;
  if (unit3(normal, W.nrm)) return ORA_EINVAL;
  if (extent) {
    double d = vdot(extent, W.nrm);
    double u[3] = {extent[0] - d * W.nrm[0], extent[1] - d * W.nrm[1],
                   extent[2] - d * W.nrm[2]};
    if (unit3(u, W.u)) return ORA_EINVAL;
    vcross(W.nrm, W.u, W.vax);
    W.hu = extent[3];
    W.hv = extent[4];
    if (!(W.hu > 0.0 && W.hv > 0.0)) return ORA_EINVAL;
    W.bounded = 1;
  }
  for (int k = 0; k < 3; ++k) {
    W.p[k] = point[k];
    W.omega[k] = omega ? omega[k] : 0.0;
    W.ax[k] = axis_point ? axis_point[k] : point[k];
  }
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  s->walls[s->nw] = W;
  if (wall_id) *wall_id = s->nw;
  s->nw += 1;
  return ORA_OK;
}

int ora_add_cylinder(ora_sim* s, const double axis_point[3], const double axis_dir[3],
                     double radius, double s_min, double s_max, int32_t inside,
                     int32_t material, double omega, double t_on, double t_off,
                     int32_t* wall_id) {
  if (!s || !axis_point || !axis_dir || s->nw >= ORA_MAX_WALLS) return ORA_EINVAL;
  if (material < 0 || material >= ORA_MAX_TYPES || !s->mat_set[material]) return ORA_EINVAL;
  if (!(radius > 0.0) || !(s_max >= s_min)) return ORA_EINVAL;
  if (s->n > 0) return ORA_ESTATE;
  ora_wall W;
  memset(&W, 0, sizeof(W));
  W.kind = 1;
  if (unit3(axis_dir, W.nrm)) return ORA_EINVAL;
  for (int k = 0; k < 3; ++k) {
    W.p[k] = axis_point[k];
    W.ax[k] = axis_point[k];
    W.omega[k] = omega * W.nrm[k];
  }
  W.radius = radius;
  W.smin = s_min;
  W.smax = s_max;
  W.inside = inside ? 1 : 0;
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  s->walls[s->nw] = W;
  if (wall_id) *wall_id = s->nw;
  s->nw += 1;
  return ORA_OK;
}

int ora_add_cone(ora_sim* s, const double axis_point[3], const double axis_dir[3],
                 double radius0, double slope, double s_min, double s_max, int32_t inside,
                 int32_t material, double omega, double t_on, double t_off, int32_t* wall_id) {
  if (!s || !axis_point || !axis_dir || s->nw >= ORA_MAX_WALLS) return ORA_EINVAL;
  if (material < 0 || material >= ORA_MAX_TYPES || !s->mat_set[material]) return ORA_EINVAL;
  if (!(s_max >= s_min) || !isfinite(slope)) return ORA_EINVAL;
  /* the surface must stay away from the axis over the whole range */
  if (!(radius0 + slope * s_min > 0.0) || !(radius0 + slope * s_max > 0.0)) return ORA_EINVAL;
  if (s->n > 0) return ORA_ESTATE;
  ora_wall W;
  memset(&W, 0, sizeof(W));
  W.kind = 2;
  if (unit3(axis_dir, W.nrm)) return ORA_EINVAL;
  for (int k = 0; k < 3; ++k) {
    W.p[k] = axis_point[k];
    W.ax[k] = axis_point[k];
    W.omega[k] = omega * W.nrm[k];
  }
  W.radius = radius0;
  W.slope = slope;
  W.smin = s_min;
  W.smax = s_max;
  W.inside = inside ? 1 : 0;
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  s->walls[s->nw] = W;
  if (wall_id) *wall_id = s->nw;
  s->nw += 1;
  return ORA_OK;
}

int ora_add_mesh(ora_sim* s, int64_t n_vertices, const double* vertices, int64_t n_triangles,
                 const int32_t* triangles, int32_t material, const double axis_point[3],
                 const double omega[3], double t_on, double t_off, int32_t* wall_id) {
  if (!s || !vertices || !triangles || s->nw >= ORA_MAX_WALLS) return ORA_EINVAL;
  if (n_vertices < 3 || n_triangles < 1 || n_vertices > ((int64_t)1 << 30)) return ORA_EINVAL;
  if (material < 0 || material >= ORA_MAX_TYPES || !s->mat_set[material]) return ORA_EINVAL;
  if (s->n > 0) return ORA_ESTATE;
  for (int64_t k = 0; k < 3 * n_vertices; ++k)
    if (!isfinite(vertices[k])) return ORA_EINVAL;
  ora_tri* T = (ora_tri*)realloc(s->tris, sizeof(ora_tri) * (size_t)(s->ntris + n_triangles));
  if (!T) return ORA_ENOMEM;
  s->tris = T;
  for (int64_t f = 0; f < n_triangles; ++f) {
    ora_tri* t = &s->tris[s->ntris + f];
    for (int c = 0; c < 3; ++c) {
      const int32_t v = triangles[3 * f + c];
      if (v < 0 || v >= n_vertices) return ORA_EINVAL;
      t->v[c] = v;
      for (int k = 0; k < 3; ++k) t->p[c][k] = vertices[3 * (int64_t)v + k];
    }
    /* no degenerate triangles: the normal must exist */
    double e01[3], e02[3], N[3];
    vsub(t->p[1], t->p[0], e01);
    vsub(t->p[2], t->p[0], e02);
    vcross(e01, e02, N);
    const double len = vnorm(N);
    if (!(len > 0.0) || !isfinite(len)) return ORA_EINVAL;
  }
  ora_wall W;
  memset(&W, 0, sizeof(W));
  W.kind = 3;
  for (int k = 0; k < 3; ++k) {
    W.p[k] = vertices[k];
    W.ax[k] = axis_point ? axis_point[k] : vertices[k];
    W.omega[k] = omega ? omega[k] : 0.0;
  }
  W.material = material;
  W.t_on = t_on;
  W.t_off = t_off;
  W.tri_begin = s->ntris;
  W.ntri = n_triangles;
  s->ntris += n_triangles;
  s->walls[s->nw] = W;
  if (wall_id) *wall_id = s->nw;
  s->nw += 1;
  return ORA_OK;
}

int ora_triangle_closest(const double corners[9], const double x[3], double out[6]) {
  if (!corners || !x || !out) return ORA_EINVAL;
  ora_tri T;
  for (int c = 0; c < 3; ++c) {
    T.v[c] = c;
    for (int k = 0; k < 3; ++k) T.p[c][k] = corners[3 * c + k];
  }
  const double zero[3] = {0.0, 0.0, 0.0};
  ora_trigeo g;
  triangle_closest(&T, zero, 0.0, x, &g);
  out[0] = g.feature == 0 ? 0.0 : (g.feature == 1 ? 1.0 + g.a : 4.0 + g.a);
  out[1] = g.s;
  out[2] = g.d2;
  for (int k = 0; k < 3; ++k) out[3 + k] = g.q[k];
  return ORA_OK;
}

int ora_set_wall_velocity(ora_sim* s, int32_t wall_id, const double vel[3]) {
  if (!s || !vel || wall_id < 0 || wall_id >= s->nw) return ORA_EINVAL;
  if (s->n > 0) return ORA_ESTATE;
  for (int k = 0; k < 3; ++k) {
    if (!isfinite(vel[k])) return ORA_EINVAL;
    s->walls[wall_id].vel[k] = vel[k];
  }
  return ORA_OK;
}

int ora_step(ora_sim* s, int64_t n_steps) {
  if (!s || n_steps < 0) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  for (int64_t k = 0; k < n_steps; ++k) {
    int rc = one_step(s);
    if (rc) return rc;
  }
  return ORA_OK;
}

int ora_get_state(ora_sim* s, double* pos, double* vel, double* omega, uint8_t* active,
                  double* time_out) {
  if (!s) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  size_t n3 = 3 * (size_t)s->n;
  if (pos) memcpy(pos, s->x, sizeof(double) * n3);
  if (vel) memcpy(vel, s->v, sizeof(double) * n3);
  if (omega) memcpy(omega, s->w, sizeof(double) * n3);
  if (active) memcpy(active, s->active, (size_t)s->n);
  if (time_out) *time_out = (double)s->step * s->cfg.dt;
  return ORA_OK;
}

int ora_get_forces(ora_sim* s, double* force, double* torque) {
  if (!s) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  size_t n3 = 3 * (size_t)s->n;
  if (force) memcpy(force, s->F, sizeof(double) * n3);
  if (torque) memcpy(torque, s->T, sizeof(double) * n3);
  return ORA_OK;
}

int ora_get_force_scale(ora_sim* s, double* scale) {
  if (!s || !scale) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  memcpy(scale, s->S, sizeof(double) * (size_t)s->n);
  return ORA_OK;
}

int ora_get_term_scale(ora_sim* s, double* scale) {
  if (!s || !scale) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  memcpy(scale, s->S2, sizeof(double) * (size_t)s->n);
  return ORA_OK;
}

int ora_num_contacts(ora_sim* s, int64_t* n_pairs, int64_t* n_wall) {
  if (!s) return ORA_EINVAL;
  if (n_pairs) *n_pairs = s->npairs;
  if (n_wall) *n_wall = s->nwpairs;
  return ORA_OK;
}

int ora_get_contacts(ora_sim* s, int64_t cap, int64_t* pairs, double* delta_t,
                     uint8_t* touching, int64_t* n_out) {
  if (!s || cap < 0) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  if (n_out) *n_out = s->npairs;
  if (cap < s->npairs) return ORA_EINVAL;
  for (int64_t p = 0; p < s->npairs; ++p) {
    int64_t i = s->pairs[p].i, j = s->pairs[p].j;
    if (pairs) {
      pairs[2 * p] = i;
      pairs[2 * p + 1] = j;
    }
    if (delta_t) memcpy(&delta_t[3 * p], s->pairs[p].dt, sizeof(double) * 3);
    if (touching) {
      double dx[3];
      vsub(&s->x[3 * j], &s->x[3 * i], dx);
      double rsum = s->R[i] + s->R[j];
      touching[p] = vdot(dx, dx) < rsum * rsum;
    }
  }
  return ORA_OK;
}

int ora_get_contact_forces(ora_sim* s, int64_t cap, int64_t* pairs, double* force,
                           int64_t* n_out) {
  if (!s || cap < 0) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  if (n_out) *n_out = s->npairs;
  if (cap < s->npairs) return ORA_EINVAL;
  for (int64_t p = 0; p < s->npairs; ++p) {
    if (pairs) {
      pairs[2 * p] = s->pairs[p].i;
      pairs[2 * p + 1] = s->pairs[p].j;
    }
    if (force) memcpy(&force[3 * p], s->pairs[p].f, sizeof(double) * 3);
  }
  return ORA_OK;
}

int ora_get_wall_contacts(ora_sim* s, int64_t cap, int64_t* pairs, double* delta_t,
                          int64_t* n_out) {
  if (!s || cap < 0) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  if (n_out) *n_out = s->nwpairs;
  if (cap < s->nwpairs) return ORA_EINVAL;
  for (int64_t p = 0; p < s->nwpairs; ++p) {
    if (pairs) {
      pairs[2 * p] = s->wpairs[p].i;
      pairs[2 * p + 1] = s->wpairs[p].w;
    }
    if (delta_t) memcpy(&delta_t[3 * p], s->wpairs[p].dt, sizeof(double) * 3);
  }
  return ORA_OK;
}

int ora_get_mesh_contacts(ora_sim* s, int64_t cap, int64_t* triples, double* delta_t,
                          int64_t* n_out) {
  if (!s || cap < 0) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  if (n_out) *n_out = s->nmpairs;
  if (cap < s->nmpairs) return ORA_EINVAL;
  for (int64_t p = 0; p < s->nmpairs; ++p) {
    if (triples) {
      const ora_mpair* M = &s->mpairs[p];
      triples[3 * p] = M->i;
      triples[3 * p + 1] = M->w;
      triples[3 * p + 2] = M->tri - s->walls[M->w].tri_begin;
    }
    if (delta_t) memcpy(&delta_t[3 * p], s->mpairs[p].dt, sizeof(double) * 3);
  }
  return ORA_OK;
}

int ora_search_params(ora_sim* s, double* out4) {
  if (!s || !out4) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  out4[0] = s->dmax;
  out4[1] = s->rs;
  out4[2] = s->h;
  out4[3] = s->skin;
  return ORA_OK;
}

int ora_bruteforce_candidates(ora_sim* s, int64_t cap, int64_t* pairs, int64_t* n_out) {
  if (!s || cap < 0) return ORA_EINVAL;
  if (!s->ready) return ORA_ESTATE;
  int64_t cnt = 0;
  for (int64_t i = 0; i < s->n; ++i) {
    if (!s->active[i]) continue;
    for (int64_t j = i + 1; j < s->n; ++j) {
      if (!s->active[j]) continue;
      double dx[3];
      vsub(&s->x[3 * j], &s->x[3 * i], dx);
      if (vdot(dx, dx) < s->rs2) {
        if (cnt < cap && pairs) {
          pairs[2 * cnt] = i;
          pairs[2 * cnt + 1] = j;
        }
        ++cnt;
      }
    }
  }
  if (n_out) *n_out = cnt;
  return cnt > cap ? ORA_EINVAL : ORA_OK;
}

int ora_pair_force(ora_sim* s, const double xi[3], const double xj[3],
                   const double vi[3], const double vj[3], const double wi[3],
                   const double wj[3], double Ri, double Rj, int32_t ti, int32_t tj,
                   double delta_t[3], double F_i[3], double M_i[3], double M_j[3],
                   int32_t* touching) {
  if (!s || ti < 0 || tj < 0 || ti >= ORA_MAX_TYPES || tj >= ORA_MAX_TYPES ||
      !s->mat_set[ti] || !s->mat_set[tj] || !(Ri > 0.0) || !(Rj > 0.0))
    return ORA_EINVAL;
  double mi = s->mat[ti].density * (4.0 / 3.0) * PI * Ri * Ri * Ri;
  double mj = s->mat[tj].density * (4.0 / 3.0) * PI * Rj * Rj * Rj;
  double fm[2];
  int t = pp_contact(s, xi, xj, vi, vj, wi, wj, Ri, Rj, mi, mj, ti, tj, delta_t, F_i, M_i,
                     M_j, fm);
  if (touching) *touching = t;
  return ORA_OK;
}
