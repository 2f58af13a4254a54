/*
 * Dense-array FP64 lattice Boltzmann oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  It shares nothing
 * with the GPU library: no headers, tables, helpers or build steps.
 *
 * What it computes (Tomczak & Szafran, "Sparse geometries handling in lattice
 * Boltzmann method implementation for graphic processors", arXiv 1703.08015):
 *   - BGK collision, Eq. (2), relaxation time tau, viscosity (tau - 1/2)/3;
 *   - two fluid models, selected by the `model` argument:
 *       model 0, quasi-compressible: equilibrium Eq. (3) with c_s^2 = 1/3,
 *         velocity Eq. (5);
 *       model 1, incompressible: equilibrium Eq. (4), velocity Eq. (6);
 *   - the MRT collision of Eq. (8) when relaxation rates are given: the
 *     collision matrix is diagonal in an orthogonal moment basis,
 *     f* = f + M^-1 [-S M (f - f_eq) + (I - S/2) M F], with f_eq of the chosen
 *     model and the same Guo source F; with every rate equal to 1/tau this
 *     is the BGK update;
 *   - the time-discrete LBGK update, Eq. (7), with delta_x = delta_t = 1;
 *   - propagation only between non-solid nodes (Sec. 3.2), realised as
 *     link-wise half-way bounce-back decided by the source node;
 *   - the gather ("pull") form of propagation used by the two-copy tile
 *     kernel (Sec. 3, Fig. 5): the stored array holds post-collision values,
 *     a step first gathers f_i(x) = f*_i(x - c_i) and then collides.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - lattice weights and velocity ordering are the standard D2Q9 / D3Q19
 *     sets (the paper's Fig. 1 is not reproduced in text);
 *   - the body force g is an acceleration applied with Guo's forcing:
 *     u = (sum_i c_i f_i)/rho + g/2 and a source term
 *     F_i = w_i rho [3 (c_i - u).g + 9 (c_i.u)(c_i.g)] scaled by (1 - omega/2);
 *   - in the incompressible model, Eqs. (4) and (6) as printed carry no
 *     density factor on the velocity terms: the reference density is 1 in
 *     lattice units.  The same holds for the force, whose density is g, so
 *     u = sum_i c_i f_i + g/2 and F_i = w_i [3 (c_i - u).g + 9 (c_i.u)(c_i.g)];
 *   - the paper does not give the MRT matrix: the bases are the published
 *     orthogonal ones, Lallemand & Luo (PRE 61, 6546, 2000) for D2Q9 and
 *     d'Humieres et al. (Phil. Trans. R. Soc. A 360, 437, 2002) for D3Q19,
 *     written here as polynomials in the velocity c; the shear-stress
 *     moments relax with 1/tau, the others with the given rates;
 *   - a source position outside the domain on a non-periodic axis is solid;
 *   - a moving wall (the lid of a driven cavity; the paper's dense cavity
 *     workload gives no boundary rule): the domain face beyond the last (side
 *     1) or before the first (side 0) node along one non-periodic axis moves
 *     with velocity u_w; a source beyond that face returns the bounce-back
 *     value plus 6 w_i rho_w (c_i . u_w) (Ladd's moving-wall rule), with
 *     rho_w = rho0 in the quasi-compressible model and 1 in the
 *     incompressible one; the face decides also for diagonal links that
 *     cross another wall at the same time;
 *   - tau = +infinity gives omega = 0 (pure streaming, used with g = 0).
 *
 * Dense layout everywhere: f[i][z][y][x] (x fastest), mask[z][y][x] with
 * nonzero = solid.  Solid entries of f are never read and are written as 0
 * only by ora_init.  Plain loops, no blocking or fusion beyond the equations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- lattice tables (standard velocity sets and weights) ------------- */

static const int C9[9][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static const int C19[19][3] = {
    {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},   {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {
    1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
  int q;
  const int (*c)[3];
  const double *w;
  int opp[19];
} lattice_t;

static int get_lattice(int q, lattice_t *L) {
  if (q == 9) {
    L->c = C9;
    L->w = W9;
  } else if (q == 19) {
    L->c = C19;
    L->w = W19;
  } else {
    return -1;
  }
  L->q = q;
  /* the opposite direction is found by search, not assumed from the order */
  for (int i = 0; i < q; ++i) {
    L->opp[i] = -1;
    for (int j = 0; j < q; ++j)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
          L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
  }
  return 0;
}

int ora_lattice(int q, int32_t *c_out, double *w_out, int32_t *opp_out) {
  lattice_t L;
  if (get_lattice(q, &L)) return -1;
  for (int i = 0; i < q; ++i) {
    for (int a = 0; a < 3; ++a) c_out[3 * i + a] = L.c[i][a];
    w_out[i] = L.w[i];
    opp_out[i] = L.opp[i];
  }
  return 0;
}

/* ---- single-node physics -------------------------------------------- */

#define MODEL_QUASI 0
#define MODEL_INCOMPRESSIBLE 1

static int valid_model(int model) {
  return model == MODEL_QUASI || model == MODEL_INCOMPRESSIBLE;
}

/* Quasi-compressible, Eq. (3):
 *   f_eq_i = w_i rho (1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2));
 * incompressible, Eq. (4):
 *   f_eq_i = w_i (rho + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2));
 * cs2 = 1/3, i.e. coefficients 3, 9/2 and 3/2. */
static void feq(const lattice_t *L, int model, double rho, const double u[3],
                double *out) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L->q; ++i) {
    double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
    double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    if (model == MODEL_QUASI)
      out[i] = L->w[i] * rho * (1.0 + poly);
    else
      out[i] = L->w[i] * (rho + poly);
  }
}

/* Guo source term without the (1 - omega/2) prefactor:
 * F_i = w_i d [3 (c_i - u).g + 9 (c_i.u)(c_i.g)], where d is the density
 * that carries the force: rho (quasi-compressible) or 1 (incompressible). */
static void guo(const lattice_t *L, int model, double rho, const double u[3],
                const double g[3], double *out) {
  double d = model == MODEL_QUASI ? rho : 1.0;
  for (int i = 0; i < L->q; ++i) {
    double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
    double cg = L->c[i][0] * g[0] + L->c[i][1] * g[1] + L->c[i][2] * g[2];
    double cmug = (L->c[i][0] - u[0]) * g[0] + (L->c[i][1] - u[1]) * g[1] +
                  (L->c[i][2] - u[2]) * g[2];
    out[i] = L->w[i] * d * (3.0 * cmug + 9.0 * cu * cg);
  }
}

/* rho = sum f; the velocity with the half-force shift:
 * Eq. (5), u = (sum c f)/rho + g/2 (quasi-compressible), or
 * Eq. (6), u = sum c f + g/2 (incompressible). */
static void macro(const lattice_t *L, int model, const double *f,
                  const double g[3], double *rho, double u[3]) {
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < L->q; ++i) r += f[i];
  for (int i = 0; i < L->q; ++i)
    for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * f[i];
  *rho = r;
  for (int a = 0; a < 3; ++a) {
    if (model == MODEL_QUASI)
      u[a] = j[a] / r + 0.5 * g[a];
    else
      u[a] = j[a] + 0.5 * g[a];
  }
}

/* ---- MRT moment bases (Eq. 8) ---------------------------------------- */

/* Relaxation class of a moment: conserved (density, momentum), energy e,
 * energy square eps, energy flux q, shear stress (rate 1/tau), the
 * fourth-order pi moments and the third-order m moments. */
enum { CL_CONS, CL_E, CL_EPS, CL_Q, CL_NU, CL_PI, CL_M };

/* Row k of the basis evaluated at velocity c (integer for both bases). */
static double mrt_entry(int q, int k, const int c[3], int *cls) {
  const double x = c[0], y = c[1], z = c[2];
  const double c2 = x * x + y * y + z * z;
  if (q == 9) {
    /* rho, e, eps, jx, qx, jy, qy, pxx, pxy */
    switch (k) {
      case 0: *cls = CL_CONS; return 1.0;
      case 1: *cls = CL_E; return 3.0 * c2 - 4.0;
      case 2: *cls = CL_EPS; return 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
      case 3: *cls = CL_CONS; return x;
      case 4: *cls = CL_Q; return (3.0 * c2 - 5.0) * x;
      case 5: *cls = CL_CONS; return y;
      case 6: *cls = CL_Q; return (3.0 * c2 - 5.0) * y;
      case 7: *cls = CL_NU; return x * x - y * y;
      default: *cls = CL_NU; return x * y;
    }
  }
  /* rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz,
   * pxz, mx, my, mz */
  switch (k) {
    case 0: *cls = CL_CONS; return 1.0;
    case 1: *cls = CL_E; return 19.0 * c2 - 30.0;
    case 2: *cls = CL_EPS; return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: *cls = CL_CONS; return x;
    case 4: *cls = CL_Q; return (5.0 * c2 - 9.0) * x;
    case 5: *cls = CL_CONS; return y;
    case 6: *cls = CL_Q; return (5.0 * c2 - 9.0) * y;
    case 7: *cls = CL_CONS; return z;
    case 8: *cls = CL_Q; return (5.0 * c2 - 9.0) * z;
    case 9: *cls = CL_NU; return 3.0 * x * x - c2;
    case 10: *cls = CL_PI; return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: *cls = CL_NU; return y * y - z * z;
    case 12: *cls = CL_PI; return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: *cls = CL_NU; return x * y;
    case 14: *cls = CL_NU; return y * z;
    case 15: *cls = CL_NU; return x * z;
    case 16: *cls = CL_M; return (y * y - z * z) * x;
    case 17: *cls = CL_M; return (z * z - x * x) * y;
    default: *cls = CL_M; return (x * x - y * y) * z;
  }
}

static void mrt_matrix(const lattice_t *L, double M[19][19], int cls[19]) {
  for (int k = 0; k < L->q; ++k)
    for (int i = 0; i < L->q; ++i) M[k][i] = mrt_entry(L->q, k, L->c[i], &cls[k]);
}

int ora_mrt_matrix(int q, double *M_out, int32_t *cls_out) {
  lattice_t L;
  double M[19][19];
  int cls[19];
  if (get_lattice(q, &L)) return -1;
  mrt_matrix(&L, M, cls);
  for (int k = 0; k < q; ++k) {
    cls_out[k] = cls[k];
    for (int i = 0; i < q; ++i) M_out[k * q + i] = M[k][i];
  }
  return 0;
}

/* Rates of the relaxation classes: mrt = {s_e, s_eps, s_q, s_pi, s_m}; the
 * shear stress relaxes with 1/tau.  Conserved moments take rate 1: their
 * relaxation term vanishes for the density, and for the momentum the rate
 * cancels against the half-force shift of u. */
static double class_rate(int cls, double omega, const double *mrt) {
  switch (cls) {
    case CL_E: return mrt[0];
    case CL_EPS: return mrt[1];
    case CL_Q: return mrt[2];
    case CL_PI: return mrt[3];
    case CL_M: return mrt[4];
    case CL_NU: return omega;
    default: return 1.0;
  }
}

/* Eqs. (2) and (7): f* = f + omega (f_eq - f) + (1 - omega/2) F (BGK, mrt ==
 * NULL); Eq. (8) with the moment basis above otherwise. */
static void collide(const lattice_t *L, int model, const double *f, double tau,
                    const double g[3], const double *mrt, double *out) {
  double rho, u[3], fe[19], F[19];
  double omega = 1.0 / tau;
  macro(L, model, f, g, &rho, u);
  feq(L, model, rho, u, fe);
  guo(L, model, rho, u, g, F);
  if (!mrt) {
    for (int i = 0; i < L->q; ++i)
      out[i] = f[i] + omega * (fe[i] - f[i]) + (1.0 - 0.5 * omega) * F[i];
    return;
  }
  double M[19][19], y[19];
  int cls[19];
  mrt_matrix(L, M, cls);
  for (int k = 0; k < L->q; ++k) {
    double dm = 0.0, fm = 0.0, norm = 0.0;
    for (int i = 0; i < L->q; ++i) {
      dm += M[k][i] * (f[i] - fe[i]);
      fm += M[k][i] * F[i];
      norm += M[k][i] * M[k][i];
    }
    double s = class_rate(cls[k], omega, mrt);
    /* rows are orthogonal, so M^-1 = M^T diag(1/norm) */
    y[k] = (-s * dm + (1.0 - 0.5 * s) * fm) / norm;
  }
  for (int i = 0; i < L->q; ++i) {
    double acc = 0.0;
    for (int k = 0; k < L->q; ++k) acc += M[k][i] * y[k];
    out[i] = f[i] + acc;
  }
}

int ora_feq(int q, int model, double rho, const double *u, double *out) {
  lattice_t L;
  if (get_lattice(q, &L) || !valid_model(model)) return -1;
  feq(&L, model, rho, u, out);
  return 0;
}

int ora_guo(int q, int model, double rho, const double *u, const double *g,
            double *out) {
  lattice_t L;
  if (get_lattice(q, &L) || !valid_model(model)) return -1;
  guo(&L, model, rho, u, g, out);
  return 0;
}

int ora_collide(int q, int model, const double *f, double tau, const double *g,
                const double *mrt, double *out) {
  lattice_t L;
  if (get_lattice(q, &L) || !valid_model(model)) return -1;
  collide(&L, model, f, tau, g, mrt, out);
  return 0;
}

/* ---- dense field operations ---------------------------------------- */

typedef struct {
  int n[3];
  int periodic[3];
  int64_t N;
} grid_t;

static void make_grid(const int32_t *shape, uint32_t periodic, grid_t *G) {
  for (int a = 0; a < 3; ++a) {
    G->n[a] = shape[a];
    G->periodic[a] = (periodic >> a) & 1u;
  }
  G->N = (int64_t)shape[0] * shape[1] * shape[2];
}

static int64_t node_index(const grid_t *G, int x, int y, int z) {
  return ((int64_t)z * G->n[1] + y) * G->n[0] + x;
}

/* Position of x - c_i, or -1 when it lies outside a non-periodic axis. */
static int64_t source_of(const grid_t *G, const int p[3], const int c[3]) {
  int s[3];
  for (int a = 0; a < 3; ++a) {
    s[a] = p[a] - c[a];
    if (s[a] < 0 || s[a] >= G->n[a]) {
      if (!G->periodic[a]) return -1;
      s[a] = (s[a] % G->n[a] + G->n[a]) % G->n[a];
    }
  }
  return node_index(G, s[0], s[1], s[2]);
}

/* Cold start (rho == NULL -> rho0, u == NULL -> 0) or given fields:
 * fluid f*_i = f_eq_i(rho, u); solid entries 0. */
int ora_init(int q, int model, const int32_t *shape, const uint8_t *mask,
             double rho0, const double *rho, const double *u, double *f) {
  lattice_t L;
  grid_t G;
  if (get_lattice(q, &L) || !valid_model(model)) return -1;
  make_grid(shape, 0u, &G);
  for (int64_t n = 0; n < G.N; ++n) {
    double fe[19], uu[3] = {0.0, 0.0, 0.0}, r = rho0;
    if (mask[n]) {
      for (int i = 0; i < q; ++i) f[i * G.N + n] = 0.0;
      continue;
    }
    if (rho) r = rho[n];
    if (u)
      for (int a = 0; a < 3; ++a) uu[a] = u[a * G.N + n];
    feq(&L, model, r, uu, fe);
    for (int i = 0; i < q; ++i) f[i * G.N + n] = fe[i];
  }
  return 0;
}

/* One pull-stream + collide pass from src into dst over fluid nodes. */
/* Moving wall: lid = {axis, side, u_x, u_y, u_z, rho_w} or NULL. */
static int beyond_lid(const grid_t *G, const double *lid, const int p[3],
                      const int c[3]) {
  if (!lid) return 0;
  int a = (int)lid[0], side = (int)lid[1];
  int s = p[a] - c[a];
  return side ? s >= G->n[a] : s < 0;
}

static void one_step(const lattice_t *L, int model, const grid_t *G,
                     const uint8_t *mask, double tau, const double g[3],
                     const double *mrt, const double *lid, const double *src,
                     double *dst, int nthreads) {
  (void)nthreads;
#pragma omp parallel for num_threads(nthreads) collapse(2) schedule(static)
  for (int z = 0; z < G->n[2]; ++z) {
    for (int y = 0; y < G->n[1]; ++y) {
      for (int x = 0; x < G->n[0]; ++x) {
        int p[3] = {x, y, z};
        int64_t n = node_index(G, x, y, z);
        double f[19], out[19];
        if (mask[n]) continue;
        for (int i = 0; i < L->q; ++i) {
          int64_t s = source_of(G, p, L->c[i]);
          if (s >= 0 && !mask[s]) {
            f[i] = src[i * G->N + s];
          } else {
            f[i] = src[L->opp[i] * G->N + n]; /* half-way bounce-back */
            if (beyond_lid(G, lid, p, L->c[i])) {
              double cu = L->c[i][0] * lid[2] + L->c[i][1] * lid[3] +
                          L->c[i][2] * lid[4];
              f[i] += 6.0 * L->w[i] * lid[5] * cu;
            }
          }
        }
        collide(L, model, f, tau, g, mrt, out);
        for (int i = 0; i < L->q; ++i) dst[i * G->N + n] = out[i];
      }
    }
  }
}

/* nsteps time steps; f holds post-collision values on entry and on return.
 * tmp is caller scratch of the same size as f. */
int ora_step(int q, int model, const int32_t *shape, uint32_t periodic,
             const uint8_t *mask, double tau, const double *g,
             const double *mrt, const double *lid, double *f, double *tmp,
             int64_t nsteps, int nthreads) {
  lattice_t L;
  grid_t G;
  if (get_lattice(q, &L) || !valid_model(model)) return -1;
  if (nthreads < 1) nthreads = 1;
  make_grid(shape, periodic, &G);
  if (lid) {
    int a = (int)lid[0];
    if (a < 0 || a > 2 || G.periodic[a] || (lid[1] != 0.0 && lid[1] != 1.0))
      return -1; /* a lid sits on a face of a non-periodic axis */
  }
  /* solid entries of tmp mirror f so that the result is complete either way */
  memcpy(tmp, f, sizeof(double) * (size_t)q * (size_t)G.N);
  double *a = f, *b = tmp;
  for (int64_t t = 0; t < nsteps; ++t) {
    one_step(&L, model, &G, mask, tau, g, mrt, lid, a, b, nthreads);
    double *s = a;
    a = b;
    b = s;
  }
  if (a != f) memcpy(f, a, sizeof(double) * (size_t)q * (size_t)G.N);
  return 0;
}

/* Macroscopic fields of the stored post-collision state:
 * rho = sum f*, u = (sum c f*)/rho - g/2 (quasi-compressible) or
 * u = sum c f* - g/2 (incompressible): equal to the step's Guo velocity
 * because the collision adds the force density (rho g or g) to the first
 * moment.  Solid nodes: 0. */
int ora_moments(int q, int model, const int32_t *shape, const uint8_t *mask,
                const double *g, const double *f, double *rho, double *u) {
  lattice_t L;
  grid_t G;
  if (get_lattice(q, &L) || !valid_model(model)) return -1;
  make_grid(shape, 0u, &G);
  for (int64_t n = 0; n < G.N; ++n) {
    if (mask[n]) {
      rho[n] = 0.0;
      for (int a = 0; a < 3; ++a) u[a * G.N + n] = 0.0;
      continue;
    }
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) r += f[i * G.N + n];
    for (int i = 0; i < q; ++i)
      for (int a = 0; a < 3; ++a) j[a] += L.c[i][a] * f[i * G.N + n];
    rho[n] = r;
    for (int a = 0; a < 3; ++a) {
      if (model == MODEL_QUASI)
        u[a * G.N + n] = j[a] / r - 0.5 * g[a];
      else
        u[a * G.N + n] = j[a] - 0.5 * g[a];
    }
  }
  return 0;
}
