/*
 * lbm_oracle.c -- plain, slow, FP64 CPU oracle for the moment-represented
 * regularized lattice Boltzmann step of Lauricella et al. (arXiv 2609.09160).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes.  The moment form of the paper (Eq. (7) followed by the
 * correction of Eq. (8)) is, by construction, a population-based regularized
 * LBM whose populations are never stored: Eq. (7) is Eq. (3) with the
 * populations expanded on the second-order Hermite basis (Eqs. (4)-(6)) and
 * projected back (Eq. (5)).  This oracle therefore stores the populations
 * f_i explicitly (Q per site) and performs, per step:
 *   1. moments of f (Eq. (5)), corrected as in Eq. (8):
 *        p* = sum f,  u = sum c f + F/(2 rho),
 *        a2 = sum H2 f + (F u + u F)/(2 rho);
 *   2. the non-equilibrium part a2neq = a2 - u u (Eq. (6): the equilibrium
 *      coefficients are p*, u, u u and only a2 has a non-equilibrium part);
 *   3. the regularized post-collision population (Eq. (3) with Eq. (4)):
 *        f_i* = feq_i + (1 - omega) fneq_i + S_i / 2,
 *      feq_i, fneq_i from the truncated Hermite series of Eq. (4), S_i the
 *      Guo term of Eq. (9) written as printed;
 *   4. streaming by pull, f_i(x, t+1) = f_i*(x - c_i); on an axis with walls
 *      a source beyond the wall is replaced by the bounce-back value
 *      f_{-i}*(x) (stationary halfway bounce-back; the paper names no-slip
 *      walls in section 4 but no scheme, so this is a reading).
 * rho = 1 (one component, section 2: rho(phi) with equal phase densities).
 *
 * D3Q27h (lattice code 270): the D3Q27 velocity set with the series of
 * Eq. (4) run over the complete Hermite basis of D3Q27 instead of stopping at
 * second order (section 2, the paragraph after Eq. (9)): the coefficients of
 * orders 3 to 6 are rebuilt from u and a2neq by the recursive closures the
 * paper cites (Shan, Yuan and Chen 2006 for the equilibrium, Malaspinas 2015
 * for the non-equilibrium part); everything else is as above.
 *
 * Everything is written with generic loops over directions and tensor
 * indices so that it can be checked against the equations by eye.  The
 * velocity sets are the textbook D3Q19 / D3Q27 (the paper defers to the
 * textbooks for them): all c in {-1,0,1}^3 (|c|^2 <= 2 for D3Q19), weights by
 * |c|^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0)

/* Number of OpenMP threads a parallel loop of this library will use. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set the number of OpenMP threads for later parallel loops (n >= 1). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Build the velocity set: enumerate {-1,0,1}^3, keep |c|^2 <= 2 for Q=19.
 * Returns Q, or -1 for an unknown Q. */
#define D3Q27H 270

int oracle_lattice(int Q, int* c, double* w) {
  double wt[4];
  int maxc2;
  if (Q == D3Q27H) Q = 27; /* same velocity set, complete Hermite basis */
  if (Q == 19) {
    wt[0] = 1.0 / 3.0; wt[1] = 1.0 / 18.0; wt[2] = 1.0 / 36.0; wt[3] = 0.0;
    maxc2 = 2;
  } else if (Q == 27) {
    wt[0] = 8.0 / 27.0; wt[1] = 2.0 / 27.0; wt[2] = 1.0 / 54.0; wt[3] = 1.0 / 216.0;
    maxc2 = 3;
  } else {
    return -1;
  }
  int q = 0;
  for (int cz = -1; cz <= 1; ++cz)
    for (int cy = -1; cy <= 1; ++cy)
      for (int cx = -1; cx <= 1; ++cx) {
        int c2 = cx * cx + cy * cy + cz * cz;
        if (c2 > maxc2) continue;
        c[3 * q + 0] = cx; c[3 * q + 1] = cy; c[3 * q + 2] = cz;
        w[q] = wt[c2];
        ++q;
      }
  return q;
}

/* D3Q27h: the components of orders 3..6 of the complete basis */
#define NHIGH 17

typedef struct {
  int Q;
  int high; /* D3Q27h: complete Hermite basis in the reconstruction */
  int c[27][3];
  double w[27];
  int opp[27];
  /* D3Q27h: per high-order component b, its index tuple (order n[b]), the
   * factor (number of orderings) / (cs^(2n) n!) of Eq. (4), and H_b(c_i) */
  int hn[NHIGH];
  int hidx[NHIGH][6];
  double hfac[NHIGH];
  double hH[NHIGH][27];
} lattice_t;

static void make_high_order_table(lattice_t* L);

static int make_lattice(int code, lattice_t* L) {
  int cc[81];
  const int Q = (code == D3Q27H) ? 27 : code;
  if (oracle_lattice(code, cc, L->w) != Q) return -1;
  L->Q = Q;
  L->high = (code == D3Q27H);
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < 3; ++a) L->c[i][a] = cc[3 * i + a];
  for (int i = 0; i < Q; ++i) {
    L->opp[i] = -1;
    for (int j = 0; j < Q; ++j)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
          L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
  }
  if (L->high) make_high_order_table(L);
  return 0;
}

/* Hermite basis of section 2: H0 = 1, H1_a = c_a, H2_ab = c_a c_b - cs^2 d_ab */
static double H2(const lattice_t* L, int i, int a, int b) {
  return (double)(L->c[i][a] * L->c[i][b]) - (a == b ? CS2 : 0.0);
}

/* Step 1 and 2 at one site: corrected moments of Eq. (8) from populations.
 * m = [p*, u(3), a2xx, a2yy, a2zz, a2xy, a2xz, a2yz]. */
static void site_moments(const lattice_t* L, const double* fs, const double F[3],
                         double rho, double m[10]) {
  double p = 0.0, j[3] = {0, 0, 0}, P[3][3] = {{0}};
  for (int i = 0; i < L->Q; ++i) {
    p += fs[i];
    for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * fs[i];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) P[a][b] += H2(L, i, a, b) * fs[i];
  }
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = j[a] + F[a] / (2.0 * rho);
  double a2[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      a2[a][b] = P[a][b] + (F[a] * u[b] + F[b] * u[a]) / (2.0 * rho);
  m[0] = p;
  m[1] = u[0]; m[2] = u[1]; m[3] = u[2];
  m[4] = a2[0][0]; m[5] = a2[1][1]; m[6] = a2[2][2];
  m[7] = a2[0][1]; m[8] = a2[0][2]; m[9] = a2[1][2];
}

static void unpack_a2(const double m[10], double a2[3][3]) {
  a2[0][0] = m[4]; a2[1][1] = m[5]; a2[2][2] = m[6];
  a2[0][1] = a2[1][0] = m[7];
  a2[0][2] = a2[2][0] = m[8];
  a2[1][2] = a2[2][1] = m[9];
}

/* Truncated Hermite series of Eq. (4): w_i sum_n H^(n):a^(n) / (cs^(2n) n!) */
static double hermite_series(const lattice_t* L, int i, double a0, const double a1[3],
                             double a2[3][3]) {
  double s1 = 0.0, s2 = 0.0;
  for (int a = 0; a < 3; ++a) s1 += L->c[i][a] * a1[a];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) s2 += H2(L, i, a, b) * a2[a][b];
  return L->w[i] * (a0 + s1 / CS2 + s2 / (2.0 * CS2 * CS2));
}

/* Guo source term of Eq. (9), as printed:
 * S_i = w_i [ (c_a - u_a)/cs^2 + (c_b u_b) c_a / cs^4 ] F_a / rho */
static double guo_source(const lattice_t* L, int i, const double u[3], const double F[3],
                         double rho) {
  double cu = 0.0;
  for (int b = 0; b < 3; ++b) cu += L->c[i][b] * u[b];
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    s += ((L->c[i][a] - u[a]) / CS2 + cu * L->c[i][a] / (CS2 * CS2)) * F[a] / rho;
  return L->w[i] * s;
}

/* ---- D3Q27h: orders 3 to 6 of the complete Hermite basis ----
 *
 * Hermite tensor of order n at velocity c, by the standard (Grad) recursion
 *   H^(n)_{a1..an} = c_an H^(n-1)_{a1..an-1}
 *                    - cs^2 sum_{k<n} d(ak, an) H^(n-2)_{a1..an-1 without ak},
 * which gives H0 = 1, H1 = c, H2 = c c - cs^2 I of section 2 for n <= 2. */
static double hermite_tensor(int n, const int* idx, const int c[3]) {
  if (n == 0) return 1.0;
  if (n == 1) return (double)c[idx[0]];
  double h = c[idx[n - 1]] * hermite_tensor(n - 1, idx, c);
  for (int k = 0; k < n - 1; ++k) {
    if (idx[k] != idx[n - 1]) continue;
    int rest[6], r = 0;
    for (int j = 0; j < n - 1; ++j)
      if (j != k) rest[r++] = idx[j];
    h -= CS2 * hermite_tensor(n - 2, rest, c);
  }
  return h;
}

/* Equilibrium coefficient by the recursive closure of Shan et al. (athermal,
 * velocity-based form of Eq. (6): a^(1)eq = u, a^(2)eq = u u):
 *   a^(n)eq_{a1..an} = a^(n-1)eq_{a1..an-1} u_an. */
static double coeff_eq(int n, const int* idx, const double u[3]) {
  if (n == 1) return u[idx[0]];
  return coeff_eq(n - 1, idx, u) * u[idx[n - 1]];
}

/* Non-equilibrium coefficient by the recursive regularization of
 * Malaspinas (2015), starting from a^(2)neq = a2neq:
 *   a^(n)neq_{a1..an} = u_an a^(n-1)neq_{a1..an-1}
 *       + sum_{l<n} [prod_{k<n, k != l} u_ak] a^(2)neq_{al an}. */
static double coeff_neq(int n, const int* idx, const double u[3], double a2neq[3][3]) {
  if (n == 2) return a2neq[idx[0]][idx[1]];
  const int an = idx[n - 1];
  double v = u[an] * coeff_neq(n - 1, idx, u, a2neq);
  for (int l = 0; l < n - 1; ++l) {
    double prod = 1.0;
    for (int k = 0; k < n - 1; ++k)
      if (k != l) prod *= u[idx[k]];
    v += prod * a2neq[idx[l]][an];
  }
  return v;
}

/* The components of orders 3..6 of the complete D3Q27 basis.  A component
 * is fixed by how often each axis occurs (kx, ky, kz <= 2: the components in
 * which an axis occurs three times vanish on D3Q27 or alias lower orders and
 * are not part of the basis); in the full contraction of Eq. (4) it occurs
 * n! / (kx! ky! kz!) times. */
static void make_high_order_table(lattice_t* L) {
  int b = 0;
  for (int kx = 0; kx <= 2; ++kx)
    for (int ky = 0; ky <= 2; ++ky)
      for (int kz = 0; kz <= 2; ++kz) {
        const int n = kx + ky + kz;
        if (n < 3) continue;
        int r = 0;
        for (int k = 0; k < kx; ++k) L->hidx[b][r++] = 0;
        for (int k = 0; k < ky; ++k) L->hidx[b][r++] = 1;
        for (int k = 0; k < kz; ++k) L->hidx[b][r++] = 2;
        double nfact = 1.0, cs2n = 1.0;
        for (int k = 2; k <= n; ++k) nfact *= k;
        for (int k = 0; k < n; ++k) cs2n *= CS2;
        const double fk[3] = {1.0, 1.0, 2.0}; /* 0!, 1!, 2! */
        const double orderings = nfact / (fk[kx] * fk[ky] * fk[kz]);
        L->hn[b] = n;
        L->hfac[b] = orderings / (cs2n * nfact);
        for (int i = 0; i < L->Q; ++i) L->hH[b][i] = hermite_tensor(n, L->hidx[b], L->c[i]);
        ++b;
      }
}

/* Orders 3..6 at one site, added to the populations:
 * fpost_i += w_i sum_b H_b(c_i) [a_b eq + (1 - omega) a_b neq] (times the
 * factor of the component). */
static void add_high_order_terms(const lattice_t* L, const double u[3], double a2neq[3][3],
                                 double omega, double* fpost) {
  double coef[NHIGH];
  for (int b = 0; b < NHIGH; ++b) {
    const int n = L->hn[b];
    coef[b] = L->hfac[b] * (coeff_eq(n, L->hidx[b], u) +
                            (1.0 - omega) * coeff_neq(n, L->hidx[b], u, a2neq));
  }
  for (int i = 0; i < L->Q; ++i) {
    double sum = 0.0;
    for (int b = 0; b < NHIGH; ++b) sum += L->hH[b][i] * coef[b];
    fpost[i] += L->w[i] * sum;
  }
}

/* Step 3 at one site: regularized post-collision populations, Eq. (3) with
 * f^eq, f^neq from Eq. (4) and the coefficients of Eq. (6) (D3Q27h: plus the
 * orders 3 to 6 of the complete basis). */
static void site_collide(const lattice_t* L, const double m[10], const double F[3],
                         double rho, double omega, double* fpost) {
  double u[3] = {m[1], m[2], m[3]};
  double a2[3][3], uu[3][3], a2neq[3][3];
  unpack_a2(m, a2);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      uu[a][b] = u[a] * u[b];
      a2neq[a][b] = a2[a][b] - uu[a][b];
    }
  const double zero3[3] = {0, 0, 0};
  for (int i = 0; i < L->Q; ++i) {
    double feq = hermite_series(L, i, m[0], u, uu);
    double fneq = hermite_series(L, i, 0.0, zero3, a2neq);
    double S = guo_source(L, i, u, F, rho);
    fpost[i] = feq + (1.0 - omega) * fneq + 0.5 * S;
  }
  if (L->high) add_high_order_terms(L, u, a2neq, omega, fpost);
}

static void site_force(const double* F, int64_t N, int64_t s, double out[3]) {
  if (F) {
    out[0] = F[s]; out[1] = F[N + s]; out[2] = F[2 * N + s];
  } else {
    out[0] = out[1] = out[2] = 0.0;
  }
}

/* Populations whose corrected moments (step 1) are exactly m:
 * f_i = w_i [a0 + c.(u - F/2rho)/cs^2 + H2:(a2 - (Fu+uF)/2rho)/(2 cs^4)],
 * i.e. Eq. (4) with the correction of Eq. (8) undone. */
int oracle_init(int lat, int64_t nx, int64_t ny, int64_t nz, const double* m,
                const double* F, double* f) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t N = nx * ny * nz;
  const double rho = 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double Fs[3], ms[10];
    site_force(F, N, s, Fs);
    for (int k = 0; k < 10; ++k) ms[k] = m[k * N + s];
    double u[3] = {ms[1], ms[2], ms[3]};
    double a1[3], a2[3][3];
    unpack_a2(ms, a2);
    for (int a = 0; a < 3; ++a) a1[a] = u[a] - Fs[a] / (2.0 * rho);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) a2[a][b] -= (Fs[a] * u[b] + Fs[b] * u[a]) / (2.0 * rho);
    for (int i = 0; i < Q; ++i) f[i * N + s] = hermite_series(&L, i, ms[0], a1, a2);
  }
  return 0;
}

/* Reported (corrected) moments of a population field: step 1 at every site. */
int oracle_moments(int lat, int64_t nx, int64_t ny, int64_t nz, const double* f,
                   const double* F, double* m) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double fs[27], Fs[3], ms[10];
    for (int i = 0; i < Q; ++i) fs[i] = f[i * N + s];
    site_force(F, N, s, Fs);
    site_moments(&L, fs, Fs, 1.0, ms);
    for (int k = 0; k < 10; ++k) m[k * N + s] = ms[k];
  }
  return 0;
}

/* Steps 1-3 at every site: fpost = collide(moments(f)). */
int oracle_collide(int lat, int64_t nx, int64_t ny, int64_t nz, double tau,
                   const double* f, const double* F, double* fpost) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t N = nx * ny * nz;
  const double omega = 1.0 / tau;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double fs[27], Fs[3], ms[10], fp[27];
    for (int i = 0; i < Q; ++i) fs[i] = f[i * N + s];
    site_force(F, N, s, Fs);
    site_moments(&L, fs, Fs, 1.0, ms);
    site_collide(&L, ms, Fs, 1.0, omega, fp);
    for (int i = 0; i < Q; ++i) fpost[i * N + s] = fp[i];
  }
  return 0;
}

/* Step 4: pull streaming with periodic wrap, or halfway bounce-back where the
 * source lies beyond a wall (bc[a] = 1 on axis a). */
int oracle_stream(int lat, int64_t nx, int64_t ny, int64_t nz, const int* bc,
                  const double* fpost, double* f) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t n[3] = {nx, ny, nz};
  const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t X[3] = {x, y, z};
        const int64_t s = x + nx * (y + ny * z);
        for (int i = 0; i < Q; ++i) {
          int64_t src[3];
          int solid = 0;
          for (int a = 0; a < 3; ++a) {
            src[a] = X[a] - L.c[i][a];
            if (src[a] < 0 || src[a] >= n[a]) {
              if (bc[a]) solid = 1;
              src[a] = ((src[a] % n[a]) + n[a]) % n[a];
            }
          }
          if (solid) {
            f[i * N + s] = fpost[L.opp[i] * N + s];
          } else {
            const int64_t ss = src[0] + nx * (src[1] + ny * src[2]);
            f[i * N + s] = fpost[i * N + ss];
          }
        }
      }
  return 0;
}

/* nsteps full steps on f (in place); scratch holds Q x N doubles. */
int oracle_run(int lat, int64_t nx, int64_t ny, int64_t nz, const int* bc, double tau,
               const double* F, double* f, double* scratch, int64_t nsteps) {
  for (int64_t t = 0; t < nsteps; ++t) {
    if (oracle_collide(lat, nx, ny, nz, tau, f, F, scratch)) return -1;
    if (oracle_stream(lat, nx, ny, nz, bc, scratch, f)) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Two-component variant (section 2): phase field phi transported by the
 * conservative Allen-Cahn equation, Eq. (2), advanced by forward-time,
 * centred-space differences; density and viscosity blended linearly in phi,
 * rho = rho_L + phi (rho_H - rho_L), nu = nu_L + phi (nu_H - nu_L); total
 * force F = F^s + F^b + F^p + F^nu with
 *   F^s = mu grad(phi),  mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi),
 *         beta = 12 sigma / W, kappa = 3 sigma W / 2;
 *   F^b = rho g (g: body acceleration);
 *   F^p = - p* cs^2 grad(rho);
 *   F^nu = - (nu omega / cs^2) (a2 - u u) . grad(rho)   (the printed form is
 *         garbled; this is the viscous-stress term nu (grad u + grad u^T) .
 *         grad(rho) with the stress written through the non-equilibrium
 *         coefficient of Eq. (6): nu omega / cs^2 = 1 - omega/2, the stress
 *         of the Guo scheme.  The paper's starred (pre-correction)
 *         coefficient, taken with the pre-correction velocity, differs from
 *         a2 - u u only by - F F / (4 rho^2), second order in the force and
 *         left out: with it a2 - u u, a uniformly accelerated flow keeps
 *         F^nu = 0 exactly, as it has no shear).
 * Spatial derivatives use the D3Q27-weighted stencils of section 2:
 *   grad_a Psi(x) = (1/cs^2) sum_i w_i Psi(x + c_i) c_ia,
 *   lap Psi(x)    = (2/cs^2) sum_{i != 0} w_i [Psi(x + c_i) - Psi(x)]
 * (the printed Laplacian stencil is garbled; this is the second-order
 * Taylor-consistent form, zero on constants).  Axes are periodic, or walled
 * (bc[a] = 1): a neighbour beyond a wall is the mirror image of the site
 * next to it, scalars and tangential vector components symmetric, the normal
 * vector component antisymmetric (no flux through the wall).
 * ------------------------------------------------------------------------ */

/* index of the neighbour x + c (c in {-1, 0, 1}^3); *flip[a] = -1 where the
 * step crossed a wall on axis a (the mirror site is returned) */
static int64_t site_shift_bc(int64_t x, int64_t y, int64_t z, const int c[3], const int64_t n[3],
                             const int* bc, int flip[3]) {
  const int64_t X[3] = {x, y, z};
  int64_t Y[3];
  for (int a = 0; a < 3; ++a) {
    int64_t v = X[a] + c[a];
    flip[a] = 1;
    if (v < 0 || v >= n[a]) {
      if (bc && bc[a]) {
        v = X[a];  /* halfway wall: the ghost beyond it mirrors the site next to it */
        flip[a] = -1;
      } else {
        v = v < 0 ? v + n[a] : v - n[a];
      }
    }
    Y[a] = v;
  }
  return Y[0] + n[0] * (Y[1] + n[1] * Y[2]);
}

/* out[a*N + s] = grad_a of the scalar field v at every site */
int oracle_grad(int64_t nx, int64_t ny, int64_t nz, const int* bc, const double* v, double* out) {
  lattice_t L;
  if (make_lattice(27, &L)) return -1;
  const int64_t N = nx * ny * nz, n[3] = {nx, ny, nz};
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t s = x + nx * (y + ny * z);
        double g[3] = {0, 0, 0};
        int flip[3];
        for (int i = 0; i < 27; ++i) {
          const double vi = v[site_shift_bc(x, y, z, L.c[i], n, bc, flip)];
          for (int a = 0; a < 3; ++a) g[a] += L.w[i] * vi * L.c[i][a];
        }
        for (int a = 0; a < 3; ++a) out[a * N + s] = g[a] / CS2;
      }
  return 0;
}

/* out[s] = lap of v at every site */
int oracle_lap(int64_t nx, int64_t ny, int64_t nz, const int* bc, const double* v, double* out) {
  lattice_t L;
  if (make_lattice(27, &L)) return -1;
  const int64_t n[3] = {nx, ny, nz};
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t s = x + nx * (y + ny * z);
        double acc = 0.0;
        int flip[3];
        for (int i = 0; i < 27; ++i) {
          if (L.c[i][0] == 0 && L.c[i][1] == 0 && L.c[i][2] == 0) continue;
          acc += L.w[i] * (v[site_shift_bc(x, y, z, L.c[i], n, bc, flip)] - v[s]);
        }
        out[s] = 2.0 * acc / CS2;
      }
  return 0;
}

/* out[s] = div of the vector field V (3 planes) at every site */
static int oracle_div(int64_t nx, int64_t ny, int64_t nz, const int* bc, const double* V,
                      double* out) {
  lattice_t L;
  if (make_lattice(27, &L)) return -1;
  const int64_t N = nx * ny * nz, n[3] = {nx, ny, nz};
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t s = x + nx * (y + ny * z);
        double acc = 0.0;
        int flip[3];
        for (int i = 0; i < 27; ++i) {
          const int64_t si = site_shift_bc(x, y, z, L.c[i], n, bc, flip);
          for (int a = 0; a < 3; ++a) acc += L.w[i] * L.c[i][a] * flip[a] * V[a * N + si];
        }
        out[s] = acc / CS2;
      }
  return 0;
}

/* One FTCS step of Eq. (2) in conservative form (unit time step):
 *   phi' = phi - div(phi u) + D lap(phi) - lambda div(phi (1 - phi) n),
 * lambda = 4 D / W, n = grad(phi) / (|grad(phi)| + eps).  u: 3 planes. */
int oracle_phase_step(int64_t nx, int64_t ny, int64_t nz, const int* bc, const double* phi,
                      const double* u, double D, double W, double eps, double* phi_new) {
  const int64_t N = nx * ny * nz;
  double* g = malloc(sizeof(double) * 3 * N);
  double* V = malloc(sizeof(double) * 3 * N);
  double* J = malloc(sizeof(double) * 3 * N);
  double* t1 = malloc(sizeof(double) * N);
  double* t2 = malloc(sizeof(double) * N);
  double* t3 = malloc(sizeof(double) * N);
  int rc = (g && V && J && t1 && t2 && t3) ? 0 : -1;
  const double lambda = 4.0 * D / W;
  if (!rc) rc = oracle_grad(nx, ny, nz, bc, phi, g);
  if (!rc) {
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
      const double gx = g[s], gy = g[N + s], gz = g[2 * N + s];
      const double mag = sqrt(gx * gx + gy * gy + gz * gz);
      const double c = phi[s] * (1.0 - phi[s]) / (mag + eps);
      for (int a = 0; a < 3; ++a) {
        V[a * N + s] = phi[s] * u[a * N + s];
        J[a * N + s] = c * g[a * N + s];
      }
    }
    rc = oracle_div(nx, ny, nz, bc, V, t1);
  }
  if (!rc) rc = oracle_lap(nx, ny, nz, bc, phi, t2);
  if (!rc) rc = oracle_div(nx, ny, nz, bc, J, t3);
  if (!rc)
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) phi_new[s] = phi[s] - t1[s] + D * t2[s] - lambda * t3[s];
  free(g); free(V); free(J); free(t1); free(t2); free(t3);
  return rc;
}

/* Capillary force F^s = mu grad(phi), plus a body force Fb (3 planes, or NULL). */
int oracle_capillary_force(int64_t nx, int64_t ny, int64_t nz, const int* bc, const double* phi,
                           double sigma, double W, const double* Fb, double* F) {
  const int64_t N = nx * ny * nz;
  double* g = malloc(sizeof(double) * 3 * N);
  double* l = malloc(sizeof(double) * N);
  int rc = (g && l) ? 0 : -1;
  const double beta = 12.0 * sigma / W, kappa = 1.5 * sigma * W;
  if (!rc) rc = oracle_grad(nx, ny, nz, bc, phi, g);
  if (!rc) rc = oracle_lap(nx, ny, nz, bc, phi, l);
  if (!rc)
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
      const double p = phi[s];
      const double mu = 4.0 * beta * p * (p - 1.0) * (p - 0.5) - kappa * l[s];
      for (int a = 0; a < 3; ++a) F[a * N + s] = mu * g[a * N + s] + (Fb ? Fb[a * N + s] : 0.0);
    }
  free(g); free(l);
  return rc;
}

/* Pressure and viscous force terms of the force split, added to F:
 *   F += - p* cs^2 grad(rho) - (nu omega / cs^2) (a2 - u u) . grad(rho),
 * with p*, u, a2 from the moments m (10 planes) and rho, nu, omega of phi. */
int oracle_contrast_force(int64_t nx, int64_t ny, int64_t nz, const int* bc, const double* phi,
                          const double* m, double rho_l, double rho_h, double nu_l, double nu_h,
                          double* F) {
  const int64_t N = nx * ny * nz;
  double* g = malloc(sizeof(double) * 3 * N);
  int rc = g ? 0 : -1;
  if (!rc) rc = oracle_grad(nx, ny, nz, bc, phi, g);
  if (!rc)
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
      double ms[10], a2[3][3];
      for (int k = 0; k < 10; ++k) ms[k] = m[k * N + s];
      unpack_a2(ms, a2);
      const double nu = nu_l + phi[s] * (nu_h - nu_l);
      const double omega = 1.0 / (nu / CS2 + 0.5);
      double grho[3];
      for (int a = 0; a < 3; ++a) grho[a] = (rho_h - rho_l) * g[a * N + s];
      for (int a = 0; a < 3; ++a) {
        double visc = 0.0;
        for (int b = 0; b < 3; ++b) visc += (a2[a][b] - ms[1 + a] * ms[1 + b]) * grho[b];
        F[a * N + s] += -ms[0] * CS2 * grho[a] - nu * omega / CS2 * visc;
      }
    }
  free(g);
  return rc;
}

/* Steps 1-3 with a relaxation rate and a density per site (omega, rho: N
 * values each): fpost = collide(moments(f)). */
int oracle_collide_var(int lat, int64_t nx, int64_t ny, int64_t nz, const double* omega,
                       const double* rho, const double* f, const double* F, double* fpost) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double fs[27], Fs[3], ms[10], fp[27];
    for (int i = 0; i < Q; ++i) fs[i] = f[i * N + s];
    site_force(F, N, s, Fs);
    site_moments(&L, fs, Fs, rho[s], ms);
    site_collide(&L, ms, Fs, rho[s], omega[s], fp);
    for (int i = 0; i < Q; ++i) fpost[i * N + s] = fp[i];
  }
  return 0;
}

/* Reported moments with a density per site in the correction of Eq. (8). */
int oracle_moments_var(int lat, int64_t nx, int64_t ny, int64_t nz, const double* rho,
                       const double* f, const double* F, double* m) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double fs[27], Fs[3], ms[10];
    for (int i = 0; i < Q; ++i) fs[i] = f[i * N + s];
    site_force(F, N, s, Fs);
    site_moments(&L, fs, Fs, rho[s], ms);
    for (int k = 0; k < 10; ++k) m[k * N + s] = ms[k];
  }
  return 0;
}

/* Populations whose corrected moments (density per site) are exactly m. */
int oracle_init_var(int lat, int64_t nx, int64_t ny, int64_t nz, const double* rho,
                    const double* m, const double* F, double* f) {
  lattice_t L;
  if (make_lattice(lat, &L)) return -1;
  const int Q = L.Q;
  const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double Fs[3], ms[10];
    site_force(F, N, s, Fs);
    for (int k = 0; k < 10; ++k) ms[k] = m[k * N + s];
    double u[3] = {ms[1], ms[2], ms[3]};
    double a1[3], a2[3][3];
    unpack_a2(ms, a2);
    for (int a = 0; a < 3; ++a) a1[a] = u[a] - Fs[a] / (2.0 * rho[s]);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) a2[a][b] -= (Fs[a] * u[b] + Fs[b] * u[a]) / (2.0 * rho[s]);
    for (int i = 0; i < Q; ++i) f[i * N + s] = hermite_series(&L, i, ms[0], a1, a2);
  }
  return 0;
}
