/*
 * FP64 direct Ewald sums: the ORACLE for the DPLR long-range step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with the
 * GPU path.
 *
 * What it computes (orthorhombic box L = (Lx, Ly, Lz), V = Lx Ly Lz):
 *
 *   Reciprocal (Gaussian-charge) energy, the E_Gt of the DPLR background
 *   section, multiplied by the Coulomb constant k_e:
 *       E = k_e/(2 pi V) sum_{m != 0, |m| <= m_cut} f(m) |S(m)|^2,
 *       f(m) = exp(-pi^2 m^2 / beta^2) / m^2,
 *       S(m) = sum_j q_j exp(2 pi i m . r_j),  m = (nx/Lx, ny/Ly, nz/Lz).
 *   The structure factor runs over ions and Wannier centroids alike (the
 *   paper's S(m) is one sum over both charge sets); the sign of the exponent
 *   does not change |S|^2 or the forces.
 *
 *   Forces F_j = -dE/dr_j
 *       = (2 k_e q_j / V) sum_m f(m) m Im( conj(S(m)) exp(2 pi i m . r_j) ).
 *
 *   Virial W_ab = -dE/d(strain_ab)
 *       = k_e/(2 pi V) sum_m f(m)|S(m)|^2 [delta_ab - 2 (1 + pi^2 m^2/beta^2) m_a m_b / m^2].
 *
 *   The real-space and self terms of the full Ewald energy are provided only to
 *   check the normalisation against the NaCl Madelung constant:
 *       E_real = (k_e/2) sum_{i,j,images}' q_i q_j erfc(beta r)/r,
 *       E_self = -k_e beta/sqrt(pi) sum_j q_j^2.
 *
 * Algorithm: the k-vectors of the half space (nx > 0, or nx = 0 and ny > 0, or
 * nx = ny = 0 and nz > 0) are grouped into rows of fixed (nx, ny); each half-
 * space term is counted twice.  Phases exp(2 pi i n r / L) come from sincos on
 * every (particle, n) directly, with no recurrences.  Particles are taken in
 * blocks, rows are split over OpenMP threads, and every sum runs in a fixed
 * order, so results do not depend on the thread count.  Built with -O2 and
 * without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_INVALID 1
#define ORACLE_E_NOMEM 2

typedef struct {
  int nx, ny;       /* row indices                         */
  int nz0, nz1;     /* inclusive nz range of the row       */
  int64_t off;      /* offset of the row's first k         */
} row_t;

typedef struct {
  int nmax[3];
  int64_t nrows, nk;
  row_t* rows;
} kset_t;

static void kset_free(kset_t* ks) { free(ks->rows); ks->rows = NULL; }

/* Enumerate the half-space rows with |m| <= mcut. */
static int kset_build(const double L[3], double mcut, kset_t* ks) {
  double m2max = mcut * mcut;
  for (int a = 0; a < 3; ++a) ks->nmax[a] = (int)floor(mcut * L[a]);
  int64_t cap = (int64_t)(ks->nmax[0] + 1) * (2 * ks->nmax[1] + 1);
  ks->rows = (row_t*)malloc(sizeof(row_t) * (size_t)(cap > 0 ? cap : 1));
  if (!ks->rows) return ORACLE_E_NOMEM;
  ks->nrows = 0;
  ks->nk = 0;
  for (int nx = 0; nx <= ks->nmax[0]; ++nx) {
    for (int ny = -ks->nmax[1]; ny <= ks->nmax[1]; ++ny) {
      if (nx == 0 && ny < 0) continue;
      double mx = nx / L[0], my = ny / L[1];
      double rest = m2max - mx * mx - my * my;
      if (rest < 0) continue;
      int nzm = (int)floor(sqrt(rest) * L[2]);
      /* guard the floor against rounding at the sphere's surface */
      while (nzm >= 0 && (mx * mx + my * my + (nzm / L[2]) * (nzm / L[2])) > m2max) --nzm;
      int nz0 = (nx == 0 && ny == 0) ? 1 : -nzm;
      int nz1 = nzm;
      if (nz1 < nz0) continue;
      row_t r = {nx, ny, nz0, nz1, ks->nk};
      ks->rows[ks->nrows++] = r;
      ks->nk += nz1 - nz0 + 1;
    }
  }
  return ORACLE_OK;
}

/* exp(2 pi i n r / L) for n in [lo, hi], written to (re, im)[n - lo]. */
static void phase_table(double r, double L, int lo, int hi, double* re, double* im) {
  for (int n = lo; n <= hi; ++n) {
    double th = 2.0 * M_PI * (double)n * r / L;
    re[n - lo] = cos(th);
    im[n - lo] = sin(th);
  }
}

static int64_t threads_used = 1;

int64_t oracle_threads_used(void) { return threads_used; }

/* Number of k-vectors (half space) for a cutoff; for sizing and tests. */
int64_t oracle_count_k(const double L[3], double mcut) {
  kset_t ks;
  if (kset_build(L, mcut, &ks) != ORACLE_OK) return -1;
  int64_t nk = ks.nk;
  kset_free(&ks);
  return nk;
}

/*
 * Reciprocal-space Ewald sum.
 *   n, pos[n*3], q[n]: all charges (ions and WCs together);
 *   L[3], beta (1/A), ke (eV A), mcut (1/A);
 *   energy: out scalar (required);
 *   virial: out [6] (xx, yy, zz, xy, xz, yz), may be NULL;
 *   force:  out [n_force*3], may be NULL; force_idx[n_force] selects which
 *           particles (NULL = the first n_force particles).
 * Returns 0 on success.
 */
int oracle_ewald_recip(int64_t n, const double* pos, const double* q, const double L[3],
                       double beta, double ke, double mcut, double* energy, double* virial,
                       int64_t n_force, const int64_t* force_idx, double* force) {
  if (n < 0 || (n > 0 && (!pos || !q)) || !L || !energy || beta <= 0 || mcut <= 0) return ORACLE_E_INVALID;
  for (int a = 0; a < 3; ++a) if (!(L[a] > 0)) return ORACLE_E_INVALID;
  if (n_force > 0 && !force) return ORACLE_E_INVALID;
  for (int64_t i = 0; i < n_force; ++i) {
    int64_t j = force_idx ? force_idx[i] : i;
    if (j < 0 || j >= n) return ORACLE_E_INVALID;
  }

  kset_t ks;
  if (kset_build(L, mcut, &ks) != ORACLE_OK) return ORACLE_E_NOMEM;
  const int64_t nk = ks.nk;
  const int nx1 = ks.nmax[0] + 1, ny1 = 2 * ks.nmax[1] + 1, nz1 = 2 * ks.nmax[2] + 1;
  const double V = L[0] * L[1] * L[2];

  double* Sre = (double*)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
  double* Sim = (double*)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
  double* fk = (double*)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
  const int64_t B = 256; /* particles per block */
  const int64_t tw = nx1 + ny1 + nz1;
  double* tre = (double*)malloc(sizeof(double) * (size_t)(B * tw));
  double* tim = (double*)malloc(sizeof(double) * (size_t)(B * tw));
  if (!Sre || !Sim || !fk || !tre || !tim) {
    free(Sre); free(Sim); free(fk); free(tre); free(tim); kset_free(&ks);
    return ORACLE_E_NOMEM;
  }

  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  threads_used = nthreads;

  /* f(m) for every k */
  for (int64_t r = 0; r < ks.nrows; ++r) {
    const row_t* R = &ks.rows[r];
    double mx = R->nx / L[0], my = R->ny / L[1];
    for (int nz = R->nz0; nz <= R->nz1; ++nz) {
      double mz = nz / L[2];
      double m2 = mx * mx + my * my + mz * mz;
      fk[R->off + (nz - R->nz0)] = exp(-M_PI * M_PI * m2 / (beta * beta)) / m2;
    }
  }

  /* Pass 1: structure factor S(m) = sum_j q_j exp(2 pi i m.r_j). */
  for (int64_t j0 = 0; j0 < n; j0 += B) {
    int64_t nb = (n - j0 < B) ? (n - j0) : B;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
      const double* r = pos + 3 * (j0 + b);
      double* xr = tre + b * tw; double* xi = tim + b * tw;
      phase_table(r[0], L[0], 0, ks.nmax[0], xr, xi);
      phase_table(r[1], L[1], -ks.nmax[1], ks.nmax[1], xr + nx1, xi + nx1);
      phase_table(r[2], L[2], -ks.nmax[2], ks.nmax[2], xr + nx1 + ny1, xi + nx1 + ny1);
    }
#pragma omp parallel for schedule(static)
    for (int64_t ri = 0; ri < ks.nrows; ++ri) {
      const row_t* R = &ks.rows[ri];
      double* sr = Sre + R->off; double* si = Sim + R->off;
      const int cnt = R->nz1 - R->nz0 + 1;
      for (int64_t b = 0; b < nb; ++b) {
        const double* xr = tre + b * tw; const double* xi = tim + b * tw;
        double ar = xr[R->nx], ai = xi[R->nx];
        double br = xr[nx1 + R->ny + ks.nmax[1]], bi = xi[nx1 + R->ny + ks.nmax[1]];
        double qj = q[j0 + b];
        double cr = qj * (ar * br - ai * bi), ci = qj * (ar * bi + ai * br);
        const double* zr = xr + nx1 + ny1 + (R->nz0 + ks.nmax[2]);
        const double* zi = xi + nx1 + ny1 + (R->nz0 + ks.nmax[2]);
        for (int t = 0; t < cnt; ++t) {
          sr[t] += cr * zr[t] - ci * zi[t];
          si[t] += cr * zi[t] + ci * zr[t];
        }
      }
    }
  }

  /* Energy and virial: fixed-order sums over rows. */
  {
    double e = 0, w[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t ri = 0; ri < ks.nrows; ++ri) {
      const row_t* R = &ks.rows[ri];
      double mx = R->nx / L[0], my = R->ny / L[1];
      for (int nz = R->nz0; nz <= R->nz1; ++nz) {
        int64_t k = R->off + (nz - R->nz0);
        double mz = nz / L[2];
        double m2 = mx * mx + my * my + mz * mz;
        double s2 = Sre[k] * Sre[k] + Sim[k] * Sim[k];
        double t = 2.0 * fk[k] * s2; /* half space counted twice */
        double c = 2.0 * (1.0 + M_PI * M_PI * m2 / (beta * beta)) / m2;
        e += t;
        w[0] += t * (1.0 - c * mx * mx);
        w[1] += t * (1.0 - c * my * my);
        w[2] += t * (1.0 - c * mz * mz);
        w[3] += t * (-c * mx * my);
        w[4] += t * (-c * mx * mz);
        w[5] += t * (-c * my * mz);
      }
    }
    double pre = ke / (2.0 * M_PI * V);
    *energy = pre * e;
    if (virial) for (int a = 0; a < 6; ++a) virial[a] = pre * w[a];
  }

  /* Pass 2: forces on the requested particles. */
  if (n_force > 0) {
    /* fold f(m) into S once: A = f(m) S(m) */
    for (int64_t k = 0; k < nk; ++k) { Sre[k] *= fk[k]; Sim[k] *= fk[k]; }
    const double pre = 2.0 * 2.0 * ke / V; /* (2 k_e / V) x 2 for the half space */
#pragma omp parallel
    {
      double* xr = (double*)malloc(sizeof(double) * (size_t)tw);
      double* xi = (double*)malloc(sizeof(double) * (size_t)tw);
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < n_force; ++i) {
        int64_t j = force_idx ? force_idx[i] : i;
        const double* r = pos + 3 * j;
        phase_table(r[0], L[0], 0, ks.nmax[0], xr, xi);
        phase_table(r[1], L[1], -ks.nmax[1], ks.nmax[1], xr + nx1, xi + nx1);
        phase_table(r[2], L[2], -ks.nmax[2], ks.nmax[2], xr + nx1 + ny1, xi + nx1 + ny1);
        double fx = 0, fy = 0, fz = 0;
        for (int64_t ri = 0; ri < ks.nrows; ++ri) {
          const row_t* R = &ks.rows[ri];
          double ar = xr[R->nx], ai = xi[R->nx];
          double br = xr[nx1 + R->ny + ks.nmax[1]], bi = xi[nx1 + R->ny + ks.nmax[1]];
          double cr = ar * br - ai * bi, ci = ar * bi + ai * br;
          const double* zr = xr + nx1 + ny1 + (R->nz0 + ks.nmax[2]);
          const double* zi = xi + nx1 + ny1 + (R->nz0 + ks.nmax[2]);
          const double* sr = Sre + R->off; const double* si = Sim + R->off;
          const int cnt = R->nz1 - R->nz0 + 1;
          double T = 0, Tz = 0;
          for (int t = 0; t < cnt; ++t) {
            double er = cr * zr[t] - ci * zi[t];
            double ei = cr * zi[t] + ci * zr[t];
            /* Im(conj(A) e) = A.re e.im - A.im e.re */
            double v = sr[t] * ei - si[t] * er;
            T += v;
            Tz += v * (double)(R->nz0 + t);
          }
          fx += T * (R->nx / L[0]);
          fy += T * (R->ny / L[1]);
          fz += Tz / L[2];
        }
        double qj = q[j];
        force[3 * i + 0] = pre * qj * fx;
        force[3 * i + 1] = pre * qj * fy;
        force[3 * i + 2] = pre * qj * fz;
      }
      free(xr); free(xi);
    }
  }

  free(Sre); free(Sim); free(fk); free(tre); free(tim);
  kset_free(&ks);
  return ORACLE_OK;
}

/*
 * Real-space Ewald term over all periodic images within rcut, and forces.
 * O(n^2 x images); meant for the small crystal checks.  force may be NULL.
 */
int oracle_ewald_real(int64_t n, const double* pos, const double* q, const double L[3],
                      double beta, double ke, double rcut, double* energy, double* force) {
  if (n < 0 || (n > 0 && (!pos || !q)) || !L || !energy || beta <= 0 || rcut <= 0) return ORACLE_E_INVALID;
  int im[3];
  for (int a = 0; a < 3; ++a) {
    if (!(L[a] > 0)) return ORACLE_E_INVALID;
    im[a] = (int)ceil(rcut / L[a]) + 1;
  }
  double e = 0;
  if (force) memset(force, 0, sizeof(double) * (size_t)(3 * n));
  const double rc2 = rcut * rcut;
  const double two_over_sqrtpi = 2.0 / sqrt(M_PI);
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : e)
  for (int64_t i = 0; i < n; ++i) {
    double fi[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
      double d0[3];
      for (int a = 0; a < 3; ++a) d0[a] = pos[3 * i + a] - pos[3 * j + a];
      for (int a0 = -im[0]; a0 <= im[0]; ++a0)
        for (int a1 = -im[1]; a1 <= im[1]; ++a1)
          for (int a2 = -im[2]; a2 <= im[2]; ++a2) {
            if (i == j && a0 == 0 && a1 == 0 && a2 == 0) continue;
            double dx = d0[0] + a0 * L[0], dy = d0[1] + a1 * L[1], dz = d0[2] + a2 * L[2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 > rc2) continue;
            double r = sqrt(r2);
            double qq = q[i] * q[j];
            e += 0.5 * qq * erfc(beta * r) / r;
            /* -d/dr [erfc(beta r)/r] = erfc/r^2 + 2 beta/sqrt(pi) exp(-beta^2 r^2)/r */
            double g = qq * (erfc(beta * r) / r2 + two_over_sqrtpi * beta * exp(-beta * beta * r2) / r) / r;
            fi[0] += g * dx; fi[1] += g * dy; fi[2] += g * dz;
          }
    }
    if (force) for (int a = 0; a < 3; ++a) force[3 * i + a] = ke * fi[a];
  }
  *energy = ke * e;
  return ORACLE_OK;
}

/* Self term of the Gaussian-charge Ewald split: -k_e beta/sqrt(pi) sum q^2. */
double oracle_ewald_self(int64_t n, const double* q, double beta, double ke) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += q[i] * q[i];
  return -ke * beta / sqrt(M_PI) * s;
}
