/* Plain FP64 Wilson hopping term on the full lattice (test infrastructure:
 * the oracle's fast path for lattices where numpy is too slow).
 *
 *   (H psi)(n) = sum_mu [ (1 - g_mu) U_mu(n) psi(n+mu) + (1 + g_mu) U_mu(n-mu)^+ psi(n-mu) ]
 *   (H^+ psi)(n): projector signs swapped.
 *
 * Written as plain loops: site, direction, then a 3x3 colour product and a full
 * 4x4 spin product with the projector (no half-spinor tricks, no intrinsics).
 * Canonical layouts: links [mu][x0][z][y][x][3][3], spinors
 * [rhs][t][z][y][x][4][3] over the dynamical slices, complex128.
 * Boundaries: 0 = Schroedinger functional (x0 = 0..T, spinors vanish on
 * x0 = 0 and T), 1 = periodic, 2 = antiperiodic in time.
 */
#include <complex.h>
#include <string.h>

typedef double complex cplx;

static cplx G[4][4][4]; /* gamma matrices, chiral basis */
static int g_ready = 0;

static void init_gamma(void) {
  /* e_0 = -1, e_k = -i sigma_k;  g_mu = [[0, e_mu], [e_mu^+, 0]] */
  cplx e[4][2][2];
  memset(e, 0, sizeof(e));
  e[0][0][0] = -1; e[0][1][1] = -1;
  e[1][0][1] = -I; e[1][1][0] = -I;              /* -i sigma_1 */
  e[2][0][1] = -1; e[2][1][0] = 1;               /* -i sigma_2 */
  e[3][0][0] = -I; e[3][1][1] = I;               /* -i sigma_3 */
  memset(G, 0, sizeof(G));
  for (int mu = 0; mu < 4; ++mu)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        G[mu][a][2 + b] = e[mu][a][b];
        G[mu][2 + a][b] = conj(e[mu][b][a]);
      }
  g_ready = 1;
}

void wilson_ref_gamma(int mu, double* out) { /* for the tests */
  if (!g_ready) init_gamma();
  memcpy(out, G[mu], sizeof(cplx) * 16);
}

void wilson_ref_hop(const cplx* U, const cplx* in, cplx* out, int lx, int ly, int lz, int T, int bc,
                    int n_rhs, int dagger) {
  if (!g_ready) init_gamma();
  const int t0 = bc == 0 ? 1 : 0;
  const int td = bc == 0 ? T - 1 : T;
  const int ns = bc == 0 ? T + 1 : T; /* stored link slices */
  const long vs = (long)lx * ly * lz; /* sites per slice */
  const long vd = vs * td;
  for (int r = 0; r < n_rhs; ++r) {
#pragma omp parallel for schedule(static)
    for (long q = 0; q < vd; ++q) {
      const int x = (int)(q % lx), y = (int)((q / lx) % ly), z = (int)((q / ((long)lx * ly)) % lz);
      const int t = (int)(q / vs);
      const int x0 = t + t0;
      cplx acc[4][3];
      memset(acc, 0, sizeof(acc));
      for (int mu = 0; mu < 4; ++mu) {
        for (int dir = 0; dir < 2; ++dir) { /* 0: forward, 1: backward */
          int c[4] = {x0, x, y, z};       /* mu = 0 time, 1 x, 2 y, 3 z */
          const int ext[4] = {0, lx, ly, lz};
          double sgn = 1.0;
          int ok = 1;
          if (dir == 0) c[mu] += 1; else c[mu] -= 1;
          if (mu == 0) {
            if (bc == 0) {
              if (c[0] < 1 || c[0] > T - 1) ok = 0; /* psi(0) = psi(T) = 0 */
            } else {
              if (c[0] == T) { c[0] = 0; if (bc == 2) sgn = -1.0; }
              if (c[0] < 0) { c[0] = T - 1; if (bc == 2) sgn = -1.0; }
            }
          } else {
            c[mu] = (c[mu] + ext[mu]) % ext[mu];
          }
          if (!ok) continue;
          const long qn = (long)(c[0] - t0) * vs + ((long)c[3] * ly + c[2]) * lx + c[1];
          const cplx* pn = in + ((long)r * vd + qn) * 12;
          /* link: U_mu(n) forward, U_mu(n - mu)^+ backward */
          const int lx0 = dir == 0 ? x0 : c[0];
          const long ql = dir == 0 ? ((long)z * ly + y) * lx + x : ((long)c[3] * ly + c[2]) * lx + c[1];
          const cplx* u = U + (((long)mu * ns + lx0) * vs + ql) * 9;
          cplx v[4][3];
          for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
              cplx sum = 0;
              for (int b = 0; b < 3; ++b)
                sum += (dir == 0 ? u[3 * a + b] : conj(u[3 * b + a])) * pn[3 * s + b];
              v[s][a] = sgn * sum;
            }
          /* projector 1 - g (forward) / 1 + g (backward); swapped for H^+ */
          const double sp = ((dir == 0) != (dagger != 0)) ? -1.0 : 1.0;
          for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
              cplx sum = v[s][a];
              for (int k = 0; k < 4; ++k) sum += sp * G[mu][s][k] * v[k][a];
              acc[s][a] += sum;
            }
        }
      }
      cplx* po = out + ((long)r * vd + q) * 12;
      for (int s = 0; s < 4; ++s)
        for (int a = 0; a < 3; ++a) po[3 * s + a] = acc[s][a];
    }
  }
}

/* Thread count of the loops above (for timing the oracle on one core); 0 or
 * less leaves OpenMP's default. */
#include <omp.h>
void wilson_ref_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
int wilson_ref_get_threads(void) { return omp_get_max_threads(); }
