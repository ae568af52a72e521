/*
 * CPU oracle for noisy mean-field annealing (NMFA) -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 implementation of what the GPU library computes,
 * written from A. D. King, W. Bernoudy, J. King, A. J. Berkley, T. Lanting, "Emulating the
 * coherent Ising machine with a mean-field algorithm", arXiv:1806.08422:
 *
 *   - the Ising energy H = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i            (Sec. I, Eq. 1)
 *   - noisy mean-field annealing over independent replicas                    (Sec. II, Alg. 1)
 *   - the sign readout s~_i = s_i / |s_i| of its result                        (Sec. II, Alg. 1)
 *   - MAX-CUT values for J = edge weights, h = 0                              (Sec. III, Table I)
 *   - a brute-force ground state by exhaustive enumeration (a check, not the method)
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark load this file's
 * library. The GPU library never links or calls it, and the two share no code: this file has its
 * own Philox generator, its own Gaussian transform, its own schedule interpolation and its own
 * energy sums.
 *
 * Readings of the paper where it is silent or ambiguous (each is listed in the design notes):
 *   R1 noise: N(0, sigma) has standard deviation sigma, is drawn i.i.d. per (t, replica, spin)
 *      and is added to the *normalised* field (Sec. II text on Alg. 1).
 *   R2 noise stream: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the 64-bit seed,
 *      counter (floor(i/4), r, t, 0); its four words give four uniforms u = (x + 1/2) 2^-32 and
 *      Box-Muller (1958) turns (u0,u1) into z(4q), z(4q+1) and (u2,u3) into z(4q+2), z(4q+3).
 *   R3 the normaliser is the root-sum-square sqrt(h_i^2 + sum_j J_ij^2) of the field formula in
 *      Alg. 1 (the prose calls it a root mean square; the formula wins). A zero
 *      normaliser (isolated spin, h_i = 0) makes the field term 0.
 *   R4 the update is synchronous: every s^_i is computed from the old spins before any s_i
 *      changes (Alg. 1 finishes all s^ before it blends any of them in).
 *   R5 readout of s_i = 0 (and -0.0) gives +1.
 *   R6 Eq. 1 sums over unordered pairs i < j of a symmetric J with zero diagonal; this is the
 *      only reading under which the field h_i + sum_j J_ij s_j is dH/ds_i.
 *   R7 the temperature T_t of iteration t = 1..t_f is read off a piecewise-exponential schedule
 *      (log T linear between knots) at relative time u = (t-1)/(t_f-1) (Fig. 2 caption: a
 *      three-segment piecewise exponential that can be compressed to any number of iterations).
 *
 * Arithmetic: IEEE-754 double, round to nearest, summation in ascending index order, built with
 * -O2 -ffp-contract=off and no fast-math, so that no multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10, from its definition in Salmon et al., "Parallel random numbers: as easy as    */
/* 1, 2, 3" (SC'11): an S-box built from two 32x32->64 multiplications per round, with the key  */
/* bumped by the Weyl constants (golden ratio, sqrt(3)-1) between rounds.                       */
/* ------------------------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void nmfa_oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* The four standard normal numbers of counter (q, r, t, 0) under key = seed (reading R2).     */
void nmfa_oracle_gauss4(uint64_t seed, uint32_t q, uint32_t r, uint32_t t, double z[4]) {
  const uint32_t ctr[4] = {q, r, t, 0u};
  const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t x[4];
  nmfa_oracle_philox4x32_10(ctr, key, x);
  const double two_pi = 6.283185307179586476925286766559;
  for (int pair = 0; pair < 2; ++pair) {
    double u0 = ((double)x[2 * pair] + 0.5) / 4294967296.0;
    double u1 = ((double)x[2 * pair + 1] + 0.5) / 4294967296.0;
    double radius = sqrt(-2.0 * log(u0));
    double angle = two_pi * u1;
    z[2 * pair] = radius * cos(angle);
    z[2 * pair + 1] = radius * sin(angle);
  }
}

/* z(seed, t, r, i): the standard normal number added (times sigma) to spin i of replica r at
 * iteration t (1-based). */
double nmfa_oracle_noise(uint64_t seed, int32_t t, int32_t r, int32_t i) {
  double z[4];
  nmfa_oracle_gauss4(seed, (uint32_t)(i / 4), (uint32_t)r, (uint32_t)t, z);
  return z[i % 4];
}

/* ------------------------------------------------------------------------------------------ */
/* Normaliser of the field in Alg. 1: sqrt(h_i^2 + sum_j J_ij^2) (reading R3).                 */
/* ------------------------------------------------------------------------------------------ */
void nmfa_oracle_normalisers(int32_t n, const double *J, const double *h, double *norm) {
  for (int32_t i = 0; i < n; ++i) {
    double hi = h ? h[i] : 0.0;
    double acc = hi * hi;
    for (int32_t j = 0; j < n; ++j) acc += J[(int64_t)i * n + j] * J[(int64_t)i * n + j];
    norm[i] = sqrt(acc);
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Temperature schedule (reading R7). Knots (u_k, T_k) with u_0 = 0 < u_1 < ... < u_K = 1 and  */
/* T_k > 0; between knots log T is linear in u. Writes T[t-1] for t = 1..t_f.                   */
/* Returns 0, or -1 for invalid knots.                                                          */
/* ------------------------------------------------------------------------------------------ */
int nmfa_oracle_schedule(int32_t n_knots, const double *ku, const double *kT, int32_t t_f,
                         double *T) {
  if (n_knots < 1 || t_f < 1) return -1;
  for (int32_t k = 0; k < n_knots; ++k) {
    if (!(kT[k] > 0.0) || !isfinite(kT[k])) return -1;
    if (k > 0 && !(ku[k] > ku[k - 1])) return -1;
  }
  if (n_knots > 1 && (ku[0] != 0.0 || ku[n_knots - 1] != 1.0)) return -1;
  for (int32_t t = 1; t <= t_f; ++t) {
    if (n_knots == 1) {
      T[t - 1] = kT[0];
      continue;
    }
    double u = (t_f == 1) ? 0.0 : (double)(t - 1) / (double)(t_f - 1);
    int32_t k = 0;
    while (k < n_knots - 2 && u > ku[k + 1]) ++k; /* segment [ku[k], ku[k+1]] holding u */
    double w = (u - ku[k]) / (ku[k + 1] - ku[k]);
    if (u == ku[k]) {
      T[t - 1] = kT[k];
    } else if (u == ku[k + 1]) {
      T[t - 1] = kT[k + 1];
    } else {
      T[t - 1] = exp((1.0 - w) * log(kT[k]) + w * log(kT[k + 1]));
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Noisy mean-field annealing (Sec. II, Alg. 1) over a set of independent replicas.             */
/*                                                                                              */
/* Replica r carries a continuous state s_r in [-1, 1]^n that starts at zero. Iteration t      */
/* replaces the whole vector at once (reading R4) by                                            */
/*     s_r  <-  alpha * b_t(s_r) + (1 - alpha) * s_r,                                           */
/*     b_t(s)_i = -tanh( Phi_i / T_t ),                                                         */
/*     Phi_i    = (h_i + sum_j J_ij s_j) / norm_i + sigma * z(seed, t, r, i),                    */
/* the Boltzmann expectation of a spin in the noisy normalised mean field, blended into the old */
/* state by the damping alpha. After the last iteration each component is read out by its sign. */
/* The three helpers below are the three factors of that map; none of them changes the state   */
/* before every component of the new one has been computed from the old one.                   */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t n;
  const double *J, *h, *norm, *T;
  double alpha, sigma;
  uint64_t seed;
  int negate_noise;
} problem_t;

/* m_i = h_i + sum_j J_ij s_j: the local field of Eq. 1 at state s (minus the gradient of H),  */
/* summed over j in ascending order.                                                            */
static void local_field(const problem_t *P, const double *s, double *m) {
  const int32_t n = P->n;
  for (int32_t i = 0; i < n; ++i) {
    const double *row = P->J + (int64_t)i * n;
    double dot = 0.0;
    for (int32_t j = 0; j < n; ++j) dot += row[j] * s[j];
    m[i] = (P->h ? P->h[i] : 0.0) + dot;
  }
}

/* Phi_i = m_i / norm_i + sigma z: the field divided by its normaliser (a zero normaliser gives */
/* a zero field term, reading R3), plus Gaussian noise of standard deviation sigma (R1, R2).   */
static void noisy_normalised_field(const problem_t *P, int32_t t, int32_t r, const double *m,
                                   double *phi) {
  for (int32_t i = 0; i < P->n; ++i) {
    const double scaled = (P->norm[i] > 0.0) ? m[i] / P->norm[i] : 0.0;
    double z = nmfa_oracle_noise(P->seed, t, r, i);
    if (P->negate_noise) z = -z;
    phi[i] = scaled + P->sigma * z;
  }
}

/* s_i <- alpha * (-tanh(Phi_i / T_t)) + (1 - alpha) * s_i, for all i (phi is already complete). */
static void damped_boltzmann_step(const problem_t *P, double T_t, const double *phi, double *s) {
  for (int32_t i = 0; i < P->n; ++i) {
    const double b = -tanh(phi[i] / T_t);
    s[i] = P->alpha * b + (1.0 - P->alpha) * s[i];
  }
}

/*
 * Run iterations t_first..t_f for the replicas rep_ids[0..n_rep-1] (NULL: replicas 0..n_rep-1).
 *
 *   n, J (n*n row-major, symmetric, zero diagonal), h (n or NULL = 0)
 *   alpha, sigma, T (t_f temperatures, T[t-1] for iteration t)
 *   t_first: first iteration to run (1 normally; > 1 resumes from s_init at the end of
 *            iteration t_first-1); s_init: n_rep*n or NULL (= zeros)
 *   seed, negate_noise (test hook: z -> -z)
 *   record, traj: if traj != NULL, traj[(k*n_rep + q)*n + i] = s_i of replica q after the
 *            k-th iteration run, k < record
 *   s_out (n_rep*n, or NULL): final continuous spins; spins_out (n_rep*n, or NULL): readout
 *            s~_i = sign(s_i) with s_i = 0 read as +1 (reading R5)
 *   nthreads: threads over replicas (<= 0: the OpenMP default)
 * Returns 0, or -1 on invalid arguments.
 */
int nmfa_oracle_anneal(int32_t n, const double *J, const double *h, double alpha, double sigma,
                       const double *T, int32_t t_f, int32_t t_first, int32_t n_rep,
                       const int32_t *rep_ids, uint64_t seed, int32_t negate_noise,
                       const double *s_init, int32_t record, double *traj, double *s_out,
                       int8_t *spins_out, int32_t nthreads) {
  if (n < 1 || !J || !T || t_f < 0 || t_first < 1 || n_rep < 0) return -1;
  double *norm = (double *)malloc(sizeof(double) * (size_t)n);
  nmfa_oracle_normalisers(n, J, h, norm);
  const problem_t P = {n, J, h, norm, T, alpha, sigma, seed, negate_noise};
  const int64_t cnt = (int64_t)n_rep * n;
  double *S = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
  for (int64_t k = 0; k < cnt; ++k) S[k] = s_init ? s_init[k] : 0.0;
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
  {
    double *m = (double *)malloc(sizeof(double) * (size_t)n);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    for (int32_t t = t_first; t <= t_f; ++t) {
      const int32_t k = t - t_first; /* 0-based index of this iteration among those run */
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
      for (int32_t q = 0; q < n_rep; ++q) {
        const int32_t r = rep_ids ? rep_ids[q] : q;
        double *s = S + (int64_t)q * n;
        local_field(&P, s, m);
        noisy_normalised_field(&P, t, r, m, phi);
        damped_boltzmann_step(&P, T[t - 1], phi, s);
        if (traj && k < record) memcpy(traj + ((int64_t)k * n_rep + q) * n, s, sizeof(double) * n);
      }
    }
    free(m);
    free(phi);
  }
  for (int64_t k = 0; k < cnt; ++k) {
    if (s_out) s_out[k] = S[k];
    if (spins_out) spins_out[k] = (S[k] < 0.0) ? (int8_t)-1 : (int8_t)1;
  }
  (void)nthreads;
  free(S);
  free(norm);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Energies and cuts (Eq. 1 under reading R6; MAX-CUT as in Table I).                          */
/* ------------------------------------------------------------------------------------------ */

/* H(s) = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i in double, i then j ascending. */
double nmfa_oracle_energy(int32_t n, const double *J, const double *h, const int8_t *s) {
  double pair = 0.0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j) pair += J[(int64_t)i * n + j] * (double)(s[i] * s[j]);
  double field = 0.0;
  if (h)
    for (int32_t i = 0; i < n; ++i) field += h[i] * (double)s[i];
  return pair + field;
}

static int is_integral(double v) { return isfinite(v) && v == floor(v) && fabs(v) < 9.0e15; }

/* The same energy in exact 64-bit integers; returns -1 if some J_ij or h_i is not an integer. */
int nmfa_oracle_energy_int(int32_t n, const double *J, const double *h, const int8_t *s,
                           int64_t *E) {
  int64_t acc = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t j = i + 1; j < n; ++j) {
      double v = J[(int64_t)i * n + j];
      if (!is_integral(v)) return -1;
      acc += (int64_t)v * (int64_t)s[i] * (int64_t)s[j];
    }
  }
  if (h) {
    for (int32_t i = 0; i < n; ++i) {
      if (!is_integral(h[i])) return -1;
      acc += (int64_t)h[i] * (int64_t)s[i];
    }
  }
  *E = acc;
  return 0;
}

/* MAX-CUT value of the partition s under edge weights W = J: the total weight of the pairs
 * i < j that s puts on opposite sides. */
double nmfa_oracle_cut(int32_t n, const double *W, const int8_t *s) {
  double cut = 0.0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j)
      if (s[i] != s[j]) cut += W[(int64_t)i * n + j];
  return cut;
}

/* ------------------------------------------------------------------------------------------ */
/* Brute-force ground state (a check of success, not part of the method).                      */
/* Enumerates spin vectors in Gray-code order, keeping the local fields f_k = h_k + sum_j J_kj */
/* s_j up to date so that each step costs O(n). With h = 0 the energy is even under s -> -s,   */
/* so the last spin is held at +1 and only 2^(n-1) vectors are visited. n <= 30.               */
/* Returns the minimum energy (recomputed exactly from the best vector) and writes the vector. */
/* ------------------------------------------------------------------------------------------ */
double nmfa_oracle_ground_state(int32_t n, const double *J, const double *h, int8_t *best) {
  if (n < 1 || n > 30) return NAN;
  int h_zero = 1;
  if (h)
    for (int32_t i = 0; i < n; ++i)
      if (h[i] != 0.0) h_zero = 0;
  const int32_t m = h_zero ? n - 1 : n; /* spins that are enumerated */
  int8_t *s = (int8_t *)malloc((size_t)n);
  double *f = (double *)malloc(sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) s[i] = 1;
  for (int32_t k = 0; k < n; ++k) {
    double acc = h ? h[k] : 0.0;
    for (int32_t j = 0; j < n; ++j) acc += J[(int64_t)k * n + j] * s[j];
    f[k] = acc;
  }
  double E = nmfa_oracle_energy(n, J, h, s);
  double E_best = E;
  uint64_t g_best = 0;
  const uint64_t count = (uint64_t)1 << m;
  for (uint64_t g = 1; g < count; ++g) {
    int32_t k = __builtin_ctzll(g); /* Gray code: flip bit k between g-1 and g */
    /* flipping s_k changes H by -2 s_k (h_k + sum_j J_kj s_j) */
    E += -2.0 * s[k] * f[k];
    s[k] = (int8_t)-s[k];
    for (int32_t j = 0; j < n; ++j) f[j] += 2.0 * J[(int64_t)j * n + k] * s[k];
    if (E < E_best) {
      E_best = E;
      g_best = g;
    }
  }
  /* reconstruct the best vector from its Gray code g ^ (g >> 1) */
  uint64_t code = g_best ^ (g_best >> 1);
  for (int32_t i = 0; i < n; ++i) best[i] = 1;
  for (int32_t k = 0; k < m; ++k)
    if ((code >> k) & 1u) best[k] = -1;
  double exact = nmfa_oracle_energy(n, J, h, best);
  free(s);
  free(f);
  return exact;
}

int nmfa_oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
