/*
 * DECO oracle: a plain, slow, FP64 CPU reference of the batched projected-gradient
 * MaxCut method of "A Scalable Lift-and-Project Differentiable Approach For the
 * Maximum Cut Problem" (Alkhouri et al.).
 *
 * This file is TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. It shares no code, header, table or helper
 * with the GPU library: every routine here is written straight from the paper's
 * definitions, in plain loops, for a reader to check by eye.
 *
 * Graph convention: symmetric CSR with both directions stored (row_ptr int64[n+1],
 * col int32[nnz]); w == NULL means unit weights (the paper's adjacency A, Sec. 2);
 * otherwise w generalises A to a symmetric weight matrix W.
 *
 * Batch layout: X is n x (l*B) doubles, row-major; for node v, component i (0 <= i < l)
 * of initialisation b sits at X[v*l*B + i*B + b]. Unlifted runs use l = 1.
 *
 * Readings of the paper taken here (each is listed with its reason in the design notes):
 *  - gradient form: "cut form" g = -1/2 W x (the exact gradient of
 *    F(x) = 1/2 sum_{(u,v) in E} w_uv (1 - x_u x_v), which equals the cut on {-1,1}^n)
 *    or "Laplacian form" g = L x exactly as printed in eq. (6);
 *  - the running best includes every scored iterate, t = 0..T (Alg. 1/2 score once at T);
 *  - IDI's (Ab)_i counts important neighbours with p = -1;
 *  - the evolutionary genome is (log10 eta for the unlifted batch, log10 eta for the
 *    lifted batch, l), plus the step count of either batch when it is searched; the
 *    initial population is drawn from the bounds (Sec. 4.3).
 * Parity status: every function here is pinned by a CPU test (brute force, closed forms,
 * identities, fixed points, finite differences, eigen-decomposition, published
 * Philox known-answer vectors, hand-worked draws of the search) except the DECO loop as a
 * whole, which is pinned only by determinism, bounds, the exactness of its returned cut
 * and brute force on tiny graphs ("parity unpinned" beyond that).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------
 * Graph checks and degrees (Sec. 2 notation: d_v, Delta, D, A)
 * ---------------------------------------------------------------------------------- */

static double wt(const double *w, int64_t k) { return w ? w[k] : 1.0; }

/* Returns 0 for a valid symmetric simple CSR, otherwise a code naming the first problem:
 * 1 bad row_ptr, 2 column out of range, 3 self-loop, 4 unsorted or duplicate column,
 * 5 asymmetric (missing mirror entry or different weight), 6 non-finite weight. */
int orc_csr_check(int64_t n, const int64_t *rp, const int32_t *col, const double *w) {
  if (n < 0 || rp[0] != 0) return 1;
  for (int64_t v = 0; v < n; v++)
    if (rp[v + 1] < rp[v]) return 1;
  for (int64_t v = 0; v < n; v++) {
    for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
      int64_t u = col[k];
      if (u < 0 || u >= n) return 2;
      if (u == v) return 3;
      if (k > rp[v] && col[k - 1] >= col[k]) return 4;
      if (w && !isfinite(w[k])) return 6;
    }
  }
  for (int64_t v = 0; v < n; v++) {
    for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
      int64_t u = col[k];
      int found = 0;
      for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
        if (col[j] == v) {
          if (w && w[j] != w[k]) return 5;
          found = 1;
          break;
        }
      }
      if (!found) return 5;
    }
  }
  return 0;
}

/* d_v = number of incident edges; dw_v = sum of incident weights; returns Delta. */
int64_t orc_degrees(int64_t n, const int64_t *rp, const double *w, int64_t *d, double *dw) {
  int64_t delta = 0;
  for (int64_t v = 0; v < n; v++) {
    d[v] = rp[v + 1] - rp[v];
    double s = 0.0;
    for (int64_t k = rp[v]; k < rp[v + 1]; k++) s += wt(w, k);
    dw[v] = s;
    if (d[v] > delta) delta = d[v];
  }
  return delta;
}

/* ------------------------------------------------------------------------------------
 * One projected gradient-ascent step (Sec. 3.1 eq. (6)-(7); lifted: Sec. 3.2, where the
 * Jacobian L X acts column by column, so the same routine serves both).
 *   form 0 (cut form):       G[v,c] = -1/2 * sum_{u in N(v)} w_vu X[u,c]
 *   form 1 (Laplacian form): G[v,c] = dw_v X[v,c] - sum_{u in N(v)} w_vu X[u,c]  (= (L X)[v,c])
 *   X'[v,c] = Proj_[-1,1](X[v,c] + eta[c] * G[v,c])
 * ---------------------------------------------------------------------------------- */
void orc_step(int64_t n, const int64_t *rp, const int32_t *col, const double *w, int64_t C,
              const double *X, double *Xn, const double *eta, int form) {
  for (int64_t v = 0; v < n; v++) {
    double dwv = 0.0;
    for (int64_t k = rp[v]; k < rp[v + 1]; k++) dwv += wt(w, k);
    for (int64_t c = 0; c < C; c++) {
      double s = 0.0;
      for (int64_t k = rp[v]; k < rp[v + 1]; k++) s += wt(w, k) * X[(int64_t)col[k] * C + c];
      double g = (form == 0) ? -0.5 * s : dwv * X[v * C + c] - s;
      double y = X[v * C + c] + eta[c] * g;
      if (y > 1.0) y = 1.0;
      if (y < -1.0) y = -1.0;
      Xn[v * C + c] = y;
    }
  }
}

/* Gradient only (no step, no projection), for finite-difference checks. */
void orc_grad(int64_t n, const int64_t *rp, const int32_t *col, const double *w, int64_t C,
              const double *X, double *G, int form) {
  for (int64_t v = 0; v < n; v++) {
    double dwv = 0.0;
    for (int64_t k = rp[v]; k < rp[v + 1]; k++) dwv += wt(w, k);
    for (int64_t c = 0; c < C; c++) {
      double s = 0.0;
      for (int64_t k = rp[v]; k < rp[v + 1]; k++) s += wt(w, k) * X[(int64_t)col[k] * C + c];
      G[v * C + c] = (form == 0) ? -0.5 * s : dwv * X[v * C + c] - s;
    }
  }
}

/* ------------------------------------------------------------------------------------
 * Rounding (Sec. 3.1 eq. (5): z_v = 1{x_v > 0}; Sec. 3.2 lifted rounding:
 * z_v = 1{sum_i X[v,i] >= 0}). z is n x B bytes.
 * sum_f32 = 1 forms the lifted row sum in single precision, component order i = 0..l-1
 * (the precision the GPU path decides in); 0 forms it in double precision.
 * ---------------------------------------------------------------------------------- */
void orc_round(int64_t n, int64_t B, int64_t l, int lifted, int sum_f32, const double *X,
               uint8_t *z) {
  int64_t C = l * B;
  for (int64_t v = 0; v < n; v++) {
    for (int64_t b = 0; b < B; b++) {
      if (!lifted) {
        z[v * B + b] = X[v * C + b] > 0.0 ? 1 : 0;
      } else if (sum_f32) {
        float s = 0.0f;
        for (int64_t i = 0; i < l; i++) s = s + (float)X[v * C + i * B + b];
        z[v * B + b] = s >= 0.0f ? 1 : 0;
      } else {
        double s = 0.0;
        for (int64_t i = 0; i < l; i++) s += X[v * C + i * B + b];
        z[v * B + b] = s >= 0.0 ? 1 : 0;
      }
    }
  }
}

/* ------------------------------------------------------------------------------------
 * Cut value, eq. (1): Cut(S) = sum_{v in S} sum_{u not in S} w_vu with S = {v : z_v = 1}.
 * Rows [r0, r1) only (one graph of a block-diagonal batch). For integer weights the sum is
 * formed in int64 (exact); otherwise in double, in CSR order.
 * ---------------------------------------------------------------------------------- */
static int weights_integral(const int64_t *rp, int64_t r0, int64_t r1, const double *w) {
  if (!w) return 1;
  for (int64_t k = rp[r0]; k < rp[r1]; k++)
    if (w[k] != floor(w[k]) || fabs(w[k]) > 9.0e15) return 0;
  return 1;
}

void orc_cut_batch(int64_t r0, int64_t r1, const int64_t *rp, const int32_t *col,
                   const double *w, int64_t B, const uint8_t *z, double *cut) {
  int integral = weights_integral(rp, r0, r1, w);
  for (int64_t b = 0; b < B; b++) {
    int64_t si = 0;
    double sd = 0.0;
    for (int64_t v = r0; v < r1; v++) {
      if (!z[v * B + b]) continue; /* v in S */
      for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
        int64_t u = col[k];
        if (z[u * B + b]) continue; /* u in S too */
        if (integral)
          si += (int64_t)wt(w, k);
        else
          sd += wt(w, k);
      }
    }
    cut[b] = integral ? (double)si : sd;
  }
}

/* Running best over scored iterates (Alg. 1/2 steps 5-6): a column improves only on a
 * strictly larger cut, so the earliest step wins ties. z_best is n x B. */
void orc_best_update(int64_t n, int64_t B, int64_t t, const double *cut, const uint8_t *z,
                     double *best, int64_t *best_step, uint8_t *z_best) {
  for (int64_t b = 0; b < B; b++) {
    if (cut[b] > best[b]) {
      best[b] = cut[b];
      best_step[b] = t;
      for (int64_t v = 0; v < n; v++) z_best[v * B + b] = z[v * B + b];
    }
  }
}

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with a Weyl-sequence key.
 * ---------------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Draw convention: key = (seed low word, seed high word); counter = (node, column,
 * purpose tag, batch index). Purpose tags: */
enum { P_UNIFORM = 1, P_DUI = 2, P_IDI_SIGN = 3, P_IDI_TIE = 4, P_GAUSS = 5, P_EVO = 6 };

static void draw(uint64_t seed, uint32_t a, uint32_t b, uint32_t purpose, uint32_t batch,
                 uint32_t out[4]) {
  uint32_t ctr[4] = {a, b, purpose, batch};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox(ctr, key, out);
}

static double u24(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }

static double gauss(const uint32_t r[4]) {
  double u1 = ((double)(r[0] >> 8) + 1.0) * (1.0 / 16777216.0); /* (0, 1] */
  double u2 = u24(r[1]);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ------------------------------------------------------------------------------------
 * Initialisations (Sec. 4.1, Sec. 4.2, Sec. 5 settings)
 * ---------------------------------------------------------------------------------- */

/* Uniform start in [-1, 1): x = 2u - 1 with u on the 2^-24 grid. */
void orc_init_uniform(int64_t n, int64_t C, uint64_t seed, uint32_t batch, double *X) {
  uint32_t r[4];
  for (int64_t v = 0; v < n; v++)
    for (int64_t c = 0; c < C; c++) {
      draw(seed, (uint32_t)v, (uint32_t)c, P_UNIFORM, batch, r);
      X[v * C + c] = 2.0 * u24(r[0]) - 1.0;
    }
}

/* DUI (Sec. 4.1): h_v ~ U[-(1 - d_v/Delta), (1 - d_v/Delta)], one draw per column. */
void orc_init_dui(int64_t n, const int64_t *rp, int64_t C, uint64_t seed, uint32_t batch,
                  double *H) {
  int64_t delta = 0;
  for (int64_t v = 0; v < n; v++)
    if (rp[v + 1] - rp[v] > delta) delta = rp[v + 1] - rp[v];
  uint32_t r[4];
  for (int64_t v = 0; v < n; v++) {
    double half = delta > 0 ? 1.0 - (double)(rp[v + 1] - rp[v]) / (double)delta : 1.0;
    for (int64_t c = 0; c < C; c++) {
      draw(seed, (uint32_t)v, (uint32_t)c, P_DUI, batch, r);
      H[v * C + c] = (2.0 * u24(r[0]) - 1.0) * half;
    }
  }
}

/* Importance threshold of IDI (Sec. 4.1): dbar + beta*sigma with the population mean and
 * standard deviation of the degrees. Returns the threshold; I = {v : d_v > threshold}. */
double orc_idi_threshold(int64_t n, const int64_t *rp, double beta) {
  if (n <= 0) return 0.0;
  double sum = 0.0;
  for (int64_t v = 0; v < n; v++) sum += (double)(rp[v + 1] - rp[v]);
  double dbar = sum / (double)n;
  double ss = 0.0;
  for (int64_t v = 0; v < n; v++) {
    double e = (double)(rp[v + 1] - rp[v]) - dbar;
    ss += e * e;
  }
  double sigma = sqrt(ss / (double)n);
  return dbar + beta * sigma;
}

/* IDI sign vector h in {-1,+1} per column (Sec. 4.1). Rows [r0, r1) form one graph whose
 * statistics define the important set. Column c draws independently. */
void orc_init_idi(int64_t r0, int64_t r1, const int64_t *rp, const int32_t *col,
                  const double *w, int64_t C, double beta, uint64_t seed, uint32_t batch,
                  double *H) {
  int64_t n = r1 - r0;
  /* threshold over this graph's rows */
  double sum = 0.0;
  for (int64_t v = r0; v < r1; v++) sum += (double)(rp[v + 1] - rp[v]);
  double dbar = n > 0 ? sum / (double)n : 0.0;
  double ss = 0.0;
  for (int64_t v = r0; v < r1; v++) {
    double e = (double)(rp[v + 1] - rp[v]) - dbar;
    ss += e * e;
  }
  double thr = dbar + beta * (n > 0 ? sqrt(ss / (double)n) : 0.0);
  uint32_t r[4];
  double *p = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); /* 0 = not important */
  for (int64_t c = 0; c < C; c++) {
    for (int64_t v = r0; v < r1; v++) {
      if ((double)(rp[v + 1] - rp[v]) > thr) {
        draw(seed, (uint32_t)v, (uint32_t)c, P_IDI_SIGN, batch, r);
        p[v - r0] = (r[0] >> 31) ? 1.0 : -1.0;
      } else {
        p[v - r0] = 0.0;
      }
    }
    for (int64_t v = r0; v < r1; v++) {
      if (p[v - r0] != 0.0) {
        H[v * C + c] = p[v - r0];
        continue;
      }
      double aa = 0.0, bb = 0.0; /* (A a)_v and (A b)_v */
      for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
        double pu = p[col[k] - r0];
        if (pu > 0.0) aa += wt(w, k);
        if (pu < 0.0) bb += wt(w, k);
      }
      if (aa == bb) {
        draw(seed, (uint32_t)v, (uint32_t)c, P_IDI_TIE, batch, r);
        H[v * C + c] = (r[0] >> 31) ? 1.0 : -1.0;
      } else if (aa < bb) {
        H[v * C + c] = 1.0;
      } else {
        H[v * C + c] = -1.0;
      }
    }
  }
  free(p);
}

/* Batch start (Sec. 4.2 with the Sec. 5 down-scaling): X[v,c] = Proj((M[v,c] + sqrt(s2) *
 * eps[v,c]) / scale), eps ~ N(0,1) by Box-Muller on the draw for (v, c). */
void orc_init_gauss(int64_t n, int64_t C, const double *M, double s2, double scale,
                    uint64_t seed, uint32_t batch, double *X) {
  uint32_t r[4];
  double sd = sqrt(s2);
  for (int64_t v = 0; v < n; v++)
    for (int64_t c = 0; c < C; c++) {
      draw(seed, (uint32_t)v, (uint32_t)c, P_GAUSS, batch, r);
      double y = (M[v * C + c] + sd * gauss(r)) / scale;
      if (y > 1.0) y = 1.0;
      if (y < -1.0) y = -1.0;
      X[v * C + c] = y;
    }
}

/* ------------------------------------------------------------------------------------
 * Evolution-based search (Sec. 4.3). Genome per member: e_q (log10 step of the unlifted
 * batch), e_l (log10 step of the lifted batch), l (lift dimension). One call ranks the
 * members by fitness (descending, ties to the lower index), keeps the top half in rank
 * order and replaces the bottom half: ranked member K/2+j is a perturbation of ranked
 * member j: e' = Proj_[lo,hi](e + 0.2*eps), eps ~ N(0,1); l' = clip(l + U{-1,0,1}, 1, lmax).
 * ---------------------------------------------------------------------------------- */
void orc_evo_next(int64_t K, const double *fitness, const double *eq, const double *el,
                  const int32_t *l, double lo, double hi, int32_t lmax, uint64_t seed,
                  uint32_t round, double *eq_out, double *el_out, int32_t *l_out) {
  int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
  for (int64_t i = 0; i < K; i++) rank[i] = i;
  /* insertion sort: descending fitness, stable (lower index first on ties) */
  for (int64_t i = 1; i < K; i++) {
    int64_t x = rank[i], j = i - 1;
    while (j >= 0 && fitness[rank[j]] < fitness[x]) {
      rank[j + 1] = rank[j];
      j--;
    }
    rank[j + 1] = x;
  }
  int64_t keep = K / 2;
  for (int64_t i = 0; i < keep; i++) {
    eq_out[i] = eq[rank[i]];
    el_out[i] = el[rank[i]];
    l_out[i] = l[rank[i]];
  }
  uint32_t r[4];
  for (int64_t i = keep; i < K; i++) {
    int64_t src = rank[i - keep];
    draw(seed, round, (uint32_t)i, P_EVO, 0, r);
    double e1 = gauss(r);
    uint32_t r2[4] = {r[2], r[3], 0, 0};
    double e2 = gauss(r2);
    double a = eq[src] + 0.2 * e1;
    double b = el[src] + 0.2 * e2;
    eq_out[i] = a < lo ? lo : (a > hi ? hi : a);
    el_out[i] = b < lo ? lo : (b > hi ? hi : b);
    draw(seed, round, (uint32_t)i, P_EVO, 1, r);
    int32_t dl = (int32_t)(r[0] % 3u) - 1;
    int32_t nl = l[src] + dl;
    l_out[i] = nl < 1 ? 1 : (nl > lmax ? lmax : nl);
  }
  free(rank);
}

/* Initial population of the evolution-based search (Sec. 4.3): every member draws its
 * combination from the bounds. Member k:
 *   e_q, e_l ~ U[lo, hi): e = lo + (hi - lo) u with u = u24 of words 0 and 1 of the draw
 *     (counter (0xFFFFFFFF, k, P_EVO, 6)); the steps are 10^e;
 *   l ~ U{1..lmax}: 1 + (word 2 mod lmax) of the same draw (the lift dimension is this
 *     build's third gene, Sec. 5 fixes l = 2 where it is not searched);
 *   T_q ~ U{Tq_lo..Tq_hi}: Tq_lo + (word 0 mod (Tq_hi - Tq_lo + 1)) of the draw
 *     (0xFFFFFFFF, k, P_EVO, 3); T_l likewise from (0xFFFFFFFF, k, P_EVO, 5).
 * The modulo draws are uniform up to a relative bias below 2^-19 for ranges below 8193. */
void orc_evo_init(int64_t K, double lo, double hi, int32_t lmax, int64_t Tq_lo, int64_t Tq_hi,
                  int64_t Tl_lo, int64_t Tl_hi, uint64_t seed, double *eq, double *el, int32_t *l,
                  int32_t *Tq, int32_t *Tl) {
  uint32_t r[4];
  for (int64_t k = 0; k < K; k++) {
    draw(seed, 0xFFFFFFFFu, (uint32_t)k, P_EVO, 6, r);
    eq[k] = lo + (hi - lo) * u24(r[0]);
    el[k] = lo + (hi - lo) * u24(r[1]);
    l[k] = 1 + (int32_t)(r[2] % (uint32_t)lmax);
    draw(seed, 0xFFFFFFFFu, (uint32_t)k, P_EVO, 3, r);
    Tq[k] = (int32_t)(Tq_lo + (int64_t)(r[0] % (uint32_t)(Tq_hi - Tq_lo + 1)));
    draw(seed, 0xFFFFFFFFu, (uint32_t)k, P_EVO, 5, r);
    Tl[k] = (int32_t)(Tl_lo + (int64_t)(r[0] % (uint32_t)(Tl_hi - Tl_lo + 1)));
  }
}

/* Step-count perturbation of Sec. 4.3: T' = floor(T0 * (1 + 0.2*(2*eps' - 1))), eps' ~ U(0,1),
 * then clipped to [Tl, Tu]. */
int64_t orc_perturb_T(int64_t T0, double eps_u, int64_t Tl, int64_t Tu) {
  int64_t t = (int64_t)floor((double)T0 * (1.0 + 0.2 * (2.0 * eps_u - 1.0)));
  if (t < Tl) t = Tl;
  if (t > Tu) t = Tu;
  return t;
}

/* Step counts of the population after one evolution round (Sec. 4.3): members ranked as in
 * orc_evo_next; the kept half is copied in rank order and slot keep + j takes the count of
 * ranked member j perturbed by orc_perturb_T with eps' = u24 of its own draw (index
 * 2 + 2 * gene: gene 0 the unlifted count, 1 the lifted one). */
void orc_evo_next_steps(int64_t K, const double *fitness, const int32_t *T, int64_t Tl, int64_t Tu,
                        uint64_t seed, uint32_t round, uint32_t gene, int32_t *T_out) {
  int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
  for (int64_t i = 0; i < K; i++) rank[i] = i;
  for (int64_t i = 1; i < K; i++) {
    int64_t x = rank[i], j = i - 1;
    while (j >= 0 && fitness[rank[j]] < fitness[x]) {
      rank[j + 1] = rank[j];
      j--;
    }
    rank[j + 1] = x;
  }
  int64_t keep = K / 2;
  for (int64_t i = 0; i < keep; i++) T_out[i] = T[rank[i]];
  uint32_t r[4];
  for (int64_t i = keep; i < K; i++) {
    draw(seed, round, (uint32_t)i, P_EVO, 2 + 2 * gene, r);
    T_out[i] = (int32_t)orc_perturb_T(T[rank[i - keep]], u24(r[0]), Tl, Tu);
  }
  free(rank);
}

/* ------------------------------------------------------------------------------------
 * One batch of pQUCO (Alg. 1) or pLUCO (Alg. 2): T steps from X (updated in place), every
 * iterate t = 0..T scored (score_every = 1) and the per-initialisation best kept.
 * eta_b[b] is the step of initialisation b (all l components share it). T_b (NULL: T for
 * every initialisation) gives initialisation b its own count: from step T_b[b] on its
 * columns stay where they are (a step of size 0) while the batch runs on to T.
 * ---------------------------------------------------------------------------------- */
void orc_run_batch(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                   int64_t B, int64_t l, int lifted, int form, const double *eta_b, int64_t T,
                   const int64_t *T_b, int64_t score_every, double *X, double *best,
                   int64_t *best_step, uint8_t *z_best) {
  int64_t C = l * B;
  double *Xn = (double *)malloc(sizeof(double) * (size_t)(n * C + 1));
  double *eta = (double *)malloc(sizeof(double) * (size_t)(C + 1));
  uint8_t *z = (uint8_t *)malloc((size_t)(n * B + 1));
  double *cut = (double *)malloc(sizeof(double) * (size_t)(B + 1));
  for (int64_t t = 0; t <= T; t++) {
    if (t % score_every == 0 || t == T) {
      orc_round(n, B, l, lifted, 0, X, z);
      orc_cut_batch(0, n, rp, col, w, B, z, cut);
      orc_best_update(n, B, t, cut, z, best, best_step, z_best);
    }
    if (t == T) break;
    for (int64_t i = 0; i < l; i++)
      for (int64_t b = 0; b < B; b++) eta[i * B + b] = (T_b && t >= T_b[b]) ? 0.0 : eta_b[b];
    orc_step(n, rp, col, w, C, X, Xn, eta, form);
    memcpy(X, Xn, sizeof(double) * (size_t)(n * C));
  }
  free(Xn);
  free(eta);
  free(z);
  free(cut);
}

/* ------------------------------------------------------------------------------------
 * pDECO (Alg. 3) with the population of Sec. 4.3 laid out as column groups.
 * B initialisations are split into K equal groups (member k owns columns
 * [k*B/K, (k+1)*B/K)). Round r:
 *   1. unlifted batch: X = Proj((mean + sqrt(s2) eps)/scale), member k steps tq[k] times
 *      (the batch runs to the longest count; a finished member keeps still) with
 *      eta = 10^eq[k]; mean = IDI draw per column in round 0, else 2 z_prev - 1;
 *   2. lift: every component of initialisation b starts at Proj((2 z* - 1 + sqrt(s2) eps)/scale)
 *      with z* the best vector of step 1; member k uses l_k <= lmax components (the rest
 *      are exactly 0 and stay 0, so they do not change the lifted rounding), eta = 10^el[k],
 *      tl[k] steps;
 *   3. project: z_prev = best vector of the lifted batch;
 *   4. fitness_k = best cut over member k's columns in this round; for the first
 *      evo_rounds rounds the population evolves (orc_evo_next for the step exponents and l;
 *      orc_evo_next_steps for the counts when Tq_min > 0 (range [Tq_min, Tq]) and
 *      Tl_min > 0 (range [Tl_min, Tl])), afterwards every member takes the first-ranked
 *      member's genes.
 * eq, el, lk, tq, tl hold the K initial genes (orc_evo_init draws them) and return the
 * final ones. Returns the best cut; z_out (n bytes) receives its vector.
 * ---------------------------------------------------------------------------------- */
double orc_deco(int64_t n, const int64_t *rp, const int32_t *col, const double *w, int64_t B,
                int64_t K, int32_t lmax, int64_t rounds, int64_t evo_rounds, int64_t Tq,
                int64_t Tl, int64_t Tq_min, int64_t Tl_min, int form, double beta, double s2,
                double scale, uint64_t seed, double *eq, double *el, int32_t *lk, int32_t *tq,
                int32_t *tl, double *trace, uint8_t *z_out) {
  int64_t Cmax = (int64_t)lmax * B;
  double *X = (double *)calloc((size_t)(n * Cmax + 1), sizeof(double));
  double *M = (double *)calloc((size_t)(n * Cmax + 1), sizeof(double));
  double *eta_b = (double *)malloc(sizeof(double) * (size_t)B);
  int64_t *T_b = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);
  double *best = (double *)malloc(sizeof(double) * (size_t)B);
  int64_t *bstep = (int64_t *)malloc(sizeof(int64_t) * (size_t)B);
  uint8_t *zb = (uint8_t *)calloc((size_t)(n * B + 1), 1);
  uint8_t *zprev = (uint8_t *)calloc((size_t)(n + 1), 1);
  double *fit = (double *)malloc(sizeof(double) * (size_t)K);
  double *eq2 = (double *)malloc(sizeof(double) * (size_t)K);
  double *el2 = (double *)malloc(sizeof(double) * (size_t)K);
  int32_t *lk2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
  int32_t *t2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
  int64_t per = B / K;
  double gbest = -INFINITY;
  uint32_t batch = 0;
  for (int64_t r = 0; r < rounds; r++) {
    /* 1. unlifted batch */
    if (r == 0) {
      orc_init_idi(0, n, rp, col, w, B, beta, seed, batch, M);
    } else {
      for (int64_t v = 0; v < n; v++)
        for (int64_t b = 0; b < B; b++) M[v * B + b] = zprev[v] ? 1.0 : -1.0;
    }
    orc_init_gauss(n, B, M, s2, scale, seed, batch, X);
    batch++;
    int64_t tmax = 0;
    for (int64_t b = 0; b < B; b++) {
      eta_b[b] = pow(10.0, eq[b / per]);
      T_b[b] = tq[b / per];
      if (T_b[b] > tmax) tmax = T_b[b];
      best[b] = -INFINITY;
      bstep[b] = -1;
    }
    orc_run_batch(n, rp, col, w, B, 1, 0, form, eta_b, tmax, T_b, 1, X, best, bstep, zb);
    for (int64_t k = 0; k < K; k++) fit[k] = -INFINITY;
    int64_t arg = 0;
    for (int64_t b = 0; b < B; b++) {
      if (best[b] > fit[b / per]) fit[b / per] = best[b];
      if (best[b] > best[arg]) arg = b;
    }
    if (best[arg] > gbest) {
      gbest = best[arg];
      for (int64_t v = 0; v < n; v++) z_out[v] = zb[v * B + arg];
    }
    for (int64_t v = 0; v < n; v++) zprev[v] = zb[v * B + arg];
    /* 2. lift */
    for (int64_t v = 0; v < n; v++)
      for (int64_t i = 0; i < lmax; i++)
        for (int64_t b = 0; b < B; b++) M[v * Cmax + i * B + b] = zprev[v] ? 1.0 : -1.0;
    orc_init_gauss(n, Cmax, M, s2, scale, seed, batch, X);
    batch++;
    for (int64_t v = 0; v < n; v++)
      for (int64_t i = 0; i < lmax; i++)
        for (int64_t b = 0; b < B; b++)
          if (i >= lk[b / per]) X[v * Cmax + i * B + b] = 0.0;
    tmax = 0;
    for (int64_t b = 0; b < B; b++) {
      eta_b[b] = pow(10.0, el[b / per]);
      T_b[b] = tl[b / per];
      if (T_b[b] > tmax) tmax = T_b[b];
      best[b] = -INFINITY;
      bstep[b] = -1;
    }
    orc_run_batch(n, rp, col, w, B, lmax, 1, form, eta_b, tmax, T_b, 1, X, best, bstep, zb);
    /* 3. project */
    arg = 0;
    for (int64_t b = 0; b < B; b++) {
      if (best[b] > fit[b / per]) fit[b / per] = best[b];
      if (best[b] > best[arg]) arg = b;
    }
    if (best[arg] > gbest) {
      gbest = best[arg];
      for (int64_t v = 0; v < n; v++) z_out[v] = zb[v * B + arg];
    }
    for (int64_t v = 0; v < n; v++) zprev[v] = zb[v * B + arg];
    if (trace) trace[r] = gbest;
    /* 4. search */
    if (r < evo_rounds) {
      orc_evo_next(K, fit, eq, el, lk, -4.0, -1.0, lmax, seed, (uint32_t)r, eq2, el2, lk2);
      memcpy(eq, eq2, sizeof(double) * (size_t)K);
      memcpy(el, el2, sizeof(double) * (size_t)K);
      memcpy(lk, lk2, sizeof(int32_t) * (size_t)K);
      if (Tq_min > 0) {
        orc_evo_next_steps(K, fit, tq, Tq_min, Tq, seed, (uint32_t)r, 0, t2);
        memcpy(tq, t2, sizeof(int32_t) * (size_t)K);
      }
      if (Tl_min > 0) {
        orc_evo_next_steps(K, fit, tl, Tl_min, Tl, seed, (uint32_t)r, 1, t2);
        memcpy(tl, t2, sizeof(int32_t) * (size_t)K);
      }
      if (r == evo_rounds - 1) {
        /* after the last evolution the ranked-first member's genes are used everywhere */
        for (int64_t k = 1; k < K; k++) {
          eq[k] = eq[0];
          el[k] = el[0];
          lk[k] = lk[0];
          tq[k] = tq[0];
          tl[k] = tl[0];
        }
      }
    }
  }
  free(X);
  free(M);
  free(eta_b);
  free(T_b);
  free(best);
  free(bstep);
  free(zb);
  free(zprev);
  free(fit);
  free(eq2);
  free(el2);
  free(lk2);
  free(t2);
  return gbest;
}

/* ------------------------------------------------------------------------------------
 * Exact maximum cut by exhaustive search (n <= 30): node n-1 stays on side 0 and the other
 * 2^(n-1) assignments are visited in Gray-code order, one flip at a time, updating the cut
 * by the flipped node's incident weights.
 * ---------------------------------------------------------------------------------- */
double orc_brute_force(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                       uint8_t *z_best) {
  if (n <= 1) {
    if (n == 1) z_best[0] = 0;
    return 0.0;
  }
  uint8_t *z = (uint8_t *)calloc((size_t)n, 1);
  double cut = 0.0, best = 0.0;
  memset(z_best, 0, (size_t)n);
  uint64_t total = (uint64_t)1 << (n - 1);
  for (uint64_t i = 1; i < total; i++) {
    int j = __builtin_ctzll(i); /* Gray code: flip bit j */
    double delta = 0.0;
    for (int64_t k = rp[j]; k < rp[j + 1]; k++) {
      int64_t u = col[k];
      delta += (z[u] == z[j]) ? wt(w, k) : -wt(w, k);
    }
    z[j] ^= 1;
    cut += delta;
    if (cut > best) {
      best = cut;
      memcpy(z_best, z, (size_t)n);
    }
  }
  free(z);
  return best;
}

/* Greedy 1/2-approximation (Sahni-Gonzalez, as described in Appendix C): vertices are
 * taken in a random order; the first goes to S; every later vertex joins the side that
 * cuts more of its weight to already-placed vertices (ties to S). Best of `orders` runs. */
double orc_greedy(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                  int64_t orders, uint64_t seed, uint8_t *z_best) {
  int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int8_t *side = (int8_t *)malloc((size_t)(n + 1)); /* -1 unplaced, 0 / 1 placed */
  double best = -INFINITY;
  uint32_t r[4];
  for (int64_t o = 0; o < orders; o++) {
    for (int64_t v = 0; v < n; v++) perm[v] = v;
    for (int64_t v = n - 1; v > 0; v--) { /* Fisher-Yates with Philox draws */
      draw(seed, (uint32_t)v, (uint32_t)o, P_EVO, 7, r);
      int64_t j = (int64_t)(((uint64_t)r[0] * (uint64_t)(v + 1)) >> 32);
      int64_t tmp = perm[v];
      perm[v] = perm[j];
      perm[j] = tmp;
    }
    for (int64_t v = 0; v < n; v++) side[v] = -1;
    double cut = 0.0;
    for (int64_t i = 0; i < n; i++) {
      int64_t v = perm[i];
      double to0 = 0.0, to1 = 0.0;
      for (int64_t k = rp[v]; k < rp[v + 1]; k++) {
        int64_t u = col[k];
        if (side[u] == 0) to0 += wt(w, k);
        if (side[u] == 1) to1 += wt(w, k);
      }
      /* joining S (side 1) cuts the weight to side 0, and vice versa */
      if (i == 0 || to0 >= to1) {
        side[v] = 1;
        cut += to0;
      } else {
        side[v] = 0;
        cut += to1;
      }
    }
    if (cut > best) {
      best = cut;
      for (int64_t v = 0; v < n; v++) z_best[v] = (uint8_t)side[v];
    }
  }
  free(perm);
  free(side);
  return best;
}
