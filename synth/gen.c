/* Seeded synthetic signed bipartite graphs (input generation only).
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, 2014) used as a
 * counter-based generator: value i of stream s under seed k is the SplitMix64
 * output function applied to  base(k, s) + (i + 1) * 0x9e3779b97f4a7c15,
 * with base(k, s) = mix(k) ^ mix(s + 0x632be59bd9b4e019).  A uniform double
 * in [0, 1) takes the top 53 bits.  Discrete laws are sampled with Walker's
 * alias method (Vose's construction).  Repeated pairs are dropped with an
 * open-addressing hash set, so the kept edges are the first m distinct pairs
 * in draw order.
 *
 * Nothing here counts butterflies: this file only draws inputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_base(uint64_t seed, uint64_t stream) {
  return mix64(seed) ^ mix64(stream + 0x632be59bd9b4e019ULL);
}

static inline uint64_t draw_u64(uint64_t base, uint64_t i) {
  return mix64(base + (i + 1) * GOLDEN);
}

static inline double draw_unit(uint64_t base, uint64_t i) {
  return (double)(draw_u64(base, i) >> 11) * 0x1.0p-53;
}

enum { ST_WU = 0, ST_WV = 1, ST_DU = 2, ST_DV = 3, ST_SIGN = 4, ST_UNI = 5 };

/* ---- open-addressing set of 64-bit keys ---------------------------------- */
typedef struct {
  uint64_t *slot; /* key + 1, 0 = empty */
  uint64_t mask;
} keyset;

static int keyset_init(keyset *s, uint64_t want) {
  uint64_t cap = 1024;
  while (cap < 2 * want) cap <<= 1;
  s->slot = (uint64_t *)calloc(cap, sizeof(uint64_t));
  s->mask = cap - 1;
  return s->slot ? 0 : -1;
}

/* returns 1 if inserted, 0 if present */
static inline int keyset_insert(keyset *s, uint64_t key) {
  uint64_t h = mix64(key + GOLDEN) & s->mask;
  for (;;) {
    uint64_t cur = s->slot[h];
    if (cur == 0) {
      s->slot[h] = key + 1;
      return 1;
    }
    if (cur == key + 1) return 0;
    h = (h + 1) & s->mask;
  }
}

/* ---- alias table ----------------------------------------------------------- */
typedef struct {
  double *prob;
  int32_t *alias;
  int64_t n;
} alias_table;

static int alias_build(alias_table *t, const double *w, int64_t n) {
  t->n = n;
  t->prob = (double *)malloc(sizeof(double) * n);
  t->alias = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t *small = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t *large = (int32_t *)malloc(sizeof(int32_t) * n);
  if (!t->prob || !t->alias || !small || !large) {
    free(small);
    free(large);
    return -1;
  }
  double sum = 0.0;
  for (int64_t i = 0; i < n; ++i) sum += w[i];
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    t->prob[i] = w[i] * (double)n / sum;
    t->alias[i] = (int32_t)i;
    if (t->prob[i] < 1.0)
      small[ns++] = (int32_t)i;
    else
      large[nl++] = (int32_t)i;
  }
  while (ns > 0 && nl > 0) {
    int32_t s = small[--ns];
    int32_t l = large[nl - 1];
    t->alias[s] = l;
    t->prob[l] = (t->prob[l] + t->prob[s]) - 1.0;
    if (t->prob[l] < 1.0) {
      --nl;
      small[ns++] = l;
    }
  }
  while (nl > 0) t->prob[large[--nl]] = 1.0;
  while (ns > 0) t->prob[small[--ns]] = 1.0;
  free(small);
  free(large);
  return 0;
}

static void alias_free(alias_table *t) {
  free(t->prob);
  free(t->alias);
}

static inline int64_t alias_draw(const alias_table *t, double x) {
  double y = x * (double)t->n;
  int64_t i = (int64_t)y;
  if (i >= t->n) i = t->n - 1;
  double coin = y - (double)i;
  return coin < t->prob[i] ? i : t->alias[i];
}

/* Pareto weights w = (1 - xi)^(-1/(gamma-1)), capped so that the expected
 * degree m * w / sum(w) is at most d_cap (one renormalisation). */
static double *side_weights(uint64_t seed, int stream, int64_t n, double gamma, int64_t m,
                            double d_cap) {
  double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  if (!w) return NULL;
  uint64_t base = stream_base(seed, (uint64_t)stream);
  double sum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double xi = draw_unit(base, (uint64_t)i);
    w[i] = pow(1.0 - xi, -1.0 / (gamma - 1.0));
    sum += w[i];
  }
  double cap = d_cap * sum / (double)(m > 0 ? m : 1);
  for (int64_t i = 0; i < n; ++i)
    if (w[i] > cap) w[i] = cap;
  return w;
}

static void draw_signs(uint64_t seed, int64_t m, double q, int8_t *s) {
  uint64_t base = stream_base(seed, ST_SIGN);
  for (int64_t i = 0; i < m; ++i) s[i] = draw_unit(base, (uint64_t)i) < q ? (int8_t)-1 : (int8_t)1;
}

/* Chung-Lu bipartite graph.  Returns the number of edges written (m), or -1
 * on allocation failure, -2 if max_draws draws did not yield m distinct
 * pairs, -3 on bad arguments. */
int64_t synth_chung_lu(int64_t n_u, int64_t n_v, int64_t m, double gamma_u, double gamma_v,
                       double q, double dcap_u, double dcap_v, uint64_t seed,
                       int64_t max_draws, int32_t *u_out, int32_t *v_out, int8_t *s_out) {
  if (n_u <= 0 || n_v <= 0 || m < 0 || m > n_u * n_v) return -3;
  if (m == 0) return 0;
  double *wu = side_weights(seed, ST_WU, n_u, gamma_u, m, dcap_u);
  double *wv = side_weights(seed, ST_WV, n_v, gamma_v, m, dcap_v);
  alias_table tu = {0}, tv = {0};
  keyset set = {0};
  int64_t rc = -1;
  if (!wu || !wv || alias_build(&tu, wu, n_u) || alias_build(&tv, wv, n_v) ||
      keyset_init(&set, (uint64_t)m))
    goto done;
  {
    uint64_t bu = stream_base(seed, ST_DU), bv = stream_base(seed, ST_DV);
    int64_t have = 0;
    for (int64_t i = 0; i < max_draws && have < m; ++i) {
      int64_t a = alias_draw(&tu, draw_unit(bu, (uint64_t)i));
      int64_t b = alias_draw(&tv, draw_unit(bv, (uint64_t)i));
      if (keyset_insert(&set, (uint64_t)a * (uint64_t)n_v + (uint64_t)b)) {
        u_out[have] = (int32_t)a;
        v_out[have] = (int32_t)b;
        ++have;
      }
    }
    if (have < m) {
      rc = -2;
      goto done;
    }
  }
  draw_signs(seed, m, q, s_out);
  rc = m;
done:
  free(wu);
  free(wv);
  alias_free(&tu);
  alias_free(&tv);
  free(set.slot);
  return rc;
}

/* m distinct pairs uniform over U x V (rejection of repeats, in draw order). */
int64_t synth_uniform(int64_t n_u, int64_t n_v, int64_t m, double q, uint64_t seed,
                      int32_t *u_out, int32_t *v_out, int8_t *s_out) {
  if (n_u <= 0 || n_v <= 0 || m < 0 || m > n_u * n_v) return -3;
  if (m == 0) return 0;
  keyset set;
  if (keyset_init(&set, (uint64_t)m)) return -1;
  uint64_t base = stream_base(seed, ST_UNI);
  uint64_t total = (uint64_t)n_u * (uint64_t)n_v;
  int64_t have = 0;
  for (uint64_t i = 0; have < m; ++i) {
    uint64_t k = (uint64_t)(draw_unit(base, i) * (double)total);
    if (k >= total) k = total - 1;
    if (keyset_insert(&set, k)) {
      u_out[have] = (int32_t)(k / (uint64_t)n_v);
      v_out[have] = (int32_t)(k % (uint64_t)n_v);
      ++have;
    }
  }
  free(set.slot);
  draw_signs(seed, m, q, s_out);
  return m;
}
