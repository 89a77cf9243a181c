/*
 * mclg_oracle.c -- reference (oracle) implementation of the D1Q3 Monte Carlo
 * Lattice Gas of Blommel & Wagner (arXiv:1706.01094).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded implementation to
 * check the HIP library against.  It shares no code with that library.
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (see build_oracle.py).
 *
 * Method, with the passages of the paper each part follows:
 *   - occupation numbers n_i(x,t), i in {-1,0,+1}, and the evolution equation
 *     n_i(x+v_i, t+1) = n_i(x,t) + Xi_i            (Sec. "The Monte Carlo
 *     Lattice Gas algorithm", evolution equation after Eq. (LB));
 *   - Xi is the accumulated effect of C binary sub-collisions, each picking a
 *     pair of particles at random (Eq. (select)) and changing the state by
 *     Eq. (omega) with the transition probabilities of Eq. (collcons);
 *   - for D1Q3 the only state-changing collisions are {-1,1} -> {0,0} with
 *     probability lambda and {0,0} -> {-1,1} or {1,-1} with lambda/16 each
 *     (Sec. "A D1Q3 implementation", table of P_{ij->kl});
 *   - periodic boundaries (D1Q3 results, measurement set-up of Fig. 3).
 *
 * Readings of the paper used here (the paper is silent or ambiguous):
 *   R1  the pair of Eq. (select) is an ordered pair of two *distinct*
 *       particles, drawn uniformly among the N(N-1) ordered pairs;
 *   R2  the state n(x,t) is the pre-collision state; one step collides every
 *       site and then streams; step t uses RNG counter t;
 *   R3  sites with N < 2 do not collide;
 *   R4  the C sub-collisions are sampled in one draw from the exact law of the
 *       C-step chain (a matrix power of exact integers), quantised to uint32
 *       thresholds floor(2^32 * cumulative probability), outcome index
 *       = #{k : thr_k <= r}; the literal sub-collision loop ("direct") is used
 *       for sites with N > n_max and, in the tests, to check the law;
 *   R5  random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the
 *       64-bit seed, counter (site word, t, replica, purpose | block << 2);
 *   R6  Poisson initial counts use thresholds built with IEEE double
 *       operations in a fixed order (mco_poisson_thresholds);
 *   R7  Galilean-invariant acceptance (MCO_FLAG_GALILEAN; the remedy the
 *       paper proposes after Eq. (D1Q3relax)): lambda = lambda~ / sqrt(1 +
 *       3 U^2) with U = J / N of the colliding site, rounded down to a
 *       multiple of 2^-32 in two exact steps (mco_galilean_lambda); the
 *       literal loop then accepts with 32-bit words (collide_direct).
 */
#include "mclg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.                           */
/* ------------------------------------------------------------------------ */
void mco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { PURPOSE_COLLIDE = 0, PURPOSE_INIT = 1, PURPOSE_DIRECT = 2 };

static void rng_block(uint64_t seed, uint32_t c0, uint32_t t, uint32_t replica,
                      uint32_t purpose, uint32_t block, uint32_t out[4]) {
  uint32_t ctr[4] = {c0, t, replica, purpose | (block << 2)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  mco_philox4x32_10(ctr, key, out);
}

/* Word stream for the direct sampler of one site: blocks j = 0, 1, ... of
 * purpose DIRECT, the four words of each block consumed in order. */
typedef struct {
  uint64_t seed;
  uint32_t x, t, replica, block, used;
  uint32_t buf[4];
} word_stream;

static uint32_t ws_next(word_stream *w) {
  if (w->used == 4) {
    rng_block(w->seed, w->x, w->t, w->replica, PURPOSE_DIRECT, w->block, w->buf);
    w->block += 1;
    w->used = 0;
  }
  return w->buf[w->used++];
}

/* Exact uniform integer in [0, s), s >= 1: Lemire's multiply-and-reject
 * ("Fast random integer generation in an interval", ACM TOMACS 2019). */
static uint32_t ws_uniform(word_stream *w, uint32_t s) {
  uint64_t m = (uint64_t)ws_next(w) * (uint64_t)s;
  uint32_t l = (uint32_t)m;
  if (l < s) {
    uint32_t thresh = (uint32_t)(-s) % s;
    while (l < thresh) {
      m = (uint64_t)ws_next(w) * (uint64_t)s;
      l = (uint32_t)m;
    }
  }
  return (uint32_t)(m >> 32);
}

/* ------------------------------------------------------------------------ */
/* Arbitrary-precision unsigned integers (little-endian 32-bit limbs).      */
/* ------------------------------------------------------------------------ */
#define BN_MAXL 192 /* 6144 bits */
typedef struct {
  uint32_t n;            /* limbs in use (no leading zero limbs) */
  uint32_t d[BN_MAXL];
} bignum;

static int bn_overflow = 0;

static void bn_trim(bignum *a) {
  while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
}
static void bn_set_u64(bignum *a, uint64_t v) {
  a->n = 0;
  while (v) { a->d[a->n++] = (uint32_t)v; v >>= 32; }
}
static int bn_is_zero(const bignum *a) { return a->n == 0; }
static int bn_cmp(const bignum *a, const bignum *b) {
  if (a->n != b->n) return a->n < b->n ? -1 : 1;
  for (uint32_t i = a->n; i-- > 0;)
    if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
  return 0;
}
/* a += b */
static void bn_add(bignum *a, const bignum *b) {
  uint32_t n = a->n > b->n ? a->n : b->n;
  uint64_t carry = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t s = carry + (i < a->n ? a->d[i] : 0) + (i < b->n ? b->d[i] : 0);
    a->d[i] = (uint32_t)s;
    carry = s >> 32;
  }
  a->n = n;
  if (carry) {
    if (n >= BN_MAXL) { bn_overflow = 1; return; }
    a->d[a->n++] = (uint32_t)carry;
  }
}
/* a -= b, requires a >= b */
static void bn_sub(bignum *a, const bignum *b) {
  int64_t borrow = 0;
  for (uint32_t i = 0; i < a->n; ++i) {
    int64_t s = (int64_t)a->d[i] - (i < b->n ? b->d[i] : 0) - borrow;
    borrow = s < 0;
    a->d[i] = (uint32_t)(s + (borrow ? ((int64_t)1 << 32) : 0));
  }
  bn_trim(a);
}
/* a += b * w for a 64-bit multiplier w, done as two 32-bit passes */
static void bn_addmul_u32_shift(bignum *a, const bignum *b, uint32_t w, uint32_t shift) {
  if (w == 0 || b->n == 0) return;
  uint32_t need = b->n + shift + 1;
  if (need > BN_MAXL) { bn_overflow = 1; return; }
  while (a->n < need) a->d[a->n++] = 0;
  uint64_t carry = 0;
  uint32_t i = 0;
  for (; i < b->n; ++i) {
    uint64_t s = (uint64_t)b->d[i] * w + a->d[i + shift] + carry;
    a->d[i + shift] = (uint32_t)s;
    carry = s >> 32;
  }
  for (uint32_t j = i + shift; carry; ++j) {
    if (j >= BN_MAXL) { bn_overflow = 1; return; }
    if (j >= a->n) a->d[a->n++] = 0;
    uint64_t s = (uint64_t)a->d[j] + carry;
    a->d[j] = (uint32_t)s;
    carry = s >> 32;
  }
  bn_trim(a);
}
static void bn_addmul_u64(bignum *a, const bignum *b, uint64_t w) {
  bn_addmul_u32_shift(a, b, (uint32_t)w, 0);
  bn_addmul_u32_shift(a, b, (uint32_t)(w >> 32), 1);
}
static void bn_mul_u64(bignum *a, uint64_t w) {
  bignum t;
  t.n = 0;
  bn_addmul_u64(&t, a, w);
  *a = t;
}
/* a /= v exactly (v divides a) -- schoolbook long division by a small number */
static void bn_divexact_u32(bignum *a, uint32_t v) {
  uint64_t rem = 0;
  for (uint32_t i = a->n; i-- > 0;) {
    uint64_t cur = (rem << 32) | a->d[i];
    a->d[i] = (uint32_t)(cur / v);
    rem = cur % v;
  }
  bn_trim(a);
}
static void bn_shl1(bignum *a) {
  uint32_t carry = 0;
  for (uint32_t i = 0; i < a->n; ++i) {
    uint32_t nc = a->d[i] >> 31;
    a->d[i] = (a->d[i] << 1) | carry;
    carry = nc;
  }
  if (carry) {
    if (a->n >= BN_MAXL) { bn_overflow = 1; return; }
    a->d[a->n++] = carry;
  }
}
/* floor(2^32 * s / d) for 0 <= s <= d, d > 0; equals 2^32 when s == d.
 * Restoring binary long division, one quotient bit per iteration. */
static uint64_t bn_quantise(const bignum *s, const bignum *d) {
  int c = bn_cmp(s, d);
  if (c == 0) return (uint64_t)1 << 32;
  bignum r = *s;
  uint64_t q = 0;
  for (int bit = 0; bit < 32; ++bit) {
    bn_shl1(&r);
    q <<= 1;
    if (bn_cmp(&r, d) >= 0) {
      bn_sub(&r, d);
      q |= 1;
    }
  }
  return q;
}

/* ------------------------------------------------------------------------ */
/* Exact collision law of one site.                                          */
/*                                                                           */
/* On the fiber of fixed N and J (the conserved mass and momentum, Eq.        */
/* (collcons)) the state is fixed by n0; write a = n_-1, c = n_+1.  One     */
/* sub-collision picks an ordered pair of distinct particles (R1):           */
/*   P(pair {-1,+1}) = 2ac / (N(N-1)),  accepted with P_{-11->00} = lambda  */
/*                   -> n0 += 2                                               */
/*   P(pair {0,0})   = n0(n0-1) / (N(N-1)), accepted with                    */
/*                   P_{00->-11} + P_{00->1-1} = lambda/8 -> n0 -= 2         */
/* Multiplying by D1 = 8 q N (N-1) (lambda = p/q) gives integer weights      */
/*   up = 16 p a c,  down = p n0 (n0 - 1),  stay = D1 - up - down >= 0.      */
/* The C-step law is the C-th power of this tridiagonal matrix (each row of  */
/* its integer power sums to D1^C).                                          */
/* C = infinity (MCO_C_EQUILIBRIUM) uses the fiber's stationary law, which by */
/* detailed balance (Eq. (transprob)) is proportional to                      */
/*   4^n0 N! / (a! n0! c!).                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t m;       /* fiber size */
  uint64_t *thr;    /* m rows of m-1 thresholds */
} block_t;

typedef struct {
  int32_t C;
  uint32_t p, q, nmax;
  int galilean;     /* per-fiber lambda of R7 */
  block_t **blocks; /* index N * (nmax + 1) + absJ, built on first use */
} table_cache;

/* R7: the numerator over 2^32 of lambda~ / sqrt(1 + 3 (J/N)^2) =
 * lambda~ N / sqrt(N^2 + 3 J^2), lambda~ = num / den:
 *   g = the largest integer with g^2 (N^2 + 3 J^2) <= 2^64 N^2 (bisection over
 *       [0, 2^32]; for N = 0 every g qualifies and g = 2^32),
 *   result = floor(g num / den). */
uint64_t mco_galilean_lambda(uint32_t num, uint32_t den, uint64_t N, uint64_t absJ) {
  typedef unsigned __int128 u128;
  const u128 scale = (u128)N * N + 3 * (u128)absJ * absJ;
  const u128 bound = ((u128)N * N) << 64;
  uint64_t lo = 0, hi = (uint64_t)1 << 32;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo + 1) / 2;
    if ((u128)mid * mid * scale <= bound) lo = mid;
    else hi = mid - 1;
  }
  return (uint64_t)((u128)lo * num / den);
}

static void fiber_geometry(uint32_t N, uint32_t absJ, uint32_t k,
                           uint64_t *n0, uint64_t *a, uint64_t *c) {
  uint32_t par = (N - absJ) & 1u;
  *n0 = par + 2ull * k;
  *a = (N - *n0 - absJ) / 2;
  *c = (N - *n0 + absJ) / 2;
}

static int build_row(int32_t C, uint64_t p, uint64_t q, uint32_t N, uint32_t absJ,
                     uint32_t k0, uint64_t *thr) {
  uint32_t m = (N - absJ) / 2 + 1;
  if (m == 1) return MCO_OK;
  bignum *v = (bignum *)calloc(m, sizeof(bignum));
  bignum *w = (bignum *)calloc(m, sizeof(bignum));
  if (!v || !w) { free(v); free(w); return MCO_E_NOMEM; }
  bn_overflow = 0;
  bignum total;
  if (C == MCO_C_EQUILIBRIUM) {
    /* stationary weights 4^n0 * binom(N, n0) * binom(N - n0, a) */
    for (uint32_t k = 0; k < m; ++k) {
      uint64_t n0, a, c;
      fiber_geometry(N, absJ, k, &n0, &a, &c);
      bignum b;
      bn_set_u64(&b, 1);
      for (uint64_t i = 1; i <= n0; ++i) { bn_mul_u64(&b, N - n0 + i); bn_divexact_u32(&b, (uint32_t)i); }
      for (uint64_t i = 1; i <= a; ++i) { bn_mul_u64(&b, (N - n0) - a + i); bn_divexact_u32(&b, (uint32_t)i); }
      for (uint64_t i = 0; i < n0; ++i) bn_mul_u64(&b, 4);
      v[k] = b;
    }
    total.n = 0;
    for (uint32_t k = 0; k < m; ++k) bn_add(&total, &v[k]);
  } else {
    const uint64_t D1 = 8ull * q * N * (N - 1ull);
    for (uint32_t k = 0; k < m; ++k) v[k].n = 0;
    bn_set_u64(&v[k0], 1);
    bn_set_u64(&total, 1);
    for (int32_t step = 0; step < C; ++step) {
      for (uint32_t j = 0; j < m; ++j) w[j].n = 0;
      for (uint32_t k = 0; k < m; ++k) {
        if (bn_is_zero(&v[k])) continue;
        uint64_t n0, a, c;
        fiber_geometry(N, absJ, k, &n0, &a, &c);
        uint64_t up = 16ull * p * a * c;
        uint64_t down = p * n0 * (n0 - (n0 > 0));
        uint64_t stay = D1 - up - down;
        bn_addmul_u64(&w[k], &v[k], stay);
        if (up) bn_addmul_u64(&w[k + 1], &v[k], up);
        if (down) bn_addmul_u64(&w[k - 1], &v[k], down);
      }
      bignum *tmp = v; v = w; w = tmp;
      bn_mul_u64(&total, D1);
    }
  }
  bignum cum;
  cum.n = 0;
  for (uint32_t k = 0; k + 1 < m; ++k) {
    bn_add(&cum, &v[k]);
    thr[k] = bn_quantise(&cum, &total);
  }
  free(v);
  free(w);
  return bn_overflow ? MCO_E_RANGE : MCO_OK;
}

static int cache_block(table_cache *tc, uint32_t N, uint32_t absJ, const block_t **out) {
  size_t idx = (size_t)N * (tc->nmax + 1) + absJ;
  if (!tc->blocks[idx]) {
    uint32_t m = (N - absJ) / 2 + 1;
    block_t *b = (block_t *)calloc(1, sizeof(block_t));
    if (!b) return MCO_E_NOMEM;
    b->m = m;
    b->thr = (uint64_t *)calloc((size_t)m * (m > 1 ? m - 1 : 1), sizeof(uint64_t));
    if (!b->thr) { free(b); return MCO_E_NOMEM; }
    uint64_t p = tc->p, q = tc->q;
    if (tc->galilean) { p = mco_galilean_lambda(tc->p, tc->q, N, absJ); q = (uint64_t)1 << 32; }
    for (uint32_t k0 = 0; k0 < m; ++k0) {
      int rc = build_row(tc->C, p, q, N, absJ, k0, b->thr + (size_t)k0 * (m - 1));
      if (rc) { free(b->thr); free(b); return rc; }
    }
    tc->blocks[idx] = b;
  }
  *out = tc->blocks[idx];
  return MCO_OK;
}

static int cache_init(table_cache *tc, int32_t C, uint32_t p, uint32_t q, uint32_t nmax,
                      int galilean) {
  tc->C = C; tc->p = p; tc->q = q; tc->nmax = nmax; tc->galilean = galilean;
  tc->blocks = (block_t **)calloc((size_t)(nmax + 1) * (nmax + 1), sizeof(block_t *));
  return tc->blocks ? MCO_OK : MCO_E_NOMEM;
}
static void cache_free(table_cache *tc) {
  if (!tc->blocks) return;
  size_t n = (size_t)(tc->nmax + 1) * (tc->nmax + 1);
  for (size_t i = 0; i < n; ++i)
    if (tc->blocks[i]) { free(tc->blocks[i]->thr); free(tc->blocks[i]); }
  free(tc->blocks);
  tc->blocks = NULL;
}

static int params_valid(int32_t C, uint32_t p, uint32_t q, uint32_t nmax) {
  if (q == 0 || p == 0 || p > q || q >= (1u << 28)) return 0; /* lambda in (0, 1] */
  if (C < MCO_C_EQUILIBRIUM || C > 4096) return 0;
  if (nmax > 4096) return 0;
  return 1;
}

int mco_row_thresholds(int32_t C, uint32_t p, uint32_t q, uint32_t flags, uint32_t N,
                       uint32_t absJ, uint32_t n0, uint64_t *thr, uint32_t *m_out) {
  if (!params_valid(C, p, q, N) || absJ > N || n0 > N - absJ || ((N - absJ - n0) & 1u) ||
      (flags & ~(uint32_t)MCO_FLAG_GALILEAN))
    return MCO_E_INVAL;
  uint32_t m = (N - absJ) / 2 + 1;
  *m_out = m;
  if (N < 2 || m == 1) {
    for (uint32_t k = 0; k + 1 < m; ++k) thr[k] = 0;
    return MCO_OK;
  }
  uint32_t par = (N - absJ) & 1u;
  if (flags & MCO_FLAG_GALILEAN)
    return build_row(C, mco_galilean_lambda(p, q, N, absJ), (uint64_t)1 << 32, N, absJ,
                     (n0 - par) / 2, thr);
  return build_row(C, p, q, N, absJ, (n0 - par) / 2, thr);
}

/* ------------------------------------------------------------------------ */
/* One site collision.                                                       */
/* ------------------------------------------------------------------------ */
/* The paper's literal loop for D1Q3 (Eq. (select), Eq. (omega), repeated C
 * times, each sub-collision acting on the state left by the previous one). */
static void collide_direct(int32_t C, uint32_t p, uint32_t q, int galilean, word_stream *ws,
                           uint64_t *a, uint64_t *b, uint64_t *c) {
  uint64_t N = *a + *b + *c;
  if (N < 2) return;
  /* R7: lambda = lam / 2^32 for the site's conserved (N, |J|) */
  const uint64_t lam = galilean ? mco_galilean_lambda(p, q, N, *c > *a ? *c - *a : *a - *c) : 0;
  for (int32_t sub = 0; sub < C; ++sub) {
    uint32_t r1 = ws_uniform(ws, (uint32_t)N);
    uint32_t r2 = ws_uniform(ws, (uint32_t)(N - 1));
    if (r2 >= r1) r2 += 1; /* ordered pair of distinct particles (R1) */
    /* Eq. (select): velocity of particle r by cumulative sums in the order
     * -1, 0, +1 */
    int s1 = r1 < *a ? -1 : (r1 < *a + *b ? 0 : 1);
    int s2 = r2 < *a ? -1 : (r2 < *a + *b ? 0 : 1);
    if (s1 * s2 == -1) {
      /* {-1,+1} -> {0,0} with probability lambda: a uniform integer below q
       * (below 2^32 under R7, one word) compared with the numerator */
      int accept = galilean ? (uint64_t)ws_next(ws) < lam : ws_uniform(ws, q) < p;
      if (accept) { *a -= 1; *c -= 1; *b += 2; }
    } else if (s1 == 0 && s2 == 0) {
      /* {0,0} -> {-1,1} or {1,-1}, total probability lambda/8: a uniform
       * integer below 8q (below 2^35 under R7: 8 w1 + the top three bits of
       * w2) compared with the numerator */
      int accept;
      if (galilean) {
        uint64_t w1 = ws_next(ws);
        uint64_t w2 = ws_next(ws);
        accept = w1 * 8u + (w2 >> 29) < lam;
      } else {
        accept = ws_uniform(ws, 8u * q) < p;
      }
      if (accept) { *b -= 2; *a += 1; *c += 1; }
    }
  }
}

typedef struct {
  int32_t C;
  uint32_t p, q, nmax;
  int galilean;
  uint64_t seed;
  table_cache tc;
} collide_params;

/* returns 0, or MCO_E_RANGE if the site could not be collided (then it is
 * left unchanged) */
static int collide_site(collide_params *cp, uint32_t replica, uint32_t t, uint32_t x,
                        uint64_t *a, uint64_t *b, uint64_t *c, int force_direct) {
  uint64_t N = *a + *b + *c;
  if (N > 65535u) return MCO_E_RANGE;
  if (N < 2 || cp->C == 0) return MCO_OK;
  int64_t J = (int64_t)*c - (int64_t)*a;
  uint32_t absJ = (uint32_t)(J < 0 ? -J : J);
  uint64_t b_new;
  if (!force_direct && N <= cp->nmax) {
    uint32_t words[4];
    rng_block(cp->seed, x >> 2, t, replica, PURPOSE_COLLIDE, 0, words);
    uint32_t r = words[x & 3u];
    const block_t *blk;
    int rc = cache_block(&cp->tc, (uint32_t)N, absJ, &blk);
    if (rc) return rc;
    uint32_t par = (uint32_t)(N - absJ) & 1u;
    uint32_t k0 = (uint32_t)(*b - par) / 2;
    const uint64_t *row = blk->thr + (size_t)k0 * (blk->m - 1);
    uint32_t idx = 0;
    for (uint32_t k = 0; k + 1 < blk->m; ++k) idx += (row[k] <= r);
    b_new = par + 2ull * idx;
  } else if (cp->C == MCO_C_EQUILIBRIUM) {
    return MCO_E_RANGE;
  } else {
    word_stream ws = {cp->seed, x, t, replica, 0, 4, {0, 0, 0, 0}};
    uint64_t aa = *a, bb = *b, cc = *c;
    collide_direct(cp->C, cp->p, cp->q, cp->galilean, &ws, &aa, &bb, &cc);
    b_new = bb;
  }
  /* exact conservation of N and J (Eq. (collcons)) */
  *a = (uint64_t)(((int64_t)N - (int64_t)b_new - J) / 2);
  *c = (uint64_t)(((int64_t)N - (int64_t)b_new + J) / 2);
  *b = b_new;
  return MCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium and Poisson initial state.                                    */
/* ------------------------------------------------------------------------ */
/* Eq. (D1Q3equil) in the component form printed just before it, evaluated
 * in IEEE double in exactly this order (no fused multiply-add). */
void mco_feq(double rho, double u, double out[3]) {
  double s = sqrt(1.0 + 3.0 * (u * u));
  out[0] = (rho / 6.0) * ((-1.0 - 3.0 * u) + 2.0 * s);
  out[1] = ((2.0 * rho) / 3.0) * (2.0 - s);
  out[2] = (rho / 6.0) * ((-1.0 + 3.0 * u) + 2.0 * s);
}

/* Poisson law of Eq. (poisson): unnormalised weights w_k relative to the
 * mode m = floor(mu), w_m = 1, extended up by w_{k+1} = w_k mu / (k+1) and
 * down by w_{k-1} = w_k k / mu while w >= 2^-60; S = sum of w ascending;
 * thr = floor(2^32 * (running sum / S)) for all but the last outcome. */
int mco_poisson_thresholds(double mu, uint32_t *k_lo, uint32_t *cnt, uint64_t *thr,
                           uint32_t cap) {
  if (!(mu > 0.0)) { *k_lo = 0; *cnt = 1; return MCO_OK; }
  if (mu > 1.0e6) return MCO_E_INVAL;
  const double tiny = ldexp(1.0, -60);
  uint32_t m = (uint32_t)floor(mu);
  /* count the range first */
  uint32_t hi = m, lo = m;
  double w = 1.0;
  for (;;) {
    double wn = (w * mu) / (double)(hi + 1);
    if (wn < tiny) break;
    w = wn; hi++;
  }
  w = 1.0;
  while (lo > 0) {
    double wn = (w * (double)lo) / mu;
    if (wn < tiny) break;
    w = wn; lo--;
  }
  uint32_t n = hi - lo + 1;
  if (n - 1 > cap) return MCO_E_INVAL;
  double *wk = (double *)malloc(sizeof(double) * n);
  if (!wk) return MCO_E_NOMEM;
  wk[m - lo] = 1.0;
  for (uint32_t k = m; k < hi; ++k) wk[k + 1 - lo] = (wk[k - lo] * mu) / (double)(k + 1);
  for (uint32_t k = m; k > lo; --k) wk[k - 1 - lo] = (wk[k - lo] * (double)k) / mu;
  double S = 0.0;
  for (uint32_t i = 0; i < n; ++i) S += wk[i];
  double cum = 0.0;
  for (uint32_t i = 0; i + 1 < n; ++i) {
    cum += wk[i];
    thr[i] = (uint64_t)floor(ldexp(cum / S, 32));
  }
  free(wk);
  *k_lo = lo;
  *cnt = n;
  return MCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Simulation object.                                                        */
/* ------------------------------------------------------------------------ */
struct mco_sim {
  uint32_t n_rep;
  uint32_t flags;
  collide_params cp;
  uint64_t *L;
  uint64_t *rid;
  uint64_t *xoff;  /* RNG site index = x + xoff (window of a larger lattice) */
  int64_t *t;
  uint16_t **cur, **nxt; /* per replica [3][L] logical order */
  int range_error;
};

int mco_create(uint32_t n_rep, const uint64_t *L, const uint64_t *replica_id, uint64_t seed,
               int32_t C, uint32_t lam_p, uint32_t lam_q, uint32_t n_max, uint32_t flags,
               mco_sim **out) {
  if (!out || n_rep == 0 || !L || !params_valid(C, lam_p, lam_q, n_max)) return MCO_E_INVAL;
  for (uint32_t r = 0; r < n_rep; ++r) {
    if (L[r] == 0 || L[r] >= (1ull << 32)) return MCO_E_INVAL;
    if (replica_id && replica_id[r] >= (1ull << 32)) return MCO_E_INVAL;
  }
  mco_sim *s = (mco_sim *)calloc(1, sizeof(mco_sim));
  if (!s) return MCO_E_NOMEM;
  s->n_rep = n_rep;
  s->flags = flags;
  s->cp.C = C; s->cp.p = lam_p; s->cp.q = lam_q; s->cp.nmax = n_max; s->cp.seed = seed;
  s->cp.galilean = (flags & MCO_FLAG_GALILEAN) != 0;
  s->L = (uint64_t *)calloc(n_rep, sizeof(uint64_t));
  s->rid = (uint64_t *)calloc(n_rep, sizeof(uint64_t));
  s->xoff = (uint64_t *)calloc(n_rep, sizeof(uint64_t));
  s->t = (int64_t *)calloc(n_rep, sizeof(int64_t));
  s->cur = (uint16_t **)calloc(n_rep, sizeof(uint16_t *));
  s->nxt = (uint16_t **)calloc(n_rep, sizeof(uint16_t *));
  int bad = !s->L || !s->rid || !s->xoff || !s->t || !s->cur || !s->nxt ||
            cache_init(&s->cp.tc, C, lam_p, lam_q, n_max, s->cp.galilean);
  for (uint32_t r = 0; !bad && r < n_rep; ++r) {
    s->L[r] = L[r];
    s->rid[r] = replica_id ? replica_id[r] : r;
    s->cur[r] = (uint16_t *)calloc(3 * L[r], sizeof(uint16_t));
    s->nxt[r] = (uint16_t *)calloc(3 * L[r], sizeof(uint16_t));
    bad = !s->cur[r] || !s->nxt[r];
  }
  if (bad) { mco_destroy(s); return MCO_E_NOMEM; }
  *out = s;
  return MCO_OK;
}

void mco_destroy(mco_sim *s) {
  if (!s) return;
  for (uint32_t r = 0; r < s->n_rep; ++r) {
    if (s->cur) free(s->cur[r]);
    if (s->nxt) free(s->nxt[r]);
  }
  free(s->cur); free(s->nxt); free(s->L); free(s->rid); free(s->xoff); free(s->t);
  cache_free(&s->cp.tc);
  free(s);
}

int mco_init_counts(mco_sim *s, uint32_t rep, const uint16_t *counts) {
  if (!s || rep >= s->n_rep || !counts) return MCO_E_INVAL;
  memcpy(s->cur[rep], counts, 3 * s->L[rep] * sizeof(uint16_t));
  s->t[rep] = 0;
  return MCO_OK;
}

int mco_init_poisson(mco_sim *s, uint32_t rep, double rho, double u0) {
  if (!s || rep >= s->n_rep || !(rho >= 0.0) || !(u0 >= -1.0 && u0 <= 1.0)) return MCO_E_INVAL;
  double mu[3];
  mco_feq(rho, u0, mu);
  enum { CAP = 1 << 16 };
  uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * CAP);
  if (!thr) return MCO_E_NOMEM;
  const uint64_t L = s->L[rep];
  for (int i = 0; i < 3; ++i) {
    uint32_t k_lo, cnt;
    int rc = mco_poisson_thresholds(mu[i], &k_lo, &cnt, thr, CAP);
    if (rc) { free(thr); return rc; }
    for (uint64_t x = 0; x < L; ++x) {
      uint32_t words[4];
      rng_block(s->cp.seed, (uint32_t)(x + s->xoff[rep]), 0, (uint32_t)s->rid[rep], PURPOSE_INIT, 0,
                words);
      uint32_t r = words[i];
      uint32_t idx = 0;
      for (uint32_t k = 0; k + 1 < cnt; ++k) idx += (thr[k] <= r);
      uint32_t n = k_lo + idx;
      if (n > 65535u) { free(thr); return MCO_E_RANGE; }
      s->cur[rep][(uint64_t)i * L + x] = (uint16_t)n;
    }
  }
  free(thr);
  s->t[rep] = 0;
  return MCO_OK;
}

int mco_step_replica(mco_sim *s, uint32_t rep, uint64_t n) {
  if (!s || rep >= s->n_rep) return MCO_E_INVAL;
  const uint64_t L = s->L[rep];
  const int stream = !(s->flags & MCO_FLAG_NO_STREAM);
  int status = MCO_OK;
  for (uint64_t step = 0; step < n; ++step) {
    const uint16_t *in = s->cur[rep];
    uint16_t *out = s->nxt[rep];
    const uint32_t t = (uint32_t)s->t[rep];
    for (uint64_t x = 0; x < L; ++x) {
      uint64_t a = in[x], b = in[L + x], c = in[2 * L + x];
      int rc = collide_site(&s->cp, (uint32_t)s->rid[rep], t, (uint32_t)(x + s->xoff[rep]),
                            &a, &b, &c, 0);
      if (rc == MCO_E_RANGE) status = MCO_E_RANGE;
      else if (rc) return rc;
      if (stream) {
        /* evolution equation: n_i(x + v_i, t + 1) = post-collision n_i(x) */
        out[(x + L - 1) % L] = (uint16_t)a;
        out[L + x] = (uint16_t)b;
        out[2 * L + (x + 1) % L] = (uint16_t)c;
      } else {
        out[x] = (uint16_t)a;
        out[L + x] = (uint16_t)b;
        out[2 * L + x] = (uint16_t)c;
      }
    }
    s->cur[rep] = out;
    s->nxt[rep] = (uint16_t *)in;
    s->t[rep] += 1;
  }
  if (status) s->range_error = 1;
  return status;
}

int mco_step(mco_sim *s, uint64_t n) {
  if (!s) return MCO_E_INVAL;
  int status = MCO_OK;
  for (uint32_t r = 0; r < s->n_rep; ++r) {
    int rc = mco_step_replica(s, r, n);
    if (rc == MCO_E_RANGE) status = rc;
    else if (rc) return rc;
  }
  return status;
}

int mco_get_counts(const mco_sim *s, uint32_t rep, uint16_t *out) {
  if (!s || rep >= s->n_rep || !out) return MCO_E_INVAL;
  memcpy(out, s->cur[rep], 3 * s->L[rep] * sizeof(uint16_t));
  return MCO_OK;
}

int mco_set_site_offset(mco_sim *s, uint32_t rep, uint64_t xoff, int64_t t) {
  if (!s || rep >= s->n_rep || xoff + s->L[rep] >= (1ull << 32) || t < 0) return MCO_E_INVAL;
  s->xoff[rep] = xoff;
  s->t[rep] = t;
  return MCO_OK;
}

int64_t mco_get_t(const mco_sim *s, uint32_t rep) {
  if (!s || rep >= s->n_rep) return -1;
  return s->t[rep];
}

/* Exact integer sums behind the observables of Sec. "Fluctuating properties
 * of the MCLG" (means, Eq. (poisson) variances, the pair products of
 * Eq. (eqn:Poisson2) / Eq. (corr)) and the projections behind Eq. (A).
 * Arithmetic is modulo 2^64 (unsigned), reinterpreted as int64. */
int mco_moments(const mco_sim *s, uint32_t rep, const int32_t *twiddle, uint32_t n_modes,
                mco_moments_t *o) {
  if (!s || rep >= s->n_rep || !o || n_modes > MCO_MAX_MODES) return MCO_E_INVAL;
  if (n_modes > 0 && !twiddle) return MCO_E_INVAL;
  const uint64_t L = s->L[rep];
  const uint16_t *st = s->cur[rep];
  uint64_t sn[3] = {0, 0, 0}, sn2[3] = {0, 0, 0}, snn[3] = {0, 0, 0};
  uint64_t sN = 0, sJ = 0, sN2 = 0, odd = 0, maxN = 0;
  uint64_t four[MCO_MAX_MODES][2];
  memset(four, 0, sizeof(four));
  for (uint64_t x = 0; x < L; ++x) {
    uint64_t a = st[x], b = st[L + x], c = st[2 * L + x];
    uint64_t N = a + b + c;
    sn[0] += a; sn[1] += b; sn[2] += c;
    sn2[0] += a * a; sn2[1] += b * b; sn2[2] += c * c;
    snn[0] += a * b; snn[1] += b * c; snn[2] += a * c;
    sN += N;
    sJ += c - a; /* modulo 2^64 */
    sN2 += N * N;
    odd += b & 1u;
    if (N > maxN) maxN = N;
    for (uint32_t md = 0; md < n_modes; ++md) {
      four[md][0] += N * (uint64_t)(int64_t)twiddle[(2 * md) * L + x];
      four[md][1] += N * (uint64_t)(int64_t)twiddle[(2 * md + 1) * L + x];
    }
  }
  memset(o, 0, sizeof(*o));
  o->t = s->t[rep];
  o->sites = (int64_t)L;
  for (int i = 0; i < 3; ++i) {
    o->sum_n[i] = (int64_t)sn[i];
    o->sum_n2[i] = (int64_t)sn2[i];
    o->sum_nn[i] = (int64_t)snn[i];
  }
  o->sum_N = (int64_t)sN;
  o->sum_J = (int64_t)sJ;
  o->sum_N2 = (int64_t)sN2;
  o->n0_odd = (int64_t)odd;
  o->max_N = (int64_t)maxN;
  for (uint32_t md = 0; md < n_modes; ++md) {
    o->fourier[md][0] = (int64_t)four[md][0];
    o->fourier[md][1] = (int64_t)four[md][1];
  }
  return MCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Single-site entry points for the statistical tests.                       */
/* ------------------------------------------------------------------------ */
static collide_params g_cp;
static int g_cp_valid = 0;

static int global_params(int32_t C, uint32_t p, uint32_t q, uint32_t nmax, int galilean,
                         uint64_t seed) {
  if (!params_valid(C, p, q, nmax)) return MCO_E_INVAL;
  if (!g_cp_valid || g_cp.C != C || g_cp.p != p || g_cp.q != q || g_cp.nmax != nmax ||
      g_cp.galilean != galilean) {
    if (g_cp_valid) cache_free(&g_cp.tc);
    g_cp_valid = 0;
    if (cache_init(&g_cp.tc, C, p, q, nmax, galilean)) return MCO_E_NOMEM;
    g_cp.C = C; g_cp.p = p; g_cp.q = q; g_cp.nmax = nmax; g_cp.galilean = galilean;
    g_cp_valid = 1;
  }
  g_cp.seed = seed;
  return MCO_OK;
}

int mco_collide_site(int32_t C, uint32_t p, uint32_t q, uint32_t flags, uint32_t n_max,
                     uint64_t seed, uint64_t replica, uint64_t t, uint64_t x, uint32_t abc[3]) {
  int rc = global_params(C, p, q, n_max, (flags & MCO_FLAG_GALILEAN) != 0, seed);
  if (rc) return rc;
  uint64_t a = abc[0], b = abc[1], c = abc[2];
  rc = collide_site(&g_cp, (uint32_t)replica, (uint32_t)t, (uint32_t)x, &a, &b, &c, 0);
  abc[0] = (uint32_t)a; abc[1] = (uint32_t)b; abc[2] = (uint32_t)c;
  return rc;
}

int mco_collide_site_direct(int32_t C, uint32_t p, uint32_t q, uint32_t flags, uint64_t seed,
                            uint64_t replica, uint64_t t, uint64_t x, uint32_t abc[3]) {
  if (C < 0 || !params_valid(C, p, q, 0)) return MCO_E_INVAL;
  uint64_t a = abc[0], b = abc[1], c = abc[2];
  word_stream ws = {seed, (uint32_t)x, (uint32_t)t, (uint32_t)replica, 0, 4, {0, 0, 0, 0}};
  collide_direct(C, p, q, (flags & MCO_FLAG_GALILEAN) != 0, &ws, &a, &b, &c);
  abc[0] = (uint32_t)a; abc[1] = (uint32_t)b; abc[2] = (uint32_t)c;
  return MCO_OK;
}

int mco_histogram(int32_t C, uint32_t p, uint32_t q, uint32_t flags, int direct, uint64_t seed,
                  uint64_t t, uint64_t n_draws, const uint32_t abc[3], uint64_t *hist) {
  uint32_t N = abc[0] + abc[1] + abc[2];
  if (!direct) {
    int rc = global_params(C, p, q, N, (flags & MCO_FLAG_GALILEAN) != 0, seed);
    if (rc) return rc;
  }
  for (uint32_t k = 0; k <= N; ++k) hist[k] = 0;
  for (uint64_t x = 0; x < n_draws; ++x) {
    uint32_t s[3] = {abc[0], abc[1], abc[2]};
    int rc = direct ? mco_collide_site_direct(C, p, q, flags, seed, 0, t, x, s)
                    : mco_collide_site(C, p, q, flags, N, seed, 0, t, x, s);
    if (rc) return rc;
    hist[s[1]] += 1;
  }
  return MCO_OK;
}

/* ======================================================================== */
/* D2Q9 (Sec. "A D2Q9 implementation").                                      */
/*                                                                           */
/* Velocities numbered as the columns of the moment matrix Eq. (MomD2Q9):    */
/*   0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1),                          */
/*   5 (1,1), 6 (-1,1), 7 (-1,-1), 8 (1,-1);                                 */
/* weights w = 4/9, 1/9 (axis), 1/36 (diagonal) = 576, 144, 36 / 1296.       */
/* A sub-collision picks an ordered pair of distinct particles (R1) with     */
/* velocities (i, j).  The binary collisions that change the state and       */
/* conserve momentum take the unordered pair A = {i, j} to another unordered */
/* pair B = {k, l} of the same total momentum (R8):                          */
/*   P(A -> B) = lambda_c min(1, m_B w_k w_l / (m_A w_i w_j)),               */
/* m = 2 for two different velocities, 1 for two equal ones: detailed       */
/* balance with respect to the product weights, the faster direction at      */
/* lambda_c, exactly as the D1Q3 table (lambda from {-1,1} to {0,0},         */
/* 2 x lambda/16 back).  The class c of a transition, numbered as the        */
/* lambda_1..9 of Eq. (D2Q9MOmega):                                          */
/*   1 {0,5}<->{1,2} (momentum (1,1)),  2 rest <-> axis pair,                */
/*   3 rest <-> diagonal pair,  4 axis <-> diagonal pair,                    */
/*   5 axis <-> axis pair,  6 diagonal <-> diagonal pair,                    */
/*   7 {0,1}<->{2,8} and {0,1}<->{4,5} (momentum (1,0), with a rest          */
/*     particle),  8 {2,8}<->{4,5},  9 {1,1}<->{5,8} (momentum (2,0)),       */
/* and their rotations by multiples of 90 degrees.                           */
/* One uniform integer u in [0, D), D = lcm(lambda denominators) * 2^7,      */
/* picks the target: targets of A in ascending (min(k,l), max(k,l)), u below */
/* the running sum of their integer weights D P(A -> B) selects one, else    */
/* nothing changes.  Random words: R9 (collide9).                            */
/* ======================================================================== */
static const int V9[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                             {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
static const uint64_t W9[9] = {576, 144, 144, 144, 144, 36, 36, 36, 36};

static int kind9(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 2); } /* rest, axis, diagonal */

/* class (1..9) of the transition between unordered pairs {i,j} and {k,l}
 * of equal momentum, 0 if they are the same pair */
static int class9(int i, int j, int k, int l) {
  if ((i == k && j == l) || (i == l && j == k)) return 0;
  int px = V9[i][0] + V9[j][0], py = V9[i][1] + V9[j][1];
  if (px == 0 && py == 0) {
    int a = kind9(i) == 0 ? 0 : kind9(i), b = kind9(k);
    if (a > b) { int t = a; a = b; b = t; }
    if (a == 0 && b == 1) return 2;
    if (a == 0 && b == 2) return 3;
    if (a == 1 && b == 2) return 4;
    if (a == 1 && b == 1) return 5;
    return 6;
  }
  if (abs(px) + abs(py) == 1) return (i == 0 || j == 0 || k == 0 || l == 0) ? 7 : 8;
  if (abs(px) == 1 && abs(py) == 1) return 1;
  return 9; /* |p| = 2 along an axis */
}

typedef struct {
  uint32_t n;         /* number of targets */
  uint8_t k[8], l[8]; /* target pair, k <= l */
  uint8_t cls[8];
  uint64_t wgt[8];    /* integer weight D * P */
} targets9;

typedef struct {
  uint64_t D;
  targets9 tg[9][9]; /* by ordered source (i, j) */
} rules9;

static uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) { uint64_t t = a % b; a = b; b = t; }
  return a;
}

/* lam[2c-2], lam[2c-1] = numerator, denominator of lambda_c */
static int rules9_build(const uint32_t lam[18], rules9 *R) {
  uint64_t L = 1;
  for (int c = 0; c < 9; ++c) {
    if (lam[2 * c + 1] == 0 || lam[2 * c] > lam[2 * c + 1]) return MCO_E_INVAL;
    L = L / gcd64(L, lam[2 * c + 1]) * lam[2 * c + 1];
    if (L >= (1u << 25)) return MCO_E_INVAL;
  }
  R->D = L << 7;
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      targets9 *T = &R->tg[i][j];
      T->n = 0;
      uint64_t mA = (i == j) ? 1 : 2, sum = 0;
      for (int k = 0; k < 9; ++k)
        for (int l = k; l < 9; ++l) {
          if (V9[k][0] + V9[l][0] != V9[i][0] + V9[j][0] ||
              V9[k][1] + V9[l][1] != V9[i][1] + V9[j][1])
            continue;
          int c = class9(i, j, k, l);
          if (!c) continue;
          uint64_t mB = (k == l) ? 1 : 2;
          uint64_t num = mB * W9[k] * W9[l], den = mA * W9[i] * W9[j];
          /* D * lambda_c * min(1, num / den), exact (num/den is a power of 2 >= 2^-7) */
          uint64_t base = R->D / lam[2 * c - 1] * lam[2 * c - 2];
          uint64_t w = num >= den ? base : base * num / den;
          if (num < den && (base * num) % den) return MCO_E_INVAL; /* cannot happen */
          T->k[T->n] = (uint8_t)k; T->l[T->n] = (uint8_t)l; T->cls[T->n] = (uint8_t)c;
          T->wgt[T->n] = w;
          T->n++;
          sum += w;
        }
      if (sum > R->D) return MCO_E_INVAL; /* total probability above one */
    }
  return MCO_OK;
}

int mco9_targets(const uint32_t lam[18], uint32_t i, uint32_t j, uint32_t *n, uint32_t k[8],
                 uint32_t l[8], uint32_t cls[8], uint64_t wgt[8], uint64_t *D) {
  if (i > 8 || j > 8) return MCO_E_INVAL;
  rules9 R;
  int rc = rules9_build(lam, &R);
  if (rc) return rc;
  const targets9 *T = &R.tg[i][j];
  *n = T->n;
  for (uint32_t q = 0; q < T->n; ++q) {
    k[q] = T->k[q]; l[q] = T->l[q]; cls[q] = T->cls[q]; wgt[q] = T->wgt[q];
  }
  *D = R.D;
  return MCO_OK;
}

/* Lemire's draw of a uniform integer in [0, s) whose first word is given;
 * rejected draws continue with words of the stream `more`. */
static uint32_t uniform_from(uint32_t first, uint32_t s, word_stream *more) {
  uint64_t m = (uint64_t)first * (uint64_t)s;
  uint32_t l = (uint32_t)m;
  if (l < s) {
    uint32_t thresh = (uint32_t)(-s) % s;
    while (l < thresh) {
      m = (uint64_t)ws_next(more) * (uint64_t)s;
      l = (uint32_t)m;
    }
  }
  return (uint32_t)(m >> 32);
}

/* The literal loop of C sub-collisions at one D2Q9 site (R1, R8).  R9:
 * sub-collision k takes Philox block (s, t, replica, DIRECT | k << 2): word
 * 0 draws the first particle (of N), word 1 the second (of N - 1), word 2
 * the target (of D), always; a rejected draw continues with the words of
 * the blocks (s, t, replica, DIRECT | (C + j) << 2), j = 0, 1, ..., shared by
 * the site's step. */
static void collide9(int32_t C, const rules9 *R, uint64_t seed, uint32_t s, uint32_t t,
                     uint32_t replica, uint64_t n[9]) {
  uint64_t N = 0;
  for (int i = 0; i < 9; ++i) N += n[i];
  if (N < 2) return;
  word_stream more = {seed, s, t, replica, (uint32_t)C, 4, {0, 0, 0, 0}};
  for (int32_t sub = 0; sub < C; ++sub) {
    uint32_t w[4];
    rng_block(seed, s, t, replica, PURPOSE_DIRECT, (uint32_t)sub, w);
    uint32_t r1 = uniform_from(w[0], (uint32_t)N, &more);
    uint32_t r2 = uniform_from(w[1], (uint32_t)(N - 1), &more);
    uint32_t u = uniform_from(w[2], (uint32_t)R->D, &more);
    if (r2 >= r1) r2 += 1;
    /* Eq. (select): velocity by cumulative sums in the order 0..8 */
    int v1 = 0, v2 = 0;
    uint64_t cum = 0;
    for (int i = 0; i < 9; ++i) { cum += n[i]; if (r1 >= cum) v1 = i + 1; }
    cum = 0;
    for (int i = 0; i < 9; ++i) { cum += n[i]; if (r2 >= cum) v2 = i + 1; }
    const targets9 *T = &R->tg[v1][v2];
    uint64_t run = 0;
    for (uint32_t q = 0; q < T->n; ++q) {
      run += T->wgt[q];
      if (u < run) {
        n[v1] -= 1; n[v2] -= 1; n[T->k[q]] += 1; n[T->l[q]] += 1; /* Eq. (omega) */
        break;
      }
    }
  }
}

int mco9_collide_site(int32_t C, const uint32_t lam[18], uint64_t seed, uint64_t replica,
                      uint64_t t, uint64_t s, uint32_t n9[9]) {
  if (C < 0) return MCO_E_INVAL;
  rules9 R;
  int rc = rules9_build(lam, &R);
  if (rc) return rc;
  uint64_t n[9];
  for (int i = 0; i < 9; ++i) n[i] = n9[i];
  collide9(C, &R, seed, (uint32_t)s, (uint32_t)t, (uint32_t)replica, n);
  for (int i = 0; i < 9; ++i) n9[i] = (uint32_t)n[i];
  return MCO_OK;
}

/* Eq. (D2Q9eqdist): the product of the D1Q3 equilibria of Eq. (D1Q3equil)
 * at unit density, times rho, evaluated as (rho * Fx[vx]) * Fy[vy]. */
void mco9_feq(double rho, double ux, double uy, double out[9]) {
  double fx[3], fy[3];
  mco_feq(1.0, ux, fx);
  mco_feq(1.0, uy, fy);
  for (int i = 0; i < 9; ++i) out[i] = (rho * fx[V9[i][0] + 1]) * fy[V9[i][1] + 1];
}

struct mco_sim9 {
  uint32_t n_rep, flags;
  int32_t C;
  uint64_t seed;
  rules9 R;
  uint64_t *Lx, *Ly, *rid;
  int64_t *t;
  uint16_t **cur, **nxt; /* per replica [9][Ly][Lx] */
};

void mco9_destroy(mco_sim9 *s) {
  if (!s) return;
  for (uint32_t r = 0; r < s->n_rep; ++r) {
    if (s->cur) free(s->cur[r]);
    if (s->nxt) free(s->nxt[r]);
  }
  free(s->cur); free(s->nxt); free(s->Lx); free(s->Ly); free(s->rid); free(s->t);
  free(s);
}

int mco9_create(uint32_t n_rep, const uint64_t *Lx, const uint64_t *Ly,
                const uint64_t *replica_id, uint64_t seed, int32_t C, const uint32_t lam[18],
                uint32_t flags, mco_sim9 **out) {
  if (!out || !n_rep || !Lx || !Ly || C < 0 || C > 4096 || (flags & ~(uint32_t)MCO_FLAG_NO_STREAM))
    return MCO_E_INVAL;
  mco_sim9 *s = (mco_sim9 *)calloc(1, sizeof(mco_sim9));
  if (!s) return MCO_E_NOMEM;
  int rc = rules9_build(lam, &s->R);
  if (rc) { free(s); return rc; }
  s->n_rep = n_rep; s->flags = flags; s->C = C; s->seed = seed;
  s->Lx = (uint64_t *)calloc(n_rep, 8); s->Ly = (uint64_t *)calloc(n_rep, 8);
  s->rid = (uint64_t *)calloc(n_rep, 8); s->t = (int64_t *)calloc(n_rep, 8);
  s->cur = (uint16_t **)calloc(n_rep, sizeof(uint16_t *));
  s->nxt = (uint16_t **)calloc(n_rep, sizeof(uint16_t *));
  if (!s->Lx || !s->Ly || !s->rid || !s->t || !s->cur || !s->nxt) { mco9_destroy(s); return MCO_E_NOMEM; }
  for (uint32_t r = 0; r < n_rep; ++r) {
    if (!Lx[r] || !Ly[r] || Lx[r] * Ly[r] >= (1ull << 32) ||
        (replica_id && replica_id[r] >= (1ull << 32))) {
      mco9_destroy(s);
      return MCO_E_INVAL;
    }
    s->Lx[r] = Lx[r]; s->Ly[r] = Ly[r];
    s->rid[r] = replica_id ? replica_id[r] : r;
    s->cur[r] = (uint16_t *)calloc(9 * Lx[r] * Ly[r], 2);
    s->nxt[r] = (uint16_t *)calloc(9 * Lx[r] * Ly[r], 2);
    if (!s->cur[r] || !s->nxt[r]) { mco9_destroy(s); return MCO_E_NOMEM; }
  }
  *out = s;
  return MCO_OK;
}

int mco9_init_counts(mco_sim9 *s, uint32_t rep, const uint16_t *counts) {
  if (!s || rep >= s->n_rep || !counts) return MCO_E_INVAL;
  memcpy(s->cur[rep], counts, 9 * s->Lx[rep] * s->Ly[rep] * 2);
  s->t[rep] = 0;
  return MCO_OK;
}

/* n_i(x, y) ~ Poisson(f_i^eq(rho, ux, uy)) with the threshold rule of R6;
 * site s = y Lx + x draws Philox blocks (s, j, replica, INIT) for j = 0, 1,
 * 2, word w of block j serving velocity 4 j + w. */
int mco9_init_poisson(mco_sim9 *s, uint32_t rep, double rho, double ux, double uy) {
  if (!s || rep >= s->n_rep || !(rho >= 0.0) || !(ux >= -1.0 && ux <= 1.0) ||
      !(uy >= -1.0 && uy <= 1.0))
    return MCO_E_INVAL;
  double mu[9];
  mco9_feq(rho, ux, uy, mu);
  enum { CAP = 1 << 16 };
  uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * CAP);
  if (!thr) return MCO_E_NOMEM;
  const uint64_t S = s->Lx[rep] * s->Ly[rep];
  for (int i = 0; i < 9; ++i) {
    uint32_t k_lo, cnt;
    int rc = mco_poisson_thresholds(mu[i], &k_lo, &cnt, thr, CAP);
    if (rc) { free(thr); return rc; }
    for (uint64_t x = 0; x < S; ++x) {
      uint32_t words[4];
      uint32_t ctr[4] = {(uint32_t)x, (uint32_t)(i / 4), (uint32_t)s->rid[rep], PURPOSE_INIT};
      uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
      mco_philox4x32_10(ctr, key, words);
      uint32_t r = words[i % 4];
      uint32_t idx = 0;
      for (uint32_t k = 0; k + 1 < cnt; ++k) idx += (thr[k] <= r);
      uint32_t n = k_lo + idx;
      if (n > 65535u) { free(thr); return MCO_E_RANGE; }
      s->cur[rep][(uint64_t)i * S + x] = (uint16_t)n;
    }
  }
  free(thr);
  s->t[rep] = 0;
  return MCO_OK;
}

/* One step: the literal loop at every site (pre-collision state, RNG counter
 * t, R2), then n_i(x + vx, y + vy) <- post-collision n_i(x, y), periodic. */
int mco9_step(mco_sim9 *s, uint64_t nsteps) {
  if (!s) return MCO_E_INVAL;
  int status = MCO_OK;
  const int stream = !(s->flags & MCO_FLAG_NO_STREAM);
  for (uint32_t r = 0; r < s->n_rep; ++r) {
    const uint64_t Lx = s->Lx[r], Ly = s->Ly[r], S = Lx * Ly;
    for (uint64_t st = 0; st < nsteps; ++st) {
      const uint16_t *in = s->cur[r];
      uint16_t *out = s->nxt[r];
      for (uint64_t y = 0; y < Ly; ++y)
        for (uint64_t x = 0; x < Lx; ++x) {
          const uint64_t site = y * Lx + x;
          uint64_t n[9], N = 0;
          for (int i = 0; i < 9; ++i) { n[i] = in[i * S + site]; N += n[i]; }
          if (N > 65535u) {
            status = MCO_E_RANGE; /* not collided (R15) */
          } else {
            collide9(s->C, &s->R, s->seed, (uint32_t)site, (uint32_t)s->t[r], (uint32_t)s->rid[r], n);
          }
          for (int i = 0; i < 9; ++i) {
            uint64_t xd = x, yd = y;
            if (stream) {
              xd = (x + Lx + (uint64_t)(int64_t)V9[i][0]) % Lx;
              yd = (y + Ly + (uint64_t)(int64_t)V9[i][1]) % Ly;
            }
            out[i * S + yd * Lx + xd] = (uint16_t)n[i];
          }
        }
      s->nxt[r] = s->cur[r];
      s->cur[r] = out;
      s->t[r] += 1;
    }
  }
  return status;
}

int mco9_get_counts(const mco_sim9 *s, uint32_t rep, uint16_t *out) {
  if (!s || rep >= s->n_rep || !out) return MCO_E_INVAL;
  memcpy(out, s->cur[rep], 9 * s->Lx[rep] * s->Ly[rep] * 2);
  return MCO_OK;
}

int64_t mco9_get_t(const mco_sim9 *s, uint32_t rep) { return s && rep < s->n_rep ? s->t[rep] : -1; }

/* Exact sums over sites: sum n_i, sum n_i n_j (i <= j, row-major upper
 * triangle, 45 values), sum N, sum Jx, sum Jy, max N. */
int mco9_moments(const mco_sim9 *s, uint32_t rep, mco_moments9_t *o) {
  if (!s || rep >= s->n_rep || !o) return MCO_E_INVAL;
  memset(o, 0, sizeof(*o));
  const uint64_t S = s->Lx[rep] * s->Ly[rep];
  const uint16_t *c = s->cur[rep];
  for (uint64_t x = 0; x < S; ++x) {
    int64_t n[9], N = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
      n[i] = c[i * S + x];
      N += n[i]; jx += V9[i][0] * n[i]; jy += V9[i][1] * n[i];
    }
    int q = 0;
    for (int i = 0; i < 9; ++i) {
      o->sum_n[i] += n[i];
      for (int j = i; j < 9; ++j) o->sum_nn[q++] += n[i] * n[j];
    }
    o->sum_N += N; o->sum_Jx += jx; o->sum_Jy += jy;
    if (N > o->max_N) o->max_N = N;
  }
  o->t = s->t[rep];
  o->sites = (int64_t)S;
  return MCO_OK;
}
