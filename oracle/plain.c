/*
 * O2: plain incremental enumerator for batch-dynamic subgraph matching.
 *
 * TEST INFRASTRUCTURE.  This file is the CPU oracle that the GPU path is
 * checked against.  Only the tests, the package smoke check and the bench's
 * CPU baseline may load it; the product path never does.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes (the paper's problem statement, Sec. II-A, Def. 1 and
 * Def. 2, with the net set-difference reading of the incremental matches):
 *   canonical batch  : each update (op, u, v) becomes (op, min, max); self
 *                      loops and ids >= n are rejected; exact duplicates
 *                      collapse; a batch holding both +e and -e is rejected;
 *                      +e with e in E and -e with e not in E are skipped.
 *   I, D             : the remaining insertions and deletions.
 *   G'               : (V, (E u I) \ D, L).
 *   result(+)        : matches of Q in G' that are not matches in G
 *                      = matches in G' with at least one image edge in I.
 *   result(-)        : matches of Q in G that are not matches in G'
 *                      = matches in G with at least one image edge in D.
 *   A match is an injective, label-preserving map f: V(Q) -> V such that
 *   every query edge maps onto a data edge (non-induced; Def. 2).
 *
 * Edge labels (Sec. II-A: the labelling function also covers edges): every
 * data edge, query edge and update carries a label in [0, L), L = 1 for an
 * unlabelled graph.  A query edge (u, w) with label e maps onto a data edge
 * {f(u), f(w)} with label e.  The graph stays simple: a pair holds at most
 * one edge, with one label.  An update names its triple {u, v, e}; two
 * updates of one pair in a batch must be the same triple with the same op
 * (duplicates) or the batch is rejected as conflicting; inserting a pair
 * that is present under another label is rejected as invalid (relabelling
 * takes a deletion and a later insertion); deleting a triple whose pair
 * has another label is a no-op.  Internally a row holds keys w * L + e in
 * ascending order, so with L = 1 the key is the neighbour itself.
 *
 * How (Sec. IV-C, Algorithm 1 and the order rule that follows it):
 *   every update edge e_i of a pass carries ord i = its rank in ascending
 *   (lo, hi) order over the canonical batch.  For each seed e_i and each
 *   DIRECTED query edge (x, y) whose labels fit (both orientations are tried,
 *   since Algorithm 1's label test names one orientation only), the partial
 *   match {x -> lo, y -> hi} is extended one query vertex at a time along a
 *   BFS order from (x, y).  A candidate c for query vertex u is taken from the
 *   neighbours of f(w0), w0 being u's first already-matched query neighbour;
 *   it must carry u's label, be unused (injectivity, which the candidate
 *   procedure of Algorithm 1 leaves implicit) and be adjacent in the pass's
 *   graph to f(w) for every matched neighbour w, through an edge that is
 *   not a batch edge of this pass with ord < i.  That last condition is the
 *   paper's rule that matches form from lower-order update edges towards
 *   higher-order ones: each match is found exactly once, from its
 *   minimum-ord batch edge.
 *   The insertion pass searches G' seeded from I; the deletion pass searches
 *   G seeded from D (the paper leaves the deletion graph implicit; G is the
 *   graph whose matches a deletion destroys).
 *
 * Output per pass: the tuples (f(0), ..., f(k-1)) with their seed ord, and
 * count / sum / xor of a per-tuple checksum built from the SplitMix64
 * finaliser `mix` (a checksum of this project, not part of the paper):
 *   h = mix( mix(qid << 1 | sign) + sum_j (f(j) + 1) * K_j ),
 *   K_j = mix(G * (j + 1)) | 1, sums and products mod 2^64,
 *   G = 0x9E3779B97F4A7C15, sign = 1 for insertions and 0 for deletions.
 *   Position keys make it order-sensitive; the outer mix makes it
 *   non-linear in the tuple.
 *
 * A `mutant` argument plants a known mistake (tests use it to show that the
 * pins catch each one); 0 is the correct oracle.
 *
 * Seed cap (a sampling control for very large result sets, not part of the
 * method): with seed_cap > 0 a seed whose matches exceed seed_cap is given
 * up as soon as its (seed_cap + 1)-th match is found.  It is flagged in
 * seed_incomplete, its tuples are dropped, and it contributes nothing to
 * the per-pass totals; its seed_count holds seed_cap + 1, a lower bound of
 * its true count.  Every seed that is not flagged is exact.
 *
 * Scan cap (the same kind of control, for searches that are long without
 * finding matches): with scan_cap > 0 a seed is given up once its search
 * has examined scan_cap neighbour-list entries.  It is flagged 2 in
 * seed_incomplete (1 marks the seed cap) and treated like a seed given up
 * at the seed cap, except that its seed_count holds only the matches found
 * before it was given up: a lower bound of its true count.
 *
 * Ord list (a sampling control too): with ords != NULL only the canonical
 * updates whose ords are listed are searched; the canonical batch, G' and
 * the visibility of every batch edge are those of the whole batch, so each
 * searched seed's figures are exactly its figures in the full run.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum {
  MUT_NONE = 0,
  MUT_NO_INJECTIVITY = 1,   /* candidates may reuse a matched data vertex */
  MUT_ONE_ORIENTATION = 2,  /* only the listed orientation of each query edge */
  MUT_NO_ORDER_RULE = 3,    /* batch edges of any ord are usable */
  MUT_DELETE_ON_GPRIME = 4, /* deletion pass searches G' instead of G */
  MUT_SKIP_FIRST_CHECK = 5, /* w0's edge is not checked against the order rule */
  MUT_NO_LABEL_CHECK = 6,   /* extension ignores labels */
  MUT_KEEP_NOOPS = 7,       /* no-op updates are not skipped */
  MUT_NO_EDGE_LABEL_CHECK = 8 /* extension ignores edge labels */
};

typedef struct {
  int32_t status; /* 0 ok, -1 invalid update, -2 conflicting +e/-e */
  uint32_t n_canonical, n_insert, n_delete, n_noop, n_dup;
  uint64_t count[2], hsum[2], hxor[2]; /* index 1 = insertions, 0 = deletions */
  uint64_t n_tuples;
  uint32_t* tuples; /* n_tuples * k */
  uint8_t* tsign;   /* n_tuples */
  uint32_t* tord;   /* n_tuples */
  uint32_t* canon_lo;
  uint32_t* canon_hi;
  uint8_t* canon_sign; /* n_canonical */
  uint64_t* seed_count;
  uint64_t* seed_hsum;
  uint64_t* seed_hxor; /* n_canonical: per seed (update) totals */
  double seconds;
  int32_t threads_used;
  uint32_t* canon_e; /* n_canonical: edge label of each canonical update */
  uint8_t* seed_incomplete; /* n_canonical: 1 = given up at the seed cap, 2 = at the scan cap */
  uint64_t n_incomplete;
  double seconds_prep; /* keys, canonical batch and G' (the oracle's own graph update) */
} o2_result;

/* ---------------------------------------------------------------- hashing */

static uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

/* The project's tuple checksum (not part of the method): position j's
 * element term is (f_j + 1) * K_j, K_j = mix(G (j + 1)) | 1 (odd, so the
 * term is a bijection of f_j), and h = mix(mix(q << 1 | sign) + sum of the
 * terms), sums mod 2^64. */
static uint64_t tuple_hash(uint32_t qid, int sign, const uint32_t* f, uint32_t k) {
  uint64_t s = mix(((uint64_t)qid << 1) | (uint64_t)(sign ? 1 : 0));
  for (uint32_t j = 0; j < k; ++j) s += ((uint64_t)f[j] + 1u) * (mix(0x9E3779B97F4A7C15ull * (j + 1)) | 1u);
  return mix(s);
}

/* ---------------------------------------------------------------- helpers */

typedef struct {
  uint32_t n;
  const uint64_t* rp;
  const uint32_t* col; /* keys w * L + e, ascending per row */
} csr_t;

/* Does row u hold a key in [k0, k1)? */
static int row_has_range(const csr_t* g, uint32_t u, uint32_t k0, uint32_t k1) {
  uint64_t lo = g->rp[u], hi = g->rp[u + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] < k0)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < g->rp[u + 1] && g->col[lo] < k1;
}

static int row_has(const csr_t* g, uint32_t u, uint32_t v) {
  uint64_t lo = g->rp[u], hi = g->rp[u + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < g->rp[u + 1] && g->col[lo] == v;
}

typedef struct {
  uint32_t lo, hi, e;
  uint8_t op;
} upd_t;

static int upd_cmp(const void* a, const void* b) {
  const upd_t* x = (const upd_t*)a;
  const upd_t* y = (const upd_t*)b;
  if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
  if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
  if (x->e != y->e) return x->e < y->e ? -1 : 1;
  if (x->op != y->op) return x->op < y->op ? -1 : 1;
  return 0;
}

static int u32_cmp(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return x < y ? -1 : x > y;
}

/* The canonical batch, ordered by (lo, hi): entry i has ord i. */
typedef struct {
  uint32_t n;
  uint32_t* lo;
  uint32_t* hi;
  uint32_t* e;
  uint8_t* sign;
} canon_t;

/* Find the pair (lo, hi) among the canonical edges; returns its ord or -1
 * (a pair occurs at most once in a canonical batch). */
static int64_t canon_find(const canon_t* c, uint32_t a, uint32_t b) {
  uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  int64_t l = 0, r = (int64_t)c->n;
  while (l < r) {
    int64_t m = l + (r - l) / 2;
    if (c->lo[m] < lo || (c->lo[m] == lo && c->hi[m] < hi))
      l = m + 1;
    else
      r = m;
  }
  if (l < (int64_t)c->n && c->lo[l] == lo && c->hi[l] == hi) return l;
  return -1;
}

static int canonicalise(const csr_t* g, uint32_t L, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                        const uint8_t* op, const uint32_t* uel, int mutant, canon_t* out, o2_result* res) {
  upd_t* u = (upd_t*)malloc(sizeof(upd_t) * (n_upd ? n_upd : 1));
  for (uint32_t i = 0; i < n_upd; ++i) {
    const uint32_t e = uel ? uel[i] : 0;
    if (src[i] == dst[i] || src[i] >= g->n || dst[i] >= g->n || e >= L) {
      free(u);
      return -1;
    }
    u[i].lo = src[i] < dst[i] ? src[i] : dst[i];
    u[i].hi = src[i] < dst[i] ? dst[i] : src[i];
    u[i].e = e;
    u[i].op = op[i] ? 1 : 0;
  }
  qsort(u, n_upd, sizeof(upd_t), upd_cmp);
  out->lo = (uint32_t*)malloc(4 * (n_upd ? n_upd : 1));
  out->hi = (uint32_t*)malloc(4 * (n_upd ? n_upd : 1));
  out->e = (uint32_t*)malloc(4 * (n_upd ? n_upd : 1));
  out->sign = (uint8_t*)malloc(n_upd ? n_upd : 1);
  out->n = 0;
  for (uint32_t i = 0; i < n_upd; ++i) {
    if (i > 0 && u[i].lo == u[i - 1].lo && u[i].hi == u[i - 1].hi) {
      if (u[i].op != u[i - 1].op || u[i].e != u[i - 1].e) {
        free(u);
        return -2;
      }
      res->n_dup++;
      continue;
    }
    int present = row_has(g, u[i].lo, u[i].hi * L + u[i].e);
    if (u[i].op && !present && row_has_range(g, u[i].lo, u[i].hi * L, u[i].hi * L + L)) {
      free(u); /* the pair is present under another label */
      return -1;
    }
    int noop = u[i].op ? present : !present;
    if (noop && mutant != MUT_KEEP_NOOPS) {
      res->n_noop++;
      continue;
    }
    out->lo[out->n] = u[i].lo;
    out->hi[out->n] = u[i].hi;
    out->e[out->n] = u[i].e;
    out->sign[out->n] = u[i].op;
    out->n++;
  }
  free(u);
  return 0;
}

/* G' = (E u I) \ D as a fresh CSR with ascending rows. */
static void build_updated(const csr_t* g, uint32_t L, const canon_t* c, uint64_t** rp_out, uint32_t** col_out) {
  uint32_t n = g->n;
  int64_t* delta = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (uint32_t i = 0; i < c->n; ++i) {
    int d = c->sign[i] ? 1 : -1;
    delta[c->lo[i]] += d;
    delta[c->hi[i]] += d;
  }
  uint64_t* rp = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  rp[0] = 0;
  for (uint32_t v = 0; v < n; ++v)
    rp[v + 1] = rp[v] + (uint64_t)((int64_t)(g->rp[v + 1] - g->rp[v]) + delta[v]);
  uint32_t* col = (uint32_t*)malloc(4 * (rp[n] ? rp[n] : 1));
  /* per vertex: the batch neighbours to add and to remove */
  uint64_t* bstart = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
  for (uint32_t i = 0; i < c->n; ++i) {
    bstart[c->lo[i] + 1]++;
    bstart[c->hi[i] + 1]++;
  }
  for (uint32_t v = 0; v < n; ++v) bstart[v + 1] += bstart[v];
  uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  memcpy(fill, bstart, sizeof(uint64_t) * ((size_t)n + 1));
  uint32_t* bn = (uint32_t*)malloc(4 * (bstart[n] ? bstart[n] : 1));
  uint8_t* bs = (uint8_t*)malloc(bstart[n] ? bstart[n] : 1);
  for (uint32_t i = 0; i < c->n; ++i) {
    uint64_t p = fill[c->lo[i]]++;
    bn[p] = c->hi[i] * L + c->e[i];
    bs[p] = c->sign[i];
    p = fill[c->hi[i]]++;
    bn[p] = c->lo[i] * L + c->e[i];
    bs[p] = c->sign[i];
  }
  /* deleted entries (keys) of v, ascending, for a binary-search membership test */
  uint32_t* dn = (uint32_t*)malloc(4 * (bstart[n] ? bstart[n] : 1));
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t nd = 0;
    for (uint64_t t = bstart[v]; t < bstart[v + 1]; ++t)
      if (!bs[t]) dn[bstart[v] + nd++] = bn[t];
    qsort(dn + bstart[v], (size_t)nd, 4, u32_cmp);
    uint64_t w = rp[v];
    for (uint64_t j = g->rp[v]; j < g->rp[v + 1]; ++j) {
      uint32_t x = g->col[j];
      uint64_t l = bstart[v], r = bstart[v] + nd;
      while (l < r) {
        uint64_t mid = l + (r - l) / 2;
        if (dn[mid] < x)
          l = mid + 1;
        else
          r = mid;
      }
      int deleted = (l < bstart[v] + nd && dn[l] == x);
      if (!deleted) col[w++] = x;
    }
    for (uint64_t t = bstart[v]; t < bstart[v + 1]; ++t)
      if (bs[t]) col[w++] = bn[t];
    qsort(col + rp[v], (size_t)(w - rp[v]), 4, u32_cmp);
  }
  free(delta);
  free(bstart);
  free(fill);
  free(bn);
  free(bs);
  free(dn);
  *rp_out = rp;
  *col_out = col;
}

/* ---------------------------------------------------------------- search */

typedef struct {
  uint32_t k;
  const uint32_t* qlab;
  uint8_t adj[16][16];
  uint32_t qel[16][16]; /* edge label of query edge {a, b} */
  uint32_t n_dqe;
  uint32_t dx[256], dy[256];
  uint32_t order[256][16]; /* BFS matching order per directed query edge */
} query_t;

typedef struct {
  uint32_t* t;
  uint8_t* s;
  uint32_t* o;
  uint64_t n, cap;
} tbuf_t;

typedef struct {
  /* shared, read-only */
  const csr_t* H[2]; /* graph searched by pass: [1] = G', [0] = G */
  const canon_t* c;
  const uint32_t* labels;
  const query_t* q;
  uint32_t L; /* number of edge labels */
  uint32_t qid;
  int mutant, want_tuples;
  uint32_t sample_mod, sample_rem;
  const uint8_t* pick; /* per canonical ord: 1 = searched (NULL: every ord) */
  uint64_t seed_cap; /* 0: none */
  uint64_t scan_cap; /* 0: none */
  /* work distribution */
  uint32_t next; /* atomic counter over canonical updates */
  /* per seed totals */
  uint64_t *seed_count, *seed_hsum, *seed_hxor;
  uint8_t* seed_incomplete;
} shared_t;

typedef struct {
  shared_t* sh;
  tbuf_t out;
  uint64_t count[2], hsum[2], hxor[2];
  int give_up;      /* the current seed passed the seed cap (1) or the scan cap (2) */
  uint64_t scanned; /* neighbour-list entries the current seed's search has examined */
} worker_t;

static void emit(worker_t* w, int sign, uint32_t ord, const uint32_t* f) {
  const shared_t* sh = w->sh;
  uint32_t k = sh->q->k;
  uint64_t h = tuple_hash(sh->qid, sign, f, k);
  (void)sign;
  sh->seed_count[ord]++;
  sh->seed_hsum[ord] += h;
  sh->seed_hxor[ord] ^= h;
  if (sh->seed_cap && sh->seed_count[ord] > sh->seed_cap) {
    w->give_up = 1;
    return;
  }
  if (!sh->want_tuples) return;
  if (w->out.n == w->out.cap) {
    w->out.cap = w->out.cap ? w->out.cap * 2 : 1024;
    w->out.t = (uint32_t*)realloc(w->out.t, 4 * w->out.cap * k);
    w->out.s = (uint8_t*)realloc(w->out.s, w->out.cap);
    w->out.o = (uint32_t*)realloc(w->out.o, 4 * w->out.cap);
  }
  memcpy(w->out.t + w->out.n * k, f, 4 * k);
  w->out.s[w->out.n] = (uint8_t)sign;
  w->out.o[w->out.n] = ord;
  w->out.n++;
}

/* Is data edge {a, b, el} usable by seed `ord` of pass `sign` on graph H?
 * (Only the batch edge of that pair with that label is subject to the
 * order rule; an edge of another label between a and b is not in the batch.) */
static int edge_ok(const shared_t* sh, const csr_t* H, int sign, uint32_t ord, uint32_t a,
                   uint32_t b, uint32_t el) {
  if (!row_has(H, a, b * sh->L + el)) return 0;
  if (sh->mutant == MUT_NO_ORDER_RULE) return 1;
  int64_t e = canon_find(sh->c, a, b);
  if (e >= 0 && sh->c->e[e] == el && sh->c->sign[e] == (uint8_t)sign && (uint32_t)e < ord) return 0;
  return 1;
}

static void extend(worker_t* w, int sign, uint32_t ord, const uint32_t* pi, uint32_t l,
                   uint32_t* f) {
  const shared_t* sh = w->sh;
  const query_t* q = sh->q;
  const csr_t* H = sh->H[sign];
  if (l == q->k) {
    emit(w, sign, ord, f);
    return;
  }
  uint32_t u = pi[l];
  uint32_t back[16], nb = 0;
  for (uint32_t j = 0; j < l; ++j)
    if (q->adj[u][pi[j]]) back[nb++] = pi[j];
  /* nb >= 1: the BFS order keeps every prefix connected */
  uint32_t a0 = f[back[0]];
  const int any_el = sh->mutant == MUT_NO_EDGE_LABEL_CHECK;
  for (uint64_t t = H->rp[a0]; t < H->rp[a0 + 1] && !w->give_up; ++t) {
    if (sh->scan_cap && ++w->scanned > sh->scan_cap) {
      w->give_up = 2;
      return;
    }
    uint32_t c = H->col[t] / sh->L, ce = H->col[t] % sh->L;
    if (!any_el && ce != q->qel[u][back[0]]) continue;
    if (sh->mutant != MUT_NO_LABEL_CHECK && sh->labels[c] != q->qlab[u]) continue;
    if (sh->mutant != MUT_NO_INJECTIVITY) {
      int used = 0;
      for (uint32_t j = 0; j < l; ++j)
        if (f[pi[j]] == c) used = 1;
      if (used) continue;
    }
    int ok = 1;
    for (uint32_t b = 0; b < nb && ok; ++b) {
      if (b == 0 && sh->mutant == MUT_SKIP_FIRST_CHECK) continue;
      ok = edge_ok(sh, H, sign, ord, f[back[b]], c, b == 0 && any_el ? ce : q->qel[u][back[b]]);
      for (uint32_t e2 = 0; any_el && b > 0 && !ok && e2 < sh->L; ++e2)
        ok = edge_ok(sh, H, sign, ord, f[back[b]], c, e2);
    }
    if (!ok) continue;
    f[u] = c;
    extend(w, sign, ord, pi, l + 1, f);
  }
}

static void* worker_main(void* arg) {
  worker_t* w = (worker_t*)arg;
  shared_t* sh = w->sh;
  const query_t* q = sh->q;
  uint32_t f[16];
  for (;;) {
    uint32_t i = __atomic_fetch_add(&sh->next, 1, __ATOMIC_RELAXED);
    if (i >= sh->c->n) break;
    if (sh->sample_mod > 1 && i % sh->sample_mod != sh->sample_rem) continue;
    if (sh->pick && !sh->pick[i]) continue;
    int sign = sh->c->sign[i];
    uint32_t lo = sh->c->lo[i], hi = sh->c->hi[i], el = sh->c->e[i];
    const uint64_t n_out0 = w->out.n;
    w->give_up = 0;
    w->scanned = 0;
    for (uint32_t d = 0; d < q->n_dqe && !w->give_up; ++d) {
      uint32_t x = q->dx[d], y = q->dy[d];
      if (sh->labels[lo] != q->qlab[x] || sh->labels[hi] != q->qlab[y]) continue;
      if (sh->mutant != MUT_NO_EDGE_LABEL_CHECK && q->qel[x][y] != el) continue;
      f[x] = lo;
      f[y] = hi;
      extend(w, sign, i, q->order[d], 2, f);
    }
    if (w->give_up) {
      /* given up at the seed or scan cap: drop what it found */
      sh->seed_incomplete[i] = (uint8_t)w->give_up;
      w->out.n = n_out0;
      continue;
    }
    w->count[sign] += sh->seed_count[i];
    w->hsum[sign] += sh->seed_hsum[i];
    w->hxor[sign] ^= sh->seed_hxor[i];
  }
  return NULL;
}

/* BFS order from the directed edge (x, y), neighbours in ascending id. */
static int bfs_order(const query_t* q, uint32_t x, uint32_t y, uint32_t* pi) {
  uint8_t seen[16] = {0};
  uint32_t len = 0, head = 0;
  pi[len++] = x;
  pi[len++] = y;
  seen[x] = seen[y] = 1;
  while (head < len) {
    uint32_t v = pi[head++];
    for (uint32_t u = 0; u < q->k; ++u)
      if (q->adj[v][u] && !seen[u]) {
        seen[u] = 1;
        pi[len++] = u;
      }
  }
  return len == q->k ? 0 : -1;
}

/* ---------------------------------------------------------------- API */

/* Row keys w * L + e of a CSR with per-entry edge labels (NULL: all 0),
 * each row sorted; NULL if a label is >= L, n * L does not fit 32 bits or
 * a row names one neighbour twice. */
static uint32_t* make_keys(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* elab,
                           uint32_t L) {
  if ((uint64_t)n * L > 0xFFFFFFFFull) return NULL;
  const uint64_t nnz = row_ptr[n];
  uint32_t* key = (uint32_t*)malloc(4 * (nnz ? nnz : 1));
  for (uint64_t j = 0; j < nnz; ++j) {
    const uint32_t e = elab ? elab[j] : 0;
    if (e >= L) {
      free(key);
      return NULL;
    }
    key[j] = col[j] * L + e;
  }
  for (uint32_t v = 0; v < n; ++v) {
    qsort(key + row_ptr[v], (size_t)(row_ptr[v + 1] - row_ptr[v]), 4, u32_cmp);
    for (uint64_t j = row_ptr[v] + 1; j < row_ptr[v + 1]; ++j)
      if (key[j] / L == key[j - 1] / L) { /* two edges on one pair: not a simple graph */
        free(key);
        return NULL;
      }
  }
  return key;
}

int o2_run_el(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* labels,
              uint32_t L, const uint32_t* elab, uint32_t qid, uint32_t k, const uint32_t* qlabels, uint32_t m,
              const uint32_t* qedges, const uint32_t* qelab, uint32_t n_upd, const uint32_t* src,
              const uint32_t* dst, const uint8_t* op, const uint32_t* uelab, int threads, uint32_t sample_mod,
              uint32_t sample_rem, uint64_t seed_cap, uint64_t scan_cap, const uint32_t* ords, uint32_t n_ords,
              int want_tuples, int mutant, o2_result* res) {
  struct timespec t0, t1, tp;
  clock_gettime(CLOCK_MONOTONIC, &t0);
  memset(res, 0, sizeof(*res));
  if (k < 2 || k > 16 || m == 0 || m > 120 || L == 0) return -3;
  query_t* q = (query_t*)calloc(1, sizeof(query_t));
  q->k = k;
  q->qlab = qlabels;
  for (uint32_t e = 0; e < m; ++e) {
    uint32_t a = qedges[2 * e], b = qedges[2 * e + 1];
    const uint32_t el = qelab ? qelab[e] : 0;
    if (a >= k || b >= k || a == b || el >= L) {
      free(q);
      return -3;
    }
    q->adj[a][b] = q->adj[b][a] = 1;
    q->qel[a][b] = q->qel[b][a] = el;
    q->dx[q->n_dqe] = a;
    q->dy[q->n_dqe] = b;
    q->n_dqe++;
    if (mutant != MUT_ONE_ORIENTATION) {
      q->dx[q->n_dqe] = b;
      q->dy[q->n_dqe] = a;
      q->n_dqe++;
    }
  }
  for (uint32_t d = 0; d < q->n_dqe; ++d)
    if (bfs_order(q, q->dx[d], q->dy[d], q->order[d]) != 0) {
      free(q);
      return -3; /* disconnected query */
    }

  uint32_t* key = make_keys(n, row_ptr, col, elab, L);
  if (!key) {
    free(q);
    return -3;
  }
  csr_t G = {n, row_ptr, key};
  canon_t c;
  memset(&c, 0, sizeof(c));
  int st = canonicalise(&G, L, n_upd, src, dst, op, uelab, mutant, &c, res);
  res->status = st;
  if (st != 0) {
    free(q);
    free(key);
    return st;
  }
  res->n_canonical = c.n;
  for (uint32_t i = 0; i < c.n; ++i) {
    if (c.sign[i])
      res->n_insert++;
    else
      res->n_delete++;
  }
  uint64_t* rp2;
  uint32_t* col2;
  build_updated(&G, L, &c, &rp2, &col2);
  csr_t G2 = {n, rp2, col2};
  clock_gettime(CLOCK_MONOTONIC, &tp);
  res->seconds_prep = (double)(tp.tv_sec - t0.tv_sec) + 1e-9 * (double)(tp.tv_nsec - t0.tv_nsec);

  shared_t sh;
  memset(&sh, 0, sizeof(sh));
  sh.H[1] = &G2;
  sh.H[0] = (mutant == MUT_DELETE_ON_GPRIME) ? &G2 : &G;
  sh.c = &c;
  sh.labels = labels;
  sh.q = q;
  sh.L = L;
  sh.qid = qid;
  sh.mutant = mutant;
  sh.want_tuples = want_tuples;
  sh.sample_mod = sample_mod;
  sh.sample_rem = sample_rem;
  uint8_t* pick = NULL;
  if (ords) {
    pick = (uint8_t*)calloc(c.n ? c.n : 1, 1);
    for (uint32_t j = 0; j < n_ords; ++j)
      if (ords[j] < c.n) pick[ords[j]] = 1;
  }
  sh.pick = pick;
  sh.seed_cap = seed_cap;
  sh.scan_cap = scan_cap;
  uint32_t nc = c.n ? c.n : 1;
  sh.seed_count = (uint64_t*)calloc(nc, 8);
  sh.seed_hsum = (uint64_t*)calloc(nc, 8);
  sh.seed_hxor = (uint64_t*)calloc(nc, 8);
  sh.seed_incomplete = (uint8_t*)calloc(nc, 1);

  if (threads < 1) threads = 1;
  worker_t* ws = (worker_t*)calloc((size_t)threads, sizeof(worker_t));
  pthread_t* th = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
  for (int t = 0; t < threads; ++t) {
    ws[t].sh = &sh;
    if (threads > 1)
      pthread_create(&th[t], NULL, worker_main, &ws[t]);
  }
  if (threads == 1) worker_main(&ws[0]);
  for (int t = 0; t < threads && threads > 1; ++t) pthread_join(th[t], NULL);

  uint64_t total = 0;
  for (int t = 0; t < threads; ++t) {
    for (int s = 0; s < 2; ++s) {
      res->count[s] += ws[t].count[s];
      res->hsum[s] += ws[t].hsum[s];
      res->hxor[s] ^= ws[t].hxor[s];
    }
    total += ws[t].out.n;
  }
  if (want_tuples) {
    res->tuples = (uint32_t*)malloc(4 * (total ? total : 1) * k);
    res->tsign = (uint8_t*)malloc(total ? total : 1);
    res->tord = (uint32_t*)malloc(4 * (total ? total : 1));
    uint64_t p = 0;
    for (int t = 0; t < threads; ++t) {
      if (ws[t].out.n) {
        memcpy(res->tuples + p * k, ws[t].out.t, 4 * ws[t].out.n * k);
        memcpy(res->tsign + p, ws[t].out.s, ws[t].out.n);
        memcpy(res->tord + p, ws[t].out.o, 4 * ws[t].out.n);
      }
      p += ws[t].out.n;
      free(ws[t].out.t);
      free(ws[t].out.s);
      free(ws[t].out.o);
    }
    res->n_tuples = total;
  }
  res->canon_lo = c.lo;
  res->canon_hi = c.hi;
  res->canon_sign = c.sign;
  res->canon_e = c.e;
  res->seed_count = sh.seed_count;
  res->seed_hsum = sh.seed_hsum;
  res->seed_hxor = sh.seed_hxor;
  res->seed_incomplete = sh.seed_incomplete;
  for (uint32_t i = 0; i < c.n; ++i) res->n_incomplete += sh.seed_incomplete[i];
  res->threads_used = threads;
  free(ws);
  free(th);
  free(pick);
  free(rp2);
  free(col2);
  free(key);
  free(q);
  clock_gettime(CLOCK_MONOTONIC, &t1);
  res->seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
  return 0;
}

/* The unlabelled case: one edge label. */
int o2_run(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* labels,
           uint32_t qid, uint32_t k, const uint32_t* qlabels, uint32_t m, const uint32_t* qedges,
           uint32_t n_upd, const uint32_t* src, const uint32_t* dst, const uint8_t* op,
           int threads, uint32_t sample_mod, uint32_t sample_rem, int want_tuples, int mutant,
           o2_result* res) {
  return o2_run_el(n, row_ptr, col, labels, 1, NULL, qid, k, qlabels, m, qedges, NULL, n_upd, src, dst, op, NULL,
                   threads, sample_mod, sample_rem, 0, 0, NULL, 0, want_tuples, mutant, res);
}

/* G' as a CSR for callers that chain batches (row_ptr n+1; col and, when
 * elab_out is not NULL, the edge labels, row_ptr[n] entries, each row
 * ascending by (neighbour, label)). */
int o2_updated_graph_el(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* elab,
                        uint32_t L, uint32_t n_upd, const uint32_t* src, const uint32_t* dst, const uint8_t* op,
                        const uint32_t* uelab, uint64_t** rp_out, uint32_t** col_out, uint32_t** elab_out) {
  if (L == 0) return -3;
  uint32_t* key = make_keys(n, row_ptr, col, elab, L);
  if (!key) return -3;
  csr_t G = {n, row_ptr, key};
  canon_t c;
  memset(&c, 0, sizeof(c));
  o2_result tmp;
  memset(&tmp, 0, sizeof(tmp));
  int st = canonicalise(&G, L, n_upd, src, dst, op, uelab, 0, &c, &tmp);
  if (st != 0) {
    free(key);
    return st;
  }
  build_updated(&G, L, &c, rp_out, col_out);
  const uint64_t nnz = (*rp_out)[n];
  uint32_t* el = (uint32_t*)malloc(4 * (nnz ? nnz : 1));
  for (uint64_t j = 0; j < nnz; ++j) {
    el[j] = (*col_out)[j] % L;
    (*col_out)[j] /= L;
  }
  if (elab_out)
    *elab_out = el;
  else
    free(el);
  free(key);
  free(c.lo);
  free(c.hi);
  free(c.e);
  free(c.sign);
  return 0;
}

int o2_updated_graph(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, uint32_t n_upd,
                     const uint32_t* src, const uint32_t* dst, const uint8_t* op,
                     uint64_t** rp_out, uint32_t** col_out) {
  return o2_updated_graph_el(n, row_ptr, col, NULL, 1, n_upd, src, dst, op, NULL, rp_out, col_out, NULL);
}

void o2_free_ptr(void* p) { free(p); }

void o2_free(o2_result* r) {
  free(r->tuples);
  free(r->tsign);
  free(r->tord);
  free(r->canon_lo);
  free(r->canon_hi);
  free(r->canon_sign);
  free(r->canon_e);
  free(r->seed_count);
  free(r->seed_hsum);
  free(r->seed_hxor);
  free(r->seed_incomplete);
  memset(r, 0, sizeof(*r));
}

uint64_t o2_tuple_hash(uint32_t qid, int sign, const uint32_t* f, uint32_t k) {
  return tuple_hash(qid, sign, f, k);
}
