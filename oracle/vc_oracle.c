/*
 * vc_oracle.c -- plain sequential CPU oracle for the vertex-cover search.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or loads this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header or table with the HIP path.
 *
 * Contents:
 *  - vco_tau_by_definition: the minimum vertex cover size by its definition (paper §II-A):
 *    the smallest |S| over all subsets S that touch every edge. Exhaustive, n <= 24.
 *  - vco_greedy: the greedy approximation that seeds `best` (paper §II-B): apply the
 *    reduction rules, take a maximum-degree vertex, repeat until no edge is left.
 *  - vco_reduce: the reduction rules (degree-one, degree-two-triangle, high-degree; §II-B)
 *    applied repeatedly until nothing changes, with the tie-breaks of the parallel rules
 *    (§IV-D) and the pass semantics described below.
 *  - vco_mvc / vco_pvc: the serial branch-and-reduce search (§II-B, Fig. 1 and the PVC
 *    differences stated in the text), depth first, child "v_max in S" before child
 *    "N(v_max) in S" (the order the hybrid method continues in, §IV-A).
 *
 * State: a degree array with one int32 per original vertex holding the vertex's current
 * degree, or SENT (-1) once the vertex has been put in the cover (§IV-B), plus the cover
 * size s kept beside it.
 *
 * Pass semantics (a reading; the paper does not spell it out): each rule is one pass that
 * first decides, for every vertex, from the degree array as it stood at the start of the
 * pass, then applies all decisions together. The three passes run in the order
 * degree-one, degree-two-triangle, high-degree, and the sequence is repeated until a whole
 * sequence changes nothing, or until s exceeds the bound (then the node is pruned).
 *   - degree-one: v live with deg 1, u its one live neighbour: u goes in the cover unless u
 *     also has degree 1 and v < u (of a pair of adjacent degree-one vertices only the
 *     smaller id is removed; a shared neighbour is removed once).
 *   - degree-two-triangle: v live with deg 2, live neighbours u, w adjacent to each other:
 *     u and w go in the cover unless u or w itself has degree 2 and a smaller id than v
 *     (in a triangle of several degree-two vertices only the smallest fires).
 *   - high-degree: r = bound - s at the start of the pass; every live v with deg > r goes in
 *     the cover. bound = best - 1 for MVC (so r = best - |S| - 1) and k for PVC (r = k - |S|).
 * Stopping condition (§II-B): with r = bound - s, prune if r < 0 or |E| > r^2.
 */

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SENT (-1)

enum {
  VCO_RULE_DEG1 = 1,
  VCO_RULE_TRI = 2,
  VCO_RULE_HIGH = 4,
  VCO_PRUNE_EDGES = 8,
  VCO_ALL = 15
};

enum { VCO_OK = 0, VCO_BUDGET = 1, VCO_BADARG = 2, VCO_NOMEM = 3 };

typedef struct {
  int32_t n;
  const int32_t *rp;
  const int32_t *ci;
} graph_t;

/* ------------------------------------------------------------------------------------ */
/* Minimum cover size by definition: try every subset.                                   */

int32_t vco_tau_by_definition(int32_t n, const int32_t *rp, const int32_t *ci,
                              uint8_t *cover_out) {
  if (n < 0 || n > 24) return -1;
  int32_t m = rp[n] / 2;
  int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  int32_t e = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j)
      if (u < ci[j]) { eu[e] = u; ev[e] = ci[j]; ++e; }
  int32_t best = n + 1;
  uint32_t best_set = 0;
  uint32_t total = (uint32_t)1 << n;
  for (uint32_t set = 0; set < total; ++set) {
    int32_t size = __builtin_popcount(set);
    if (size >= best) continue;
    int covers = 1;
    for (int32_t i = 0; i < e; ++i) {
      if (!(((set >> eu[i]) | (set >> ev[i])) & 1u)) { covers = 0; break; }
    }
    if (covers) { best = size; best_set = set; }
  }
  free(eu);
  free(ev);
  if (cover_out)
    for (int32_t v = 0; v < n; ++v) cover_out[v] = (uint8_t)((best_set >> v) & 1u);
  return best;
}

/* ------------------------------------------------------------------------------------ */
/* Degree-array helpers.                                                                 */

static int64_t edge_count(int32_t n, const int32_t *deg) {
  int64_t sum = 0;
  for (int32_t v = 0; v < n; ++v)
    if (deg[v] >= 0) sum += deg[v];
  return sum / 2;
}

/* Vertex of maximum degree, smallest id among ties; -1 if no live vertex. */
static int32_t max_degree_vertex(int32_t n, const int32_t *deg) {
  int32_t best = -1;
  for (int32_t v = 0; v < n; ++v)
    if (deg[v] >= 0 && (best < 0 || deg[v] > deg[best])) best = v;
  return best;
}

/* Remove every flagged vertex: it joins the cover (deg = SENT) and each of its live
 * neighbours loses one degree per removed neighbour. Clears the flags. Returns the count. */
static int32_t remove_flagged(const graph_t *g, int32_t *deg, uint8_t *flag) {
  int32_t count = 0;
  for (int32_t v = 0; v < g->n; ++v)
    if (flag[v]) { deg[v] = SENT; ++count; }
  for (int32_t v = 0; v < g->n; ++v) {
    if (!flag[v]) continue;
    for (int32_t j = g->rp[v]; j < g->rp[v + 1]; ++j) {
      int32_t x = g->ci[j];
      if (deg[x] >= 0) deg[x] -= 1;
    }
    flag[v] = 0;
  }
  return count;
}

static int adjacent(const graph_t *g, int32_t u, int32_t w) {
  int32_t lo = g->rp[u], hi = g->rp[u + 1];
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if (g->ci[mid] == w) return 1;
    if (g->ci[mid] < w) lo = mid + 1; else hi = mid;
  }
  return 0;
}

/* Degree-one rule (§II-B; parallel tie-breaks §IV-D). */
static int32_t pass_degree_one(const graph_t *g, int32_t *deg, uint8_t *flag) {
  int32_t any = 0;
  for (int32_t v = 0; v < g->n; ++v) {
    if (deg[v] != 1) continue;
    int32_t u = -1;
    for (int32_t j = g->rp[v]; j < g->rp[v + 1]; ++j)
      if (deg[g->ci[j]] >= 0) { u = g->ci[j]; break; }
    if (u < 0) continue; /* cannot happen for a consistent degree array */
    if (deg[u] != 1 || u < v) { flag[u] = 1; any = 1; }
  }
  return any ? remove_flagged(g, deg, flag) : 0;
}

/* Degree-two-triangle rule (§II-B; tie-break §IV-D). */
static int32_t pass_degree_two_triangle(const graph_t *g, int32_t *deg, uint8_t *flag) {
  int32_t any = 0;
  for (int32_t v = 0; v < g->n; ++v) {
    if (deg[v] != 2) continue;
    int32_t nb[2], c = 0;
    for (int32_t j = g->rp[v]; j < g->rp[v + 1] && c < 2; ++j)
      if (deg[g->ci[j]] >= 0) nb[c++] = g->ci[j];
    if (c < 2) continue;
    int32_t u = nb[0], w = nb[1];
    if (!adjacent(g, u, w)) continue;
    if ((deg[u] == 2 && u < v) || (deg[w] == 2 && w < v)) continue;
    flag[u] = 1;
    flag[w] = 1;
    any = 1;
  }
  return any ? remove_flagged(g, deg, flag) : 0;
}

/* High-degree rule (§II-B): deg(v) > bound - s puts v in the cover. */
static int32_t pass_high_degree(const graph_t *g, int32_t *deg, uint8_t *flag, int64_t r) {
  int32_t any = 0;
  for (int32_t v = 0; v < g->n; ++v)
    if (deg[v] >= 0 && (int64_t)deg[v] > r) { flag[v] = 1; any = 1; }
  return any ? remove_flagged(g, deg, flag) : 0;
}

/* Apply the enabled rules until the graph stops changing (§II-B) or s exceeds bound. */
static void reduce(const graph_t *g, int32_t *deg, int32_t *s, int64_t bound, int rules,
                   uint8_t *flag) {
  int changed = 1;
  while (changed) {
    changed = 0;
    if (*s > bound) return;
    if (rules & VCO_RULE_DEG1) {
      int32_t k = pass_degree_one(g, deg, flag);
      *s += k;
      changed |= k > 0;
      if (*s > bound) return;
    }
    if (rules & VCO_RULE_TRI) {
      int32_t k = pass_degree_two_triangle(g, deg, flag);
      *s += k;
      changed |= k > 0;
      if (*s > bound) return;
    }
    if (rules & VCO_RULE_HIGH) {
      int32_t k = pass_high_degree(g, deg, flag, bound - *s);
      *s += k;
      changed |= k > 0;
    }
  }
}

void vco_reduce(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *deg, int32_t *s,
                int64_t bound, int32_t rules) {
  graph_t g = {n, rp, ci};
  uint8_t *flag = (uint8_t *)calloc((size_t)n + 1, 1);
  reduce(&g, deg, s, bound, rules, flag);
  free(flag);
}

/* ------------------------------------------------------------------------------------ */
/* Greedy approximation (§II-B): rules, then take a max-degree vertex, until edgeless.   */
/* The high-degree rule needs a bound and is not used here.                              */

int32_t vco_greedy(int32_t n, const int32_t *rp, const int32_t *ci, uint8_t *cover_out) {
  graph_t g = {n, rp, ci};
  int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  uint8_t *flag = (uint8_t *)calloc((size_t)n + 1, 1);
  int32_t s = 0;
  for (int32_t v = 0; v < n; ++v) deg[v] = rp[v + 1] - rp[v];
  for (;;) {
    reduce(&g, deg, &s, INT64_MAX, VCO_RULE_DEG1 | VCO_RULE_TRI, flag);
    if (edge_count(n, deg) == 0) break;
    int32_t v = max_degree_vertex(n, deg);
    flag[v] = 1;
    s += remove_flagged(&g, deg, flag);
  }
  if (cover_out)
    for (int32_t v = 0; v < n; ++v) cover_out[v] = (uint8_t)(deg[v] == SENT);
  free(deg);
  free(flag);
  return s;
}

/* ------------------------------------------------------------------------------------ */
/* Branch-and-reduce search (§II-B, Fig. 1; PVC differences stated in §II-B).            */

typedef struct {
  graph_t g;
  int pvc;          /* 0: MVC, 1: PVC */
  int64_t k;        /* PVC parameter */
  int32_t best;     /* MVC: size of the best cover found so far */
  int rules;
  int64_t nodes;
  int64_t node_cap; /* <= 0: no cap */
  int aborted;
  int found;        /* PVC: a cover of size <= k was found */
  int32_t *arena;   /* one degree array per depth */
  int32_t depth_cap;
  uint8_t *flag;
  uint8_t *cover;   /* best (MVC) or found (PVC) cover */
} search_t;

static int64_t current_bound(const search_t *t) {
  return t->pvc ? t->k : (int64_t)t->best - 1;
}

/* Visit one search-tree node whose degree array is arena[depth]. */
static void visit(search_t *t, int32_t depth, int32_t s) {
  if (t->aborted || t->found) return;
  if (t->node_cap > 0 && t->nodes >= t->node_cap) { t->aborted = 1; return; }
  t->nodes += 1;
  const int32_t n = t->g.n;
  int32_t *deg = t->arena + (size_t)depth * (size_t)(n + 1);

  int64_t bound = current_bound(t);
  reduce(&t->g, deg, &s, bound, t->rules, t->flag);

  /* stopping condition */
  int64_t r = bound - s;
  if (r < 0) return;
  int64_t e = edge_count(n, deg);
  if ((t->rules & VCO_PRUNE_EDGES) && (t->rules & VCO_RULE_HIGH) && e > r * r) return;

  if (e == 0) { /* a vertex cover */
    for (int32_t v = 0; v < n; ++v) t->cover[v] = (uint8_t)(deg[v] == SENT);
    if (t->pvc) t->found = 1;
    else t->best = s;
    return;
  }

  if (depth + 1 >= t->depth_cap) { t->aborted = 2; return; }
  int32_t vmax = max_degree_vertex(n, deg);
  int32_t *child = deg + (n + 1);

  /* child 1: v_max joins the cover */
  memcpy(child, deg, sizeof(int32_t) * (size_t)n);
  t->flag[vmax] = 1;
  int32_t added = remove_flagged(&t->g, child, t->flag);
  visit(t, depth + 1, s + added);
  if (t->aborted || t->found) return;

  /* child 2: every live neighbour of v_max joins the cover */
  memcpy(child, deg, sizeof(int32_t) * (size_t)n);
  for (int32_t j = t->g.rp[vmax]; j < t->g.rp[vmax + 1]; ++j)
    if (deg[t->g.ci[j]] >= 0) t->flag[t->g.ci[j]] = 1;
  added = remove_flagged(&t->g, child, t->flag);
  visit(t, depth + 1, s + added);
}

/* Common driver. Returns VCO_* status. */
static int search(int32_t n, const int32_t *rp, const int32_t *ci, int pvc, int64_t k,
                  int32_t rules, int64_t node_cap, int32_t *size_out, int32_t *yes_out,
                  uint8_t *cover_out, int64_t *nodes_out, int32_t *greedy_out) {
  if (n < 0 || (pvc && k < 0)) return VCO_BADARG;
  search_t t;
  memset(&t, 0, sizeof t);
  t.g.n = n; t.g.rp = rp; t.g.ci = ci;
  t.pvc = pvc;
  t.k = k;
  t.rules = rules;
  t.node_cap = node_cap;
  t.cover = (uint8_t *)calloc((size_t)n + 1, 1);
  t.flag = (uint8_t *)calloc((size_t)n + 1, 1);
  if (!t.cover || !t.flag) { free(t.cover); free(t.flag); return VCO_NOMEM; }

  int64_t m = n ? rp[n] / 2 : 0;
  int32_t greedy = 0;
  if (!pvc) {
    greedy = vco_greedy(n, rp, ci, t.cover);
    t.best = greedy;
  }
  if (greedy_out) *greedy_out = greedy;

  int rc = VCO_OK;
  if (m > 0) {
    /* Every branching on a path raises s by at least one and needs r >= 1, so a path has
     * at most `bound` branchings: bound + 2 degree arrays suffice. */
    int64_t bound = pvc ? (k < n ? k : n) : (int64_t)t.best - 1;
    if (bound < 0) bound = 0;
    t.depth_cap = (int32_t)bound + 2;
    t.arena = (int32_t *)malloc(sizeof(int32_t) * (size_t)t.depth_cap * ((size_t)n + 1));
    if (!t.arena) { free(t.cover); free(t.flag); return VCO_NOMEM; }
    for (int32_t v = 0; v < n; ++v) t.arena[v] = rp[v + 1] - rp[v];
    visit(&t, 0, 0);
    if (t.aborted == 1) rc = VCO_BUDGET;
    else if (t.aborted == 2) rc = VCO_NOMEM; /* depth bound violated: cannot happen */
  } else if (pvc) {
    t.found = 1; /* the empty set covers an edgeless graph */
  }

  if (rc == VCO_OK) {
    if (pvc) {
      *yes_out = t.found;
      *size_out = -1;
      if (t.found) {
        int32_t c = 0;
        for (int32_t v = 0; v < n; ++v) c += t.cover[v];
        *size_out = c;
      }
      if (cover_out) {
        if (t.found) memcpy(cover_out, t.cover, (size_t)n);
        else memset(cover_out, 0, (size_t)n);
      }
    } else {
      *size_out = t.best;
      if (cover_out) memcpy(cover_out, t.cover, (size_t)n);
    }
  }
  if (nodes_out) *nodes_out = t.nodes;
  free(t.arena);
  free(t.cover);
  free(t.flag);
  return rc;
}

int vco_mvc(int32_t n, const int32_t *rp, const int32_t *ci, int32_t rules, int64_t node_cap,
            int32_t *size_out, uint8_t *cover_out, int64_t *nodes_out, int32_t *greedy_out) {
  return search(n, rp, ci, 0, 0, rules, node_cap, size_out, NULL, cover_out, nodes_out,
                greedy_out);
}

int vco_pvc(int32_t n, const int32_t *rp, const int32_t *ci, int64_t k, int32_t rules,
            int64_t node_cap, int32_t *yes_out, int32_t *size_out, uint8_t *cover_out,
            int64_t *nodes_out) {
  int32_t yes = 0;
  int rc = search(n, rp, ci, 1, k, rules, node_cap, size_out, &yes, cover_out, nodes_out,
                  NULL);
  if (rc == VCO_OK) *yes_out = yes;
  return rc;
}
