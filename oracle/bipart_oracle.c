/*
 * Sequential oracle of BiPart (Maleki, Agarwal, Burtscher, Pingali, PPoPP'21).
 *
 * TEST INFRASTRUCTURE ONLY: this file defines the exact output the HIP
 * library must reproduce.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It is deliberately plain: one thread,
 * straightforward loops, qsort where the paper sorts, no blocking or fusion.
 *
 * Readings of the paper that the text leaves open are fixed as follows and
 * are the same contract the HIP path implements:
 *   - hash(id) is the MurmurHash3 32-bit finalizer of (id + 1), a bijection,
 *     taken on the hyperedge's index within the (sub)graph being coarsened;
 *   - a node's matched hyperedge is the lexicographic minimum of
 *     (priority, hash) over its incident hyperedges (Algorithm 1);
 *   - a singleton joins the step-one group, among those of its hyperedge's
 *     other pins, of least group weight, ties to the smaller node id
 *     (Algorithm 2, second loop);
 *   - coarse node ids follow the smallest fine id of each group; coarse
 *     hyperedges are the sorted distinct parents, kept when at least two, and
 *     identical ones are merged into the one of least source id with summed
 *     weight;
 *   - gains add/subtract the hyperedge weight (Algorithm 4 for weighted cut);
 *   - "sqrt(n)" is the integer ceiling of the square root; ties between equal
 *     gains go to the smaller node id; the refinement filter keeps gain >= 0;
 *   - the balance step moves, from the over-weight side, the shortest prefix
 *     (at most ceil(sqrt(n)) nodes, in gain order) that brings it under its
 *     bound, cut back so the other side never exceeds its own bound;
 *   - recursive bisection splits k into ceil(k/2) : floor(k/2), gives every
 *     bisection the imbalance (1+eps)^(1/ceil(log2 k)) - 1 and builds each
 *     child by cut-net splitting (Algorithm 6);
 *   - coarsening stops after max_levels steps, when no hyperedge is left, or
 *     when at most min_coarse_nodes nodes remain (Section 3.4).
 */
#include "bipart_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NONE64 0xFFFFFFFFFFFFFFFFull

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

static void *xcalloc(size_t count, size_t size)
{
    void *p = calloc(count ? count : 1, size ? size : 1);
    if (!p) abort();
    return p;
}

static int32_t node_weight(const int32_t *nw, int32_t v) { return nw ? nw[v] : 1; }
static int32_t hedge_weight(const int32_t *hw, int32_t h) { return hw ? hw[h] : 1; }

uint32_t oracle_hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

/* Smallest m with m*m >= n ("sqrt(n) nodes", Algorithm 3), by counting up. */
static int64_t ceil_sqrt(int64_t n)
{
    int64_t m = 0;
    while (m * m < n) m++;
    return m;
}

/* ---- problem statement (Section 1.1): connectivity minus one -------------- */

int64_t oracle_cut(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                   const int32_t *nw, const int32_t *hw, int32_t k, const int32_t *part,
                   int64_t *maxw)
{
    int32_t *seen = (int32_t *)xmalloc((size_t)k * sizeof(int32_t));
    for (int32_t p = 0; p < k; p++) seen[p] = -1;
    int64_t cut = 0;
    for (int32_t h = 0; h < e; h++) {
        int64_t spans = 0; /* lambda_e: number of parts the hyperedge touches */
        for (int32_t i = off[h]; i < off[h + 1]; i++) {
            int32_t p = part[pins[i]];
            if (seen[p] != h) {
                seen[p] = h;
                spans++;
            }
        }
        if (spans > 1) cut += (int64_t)hedge_weight(hw, h) * (spans - 1);
    }
    if (maxw) {
        int64_t *pw = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
        for (int32_t v = 0; v < n; v++) pw[part[v]] += node_weight(nw, v);
        int64_t best = 0;
        for (int32_t p = 0; p < k; p++)
            if (pw[p] > best) best = pw[p];
        *maxw = best;
        free(pw);
    }
    free(seen);
    return cut;
}

/* ---- Algorithm 1: parallel matching policy (run sequentially) ------------- */

/* Table 1: a smaller value is a higher priority. */
static uint64_t hedge_priority(int32_t policy, int32_t h, int32_t degree, int32_t w)
{
    switch (policy) {
    case OR_HDH: return 0xFFFFFFFFull - (uint32_t)degree;
    case OR_LWD: return (uint32_t)w;
    case OR_HWD: return 0xFFFFFFFFull - (uint32_t)w;
    case OR_RAND: return oracle_hash32((uint32_t)h + 1u);
    default: return (uint32_t)degree; /* LDH */
    }
}

void oracle_match(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                  const int32_t *hw, int32_t policy, int32_t *match)
{
    uint64_t *prio = (uint64_t *)xmalloc((size_t)n * sizeof(uint64_t));
    uint64_t *rnd = (uint64_t *)xmalloc((size_t)n * sizeof(uint64_t));
    int64_t *hid = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    /* node initialisation: all three fields start at infinity */
    for (int32_t v = 0; v < n; v++) {
        prio[v] = NONE64;
        rnd[v] = NONE64;
        hid[v] = INT64_MAX;
    }
    /* first pass: node priority = min over incident hyperedge priorities */
    for (int32_t h = 0; h < e; h++) {
        uint64_t hp = hedge_priority(policy, h, off[h + 1] - off[h], hedge_weight(hw, h));
        for (int32_t i = off[h]; i < off[h + 1]; i++)
            if (hp < prio[pins[i]]) prio[pins[i]] = hp;
    }
    /* second pass: among hyperedges of that priority, the minimum hash */
    for (int32_t h = 0; h < e; h++) {
        uint64_t hp = hedge_priority(policy, h, off[h + 1] - off[h], hedge_weight(hw, h));
        uint64_t hr = oracle_hash32((uint32_t)h + 1u);
        for (int32_t i = off[h]; i < off[h + 1]; i++) {
            int32_t v = pins[i];
            if (hp == prio[v] && hr < rnd[v]) rnd[v] = hr;
        }
    }
    /* third pass: the hyperedge whose hash equals the node's, min id */
    for (int32_t h = 0; h < e; h++) {
        uint64_t hr = oracle_hash32((uint32_t)h + 1u);
        for (int32_t i = off[h]; i < off[h + 1]; i++) {
            int32_t v = pins[i];
            if (hr == rnd[v] && h < hid[v]) hid[v] = h;
        }
    }
    for (int32_t v = 0; v < n; v++) match[v] = hid[v] == INT64_MAX ? -1 : (int32_t)hid[v];
    free(prio);
    free(rnd);
    free(hid);
}

/* ---- Algorithm 2: one coarsening step -------------------------------------- */

typedef struct {
    int32_t src; /* fine hyperedge id */
    int32_t len; /* number of distinct parents */
    const int32_t *q;
} cand_t;

static int cmp_int32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* order candidate coarse hyperedges by pin set, then by source id */
static int cmp_cand(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->len != y->len) return x->len < y->len ? -1 : 1;
    for (int32_t i = 0; i < x->len; i++)
        if (x->q[i] != y->q[i]) return x->q[i] < y->q[i] ? -1 : 1;
    return (x->src > y->src) - (x->src < y->src);
}

void oracle_coarsen(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                    const int32_t *nw, const int32_t *hw, int32_t policy,
                    int32_t *parent, int32_t *cn, int32_t *ce, int32_t *c_off,
                    int32_t *c_pins, int32_t *c_nw, int32_t *c_hw)
{
    int32_t *match = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    oracle_match(n, e, off, pins, hw, policy, match);

    /* S(h) = nodes matched to h; its size and total weight */
    int32_t *count = (int32_t *)xcalloc((size_t)e, sizeof(int32_t));
    int64_t *gweight = (int64_t *)xcalloc((size_t)e, sizeof(int64_t));
    for (int32_t v = 0; v < n; v++)
        if (match[v] >= 0) {
            count[match[v]]++;
            gweight[match[v]] += node_weight(nw, v);
        }

    /* first loop: sets of more than one matched node are merged */
    int32_t *group = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    for (int32_t v = 0; v < n; v++)
        group[v] = (match[v] >= 0 && count[match[v]] >= 2) ? match[v] : -1;

    /* second loop: a singleton set {u} joins the lightest merged node among the
     * other pins of its hyperedge (ties: smaller node id); else it stays alone */
    for (int32_t h = 0; h < e; h++) {
        if (count[h] != 1) continue;
        int32_t u = -1;
        for (int32_t i = off[h]; i < off[h + 1]; i++)
            if (match[pins[i]] == h) u = pins[i];
        int32_t best = -1;
        for (int32_t i = off[h]; i < off[h + 1]; i++) {
            int32_t v = pins[i];
            if (v == u || count[match[v]] < 2) continue;
            if (best < 0 || gweight[match[v]] < gweight[match[best]] ||
                (gweight[match[v]] == gweight[match[best]] && v < best))
                best = v;
        }
        if (best >= 0) group[u] = match[best];
    }

    /* coarse nodes, numbered by the smallest fine id of each group */
    int32_t *leader = (int32_t *)xmalloc((size_t)e * sizeof(int32_t));
    for (int32_t h = 0; h < e; h++) leader[h] = INT32_MAX;
    for (int32_t v = 0; v < n; v++)
        if (group[v] >= 0 && v < leader[group[v]]) leader[group[v]] = v;
    int32_t *cid = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    int32_t ncoarse = 0;
    for (int32_t v = 0; v < n; v++)
        if (group[v] < 0 || leader[group[v]] == v) cid[v] = ncoarse++;
    for (int32_t c = 0; c < ncoarse; c++) c_nw[c] = 0;
    for (int32_t v = 0; v < n; v++) {
        parent[v] = group[v] < 0 ? cid[v] : cid[leader[group[v]]];
        c_nw[parent[v]] += node_weight(nw, v);
    }

    /* third loop: each hyperedge becomes the set of its pins' parents, kept
     * when it has more than one */
    int32_t *qbuf = (int32_t *)xmalloc((size_t)(e ? off[e] : 0) * sizeof(int32_t));
    cand_t *cand = (cand_t *)xmalloc((size_t)e * sizeof(cand_t));
    int32_t *qlen = (int32_t *)xmalloc((size_t)e * sizeof(int32_t));
    int32_t ncand = 0;
    for (int32_t h = 0; h < e; h++) {
        int32_t d = off[h + 1] - off[h];
        int32_t *q = qbuf + off[h];
        for (int32_t i = 0; i < d; i++) q[i] = parent[pins[off[h] + i]];
        qsort(q, (size_t)d, sizeof(int32_t), cmp_int32);
        int32_t len = 0;
        for (int32_t i = 0; i < d; i++)
            if (len == 0 || q[i] != q[len - 1]) q[len++] = q[i];
        qlen[h] = len;
        if (len >= 2) {
            cand[ncand].src = h;
            cand[ncand].len = len;
            cand[ncand].q = q;
            ncand++;
        }
    }

    /* identical coarse hyperedges: keep the one of least source id, sum weights */
    qsort(cand, (size_t)ncand, sizeof(cand_t), cmp_cand);
    int32_t *rep = (int32_t *)xmalloc((size_t)e * sizeof(int32_t));
    int64_t *wsum = (int64_t *)xcalloc((size_t)e, sizeof(int64_t));
    for (int32_t h = 0; h < e; h++) rep[h] = -1;
    for (int32_t i = 0; i < ncand; i++) {
        int same = i > 0 && cand[i].len == cand[i - 1].len &&
                   memcmp(cand[i].q, cand[i - 1].q, (size_t)cand[i].len * sizeof(int32_t)) == 0;
        rep[cand[i].src] = same ? rep[cand[i - 1].src] : cand[i].src;
        wsum[rep[cand[i].src]] += hedge_weight(hw, cand[i].src);
    }
    int32_t nce = 0, np = 0;
    c_off[0] = 0;
    for (int32_t h = 0; h < e; h++) {
        if (rep[h] != h) continue;
        const int32_t *q = qbuf + off[h];
        int32_t len = qlen[h];
        memcpy(c_pins + np, q, (size_t)len * sizeof(int32_t));
        np += len;
        c_hw[nce] = (int32_t)wsum[h];
        c_off[++nce] = np;
    }
    *cn = ncoarse;
    *ce = nce;

    free(match);
    free(count);
    free(gweight);
    free(group);
    free(leader);
    free(cid);
    free(qbuf);
    free(cand);
    free(qlen);
    free(rep);
    free(wsum);
}

/* ---- Algorithm 4: move gains ------------------------------------------------ */

void oracle_gains(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                  const int32_t *hw, const uint8_t *side, int32_t *gain)
{
    for (int32_t v = 0; v < n; v++) gain[v] = 0;
    for (int32_t h = 0; h < e; h++) {
        int32_t d = off[h + 1] - off[h];
        int32_t n1 = 0;
        for (int32_t i = off[h]; i < off[h + 1]; i++) n1 += side[pins[i]];
        int32_t n0 = d - n1;
        int32_t w = hedge_weight(hw, h);
        for (int32_t i = off[h]; i < off[h + 1]; i++) {
            int32_t u = pins[i];
            int32_t ni = side[u] ? n1 : n0;
            if (ni == 1)
                gain[u] += w; /* u alone on its side: moving it uncuts h */
            else if (ni == d)
                gain[u] -= w; /* h entirely on u's side: moving u cuts h */
        }
    }
}

/* ---- balance bounds (problem statement, applied per bisection) ------------- */

void oracle_bounds(int64_t total_w, int32_t k0, int32_t k1, uint64_t F, int64_t *max0,
                   int64_t *max1)
{
    int64_t ks = (int64_t)k0 + k1;
    for (int s = 0; s < 2; s++) {
        int64_t kk = s ? k1 : k0;
        unsigned __int128 a = (unsigned __int128)(uint64_t)total_w * (uint64_t)kk * F;
        int64_t fl = (int64_t)(a / ((unsigned __int128)(uint64_t)ks << 32));
        int64_t ce = (total_w * kk + ks - 1) / ks;
        int64_t m = fl > ce ? fl : ce;
        if (s) *max1 = m;
        else *max0 = m;
    }
}

uint64_t oracle_eps_factor(int32_t k, double eps)
{
    int32_t levels = 0;
    while (((int64_t)1 << levels) < (int64_t)k) levels++;
    if (levels < 1) levels = 1;
    double f = pow(1.0 + eps, 1.0 / (double)levels);
    /* Any factor of 2^30 or more already lets one side hold the whole weight
     * (weights sum below 2^31), so larger ones are capped at 2^62: the bounds
     * they give behave identically, and the conversion stays in range. */
    if (!(f < 1073741824.0)) return (uint64_t)1 << 62;
    return (uint64_t)floor(ldexp(f, 32));
}

/* ---- ordering by (gain descending, node id ascending) ----------------------- */

typedef struct {
    int32_t gain;
    int32_t id;
} gain_id_t;

static int cmp_gain_id(const void *a, const void *b)
{
    const gain_id_t *x = (const gain_id_t *)a, *y = (const gain_id_t *)b;
    if (x->gain != y->gain) return x->gain > y->gain ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* ---- Algorithm 3: initial partitioning -------------------------------------- */

void oracle_initial(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                    const int32_t *nw, const int32_t *hw, int32_t k0, int32_t k1,
                    uint8_t *side)
{
    int64_t ks = (int64_t)k0 + k1;
    int64_t total = 0, w0 = 0;
    for (int32_t v = 0; v < n; v++) {
        side[v] = 1; /* P0 empty, P1 = all nodes */
        total += node_weight(nw, v);
    }
    int64_t m = ceil_sqrt(n);
    int32_t in_p1 = n;
    int32_t *gain = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    gain_id_t *cand = (gain_id_t *)xmalloc((size_t)n * sizeof(gain_id_t));
    /* grow P0 until it holds its share (k0 of k_sub parts) of the weight */
    while (w0 * ks < total * k0 && in_p1 > 0) {
        oracle_gains(n, e, off, pins, hw, side, gain);
        int32_t c = 0;
        for (int32_t v = 0; v < n; v++)
            if (side[v] == 1) {
                cand[c].gain = gain[v];
                cand[c].id = v;
                c++;
            }
        qsort(cand, (size_t)c, sizeof(gain_id_t), cmp_gain_id);
        int32_t take = (int32_t)(m < c ? m : c);
        for (int32_t i = 0; i < take; i++) {
            side[cand[i].id] = 0;
            w0 += node_weight(nw, cand[i].id);
        }
        in_p1 -= take;
    }
    free(gain);
    free(cand);
}

/* ---- Algorithm 5: refinement and the balance step --------------------------- */

int32_t oracle_refine(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                      const int32_t *nw, const int32_t *hw, int32_t iters, int64_t max0,
                      int64_t max1, uint8_t *side)
{
    int32_t *gain = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    gain_id_t *l0 = (gain_id_t *)xmalloc((size_t)n * sizeof(gain_id_t));
    gain_id_t *l1 = (gain_id_t *)xmalloc((size_t)n * sizeof(gain_id_t));

    for (int32_t it = 0; it < iters; it++) {
        oracle_gains(n, e, off, pins, hw, side, gain);
        int32_t c0 = 0, c1 = 0;
        for (int32_t v = 0; v < n; v++) {
            if (gain[v] < 0) continue;
            gain_id_t g = {gain[v], v};
            if (side[v] == 0) l0[c0++] = g;
            else l1[c1++] = g;
        }
        qsort(l0, (size_t)c0, sizeof(gain_id_t), cmp_gain_id);
        qsort(l1, (size_t)c1, sizeof(gain_id_t), cmp_gain_id);
        int32_t l = c0 < c1 ? c0 : c1;
        for (int32_t i = 0; i < l; i++) {
            side[l0[i].id] = 1;
            side[l1[i].id] = 0;
        }
    }

    /* balance: move top-gain nodes off the heavier-than-allowed side */
    int64_t m = ceil_sqrt(n);
    int32_t stuck = 0;
    for (;;) {
        int64_t w[2] = {0, 0};
        for (int32_t v = 0; v < n; v++) w[side[v]] += node_weight(nw, v);
        int h;
        if (w[0] > max0) h = 0;
        else if (w[1] > max1) h = 1;
        else break;
        int64_t need = w[h] - (h ? max1 : max0);
        int64_t room = (h ? max0 : max1) - w[1 - h];
        oracle_gains(n, e, off, pins, hw, side, gain);
        int32_t c = 0;
        for (int32_t v = 0; v < n; v++)
            if (side[v] == h) {
                l0[c].gain = gain[v];
                l0[c].id = v;
                c++;
            }
        qsort(l0, (size_t)c, sizeof(gain_id_t), cmp_gain_id);
        int32_t lim = (int32_t)(m < c ? m : c);
        /* shortest prefix that removes the excess (or the whole limit) ... */
        int32_t p1 = lim;
        int64_t acc = 0;
        for (int32_t j = 0; j < lim; j++) {
            acc += node_weight(nw, l0[j].id);
            if (acc >= need) {
                p1 = j + 1;
                break;
            }
        }
        /* ... cut back to what the other side can take */
        int32_t p = 0;
        acc = 0;
        for (int32_t j = 0; j < p1; j++) {
            int64_t wj = node_weight(nw, l0[j].id);
            if (acc + wj > room) break;
            acc += wj;
            p = j + 1;
        }
        if (p == 0) {
            stuck = 1;
            break;
        }
        for (int32_t j = 0; j < p; j++) side[l0[j].id] = (uint8_t)(1 - h);
    }
    free(gain);
    free(l0);
    free(l1);
    return stuck;
}

/* ---- multilevel bisection (Section 2.3 with Algorithms 1-5) ----------------- */

typedef struct {
    int32_t n, e;
    int32_t *off, *pins, *nw, *hw;
} level_t;

static oracle_params default_params(void)
{
    oracle_params p = {OR_LDH, 25, 2, 100};
    return p;
}

void oracle_bisect(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                   const int32_t *nw, const int32_t *hw, int32_t k0, int32_t k1, uint64_t F,
                   const oracle_params *prm_in, uint8_t *side, int32_t *levels_out)
{
    oracle_params prm = prm_in ? *prm_in : default_params();
    int32_t maxl = prm.max_levels < 0 ? 0 : prm.max_levels;
    level_t *lv = (level_t *)xcalloc((size_t)maxl + 1, sizeof(level_t));
    int32_t **parent = (int32_t **)xcalloc((size_t)maxl + 1, sizeof(int32_t *));

    /* level 0 is the input itself (copied so every level owns its arrays) */
    int32_t p0 = e ? off[e] : 0;
    lv[0].n = n;
    lv[0].e = e;
    lv[0].off = (int32_t *)xmalloc(((size_t)e + 1) * sizeof(int32_t));
    lv[0].pins = (int32_t *)xmalloc((size_t)p0 * sizeof(int32_t));
    lv[0].nw = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    lv[0].hw = (int32_t *)xmalloc((size_t)e * sizeof(int32_t));
    memcpy(lv[0].off, off, ((size_t)e + 1) * sizeof(int32_t));
    memcpy(lv[0].pins, pins, (size_t)p0 * sizeof(int32_t));
    int64_t total = 0;
    for (int32_t v = 0; v < n; v++) {
        lv[0].nw[v] = node_weight(nw, v);
        total += lv[0].nw[v];
    }
    for (int32_t h = 0; h < e; h++) lv[0].hw[h] = hedge_weight(hw, h);

    int64_t max0, max1;
    oracle_bounds(total, k0, k1, F, &max0, &max1);

    /* coarsening phase */
    int32_t l = 0;
    while (l < maxl && lv[l].e > 0 && lv[l].n > prm.min_coarse_nodes) {
        level_t *f = &lv[l], *c = &lv[l + 1];
        int32_t fp = f->off[f->e];
        parent[l] = (int32_t *)xmalloc((size_t)f->n * sizeof(int32_t));
        c->off = (int32_t *)xmalloc(((size_t)f->e + 1) * sizeof(int32_t));
        c->pins = (int32_t *)xmalloc((size_t)fp * sizeof(int32_t));
        c->nw = (int32_t *)xmalloc((size_t)f->n * sizeof(int32_t));
        c->hw = (int32_t *)xmalloc((size_t)f->e * sizeof(int32_t));
        oracle_coarsen(f->n, f->e, f->off, f->pins, f->nw, f->hw, prm.policy, parent[l], &c->n,
                       &c->e, c->off, c->pins, c->nw, c->hw);
        l++;
    }
    if (levels_out) *levels_out = l;

    /* initial partitioning of the coarsest graph, then refinement upwards */
    uint8_t *cur = (uint8_t *)xmalloc((size_t)lv[l].n);
    oracle_initial(lv[l].n, lv[l].e, lv[l].off, lv[l].pins, lv[l].nw, lv[l].hw, k0, k1, cur);
    oracle_refine(lv[l].n, lv[l].e, lv[l].off, lv[l].pins, lv[l].nw, lv[l].hw,
                  prm.refine_iters, max0, max1, cur);
    for (int32_t j = l - 1; j >= 0; j--) {
        uint8_t *fine = (uint8_t *)xmalloc((size_t)lv[j].n);
        for (int32_t v = 0; v < lv[j].n; v++) fine[v] = cur[parent[j][v]]; /* projection */
        free(cur);
        cur = fine;
        oracle_refine(lv[j].n, lv[j].e, lv[j].off, lv[j].pins, lv[j].nw, lv[j].hw,
                      prm.refine_iters, max0, max1, cur);
    }
    memcpy(side, cur, (size_t)n);
    free(cur);
    for (int32_t j = 0; j <= l; j++) {
        free(lv[j].off);
        free(lv[j].pins);
        free(lv[j].nw);
        free(lv[j].hw);
        free(parent[j]);
    }
    free(lv);
    free(parent);
}

/* ---- Algorithm 6: nested k-way by recursive bisection ----------------------- */

typedef struct {
    level_t g;
    int32_t *orig; /* node id in the input graph */
    int32_t lo, ks;
} task_t;

int32_t oracle_partition(int32_t n, int32_t e, const int32_t *off, const int32_t *pins,
                         const int32_t *nw, const int32_t *hw, int32_t k, double eps,
                         const oracle_params *prm_in, int32_t *part_out, int64_t *cut_out)
{
    if (n < 0 || e < 0 || k < 1 || !(eps >= 0.0) || (e > 0 && (!off || !pins))) return -1;
    oracle_params prm = prm_in ? *prm_in : default_params();
    int32_t *part = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));

    if (k > 1) {
        uint64_t F = oracle_eps_factor(k, eps);
        /* hyperedges with fewer than two pins can never be cut: drop them */
        task_t root;
        memset(&root, 0, sizeof(root));
        root.g.n = n;
        root.g.off = (int32_t *)xmalloc(((size_t)e + 1) * sizeof(int32_t));
        root.g.pins = (int32_t *)xmalloc((size_t)(e ? off[e] : 0) * sizeof(int32_t));
        root.g.hw = (int32_t *)xmalloc((size_t)e * sizeof(int32_t));
        root.g.nw = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
        root.orig = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
        root.g.off[0] = 0;
        for (int32_t h = 0; h < e; h++) {
            int32_t d = off[h + 1] - off[h];
            if (d < 2) continue;
            memcpy(root.g.pins + root.g.off[root.g.e], pins + off[h], (size_t)d * sizeof(int32_t));
            root.g.hw[root.g.e] = hedge_weight(hw, h);
            root.g.off[root.g.e + 1] = root.g.off[root.g.e] + d;
            root.g.e++;
        }
        for (int32_t v = 0; v < n; v++) {
            root.g.nw[v] = node_weight(nw, v);
            root.orig[v] = v;
        }
        root.lo = 0;
        root.ks = k;

        /* breadth-first over the bisection tree: one tree level after another */
        size_t cap = 16, head = 0, tail = 0;
        task_t *q = (task_t *)xmalloc(cap * sizeof(task_t));
        q[tail++] = root;
        while (head < tail) {
            task_t t = q[head++];
            if (t.ks == 1) {
                for (int32_t v = 0; v < t.g.n; v++) part[t.orig[v]] = t.lo;
            } else {
                int32_t k0 = (t.ks + 1) / 2, k1 = t.ks - k0;
                uint8_t *side = (uint8_t *)xmalloc((size_t)t.g.n);
                oracle_bisect(t.g.n, t.g.e, t.g.off, t.g.pins, t.g.nw, t.g.hw, k0, k1, F, &prm,
                              side, NULL);
                int32_t *local = (int32_t *)xmalloc((size_t)t.g.n * sizeof(int32_t));
                for (int s = 0; s < 2; s++) {
                    task_t c;
                    memset(&c, 0, sizeof(c));
                    c.lo = t.lo + (s ? k0 : 0);
                    c.ks = s ? k1 : k0;
                    /* nodes of side s, in ascending id, renumbered from 0 */
                    for (int32_t v = 0; v < t.g.n; v++)
                        if (side[v] == s) local[v] = c.g.n++;
                    c.g.nw = (int32_t *)xmalloc((size_t)c.g.n * sizeof(int32_t));
                    c.orig = (int32_t *)xmalloc((size_t)c.g.n * sizeof(int32_t));
                    for (int32_t v = 0; v < t.g.n; v++)
                        if (side[v] == s) {
                            c.g.nw[local[v]] = t.g.nw[v];
                            c.orig[local[v]] = t.orig[v];
                        }
                    /* cut-net splitting: each hyperedge keeps its side-s pins,
                     * and survives when at least two remain */
                    c.g.off = (int32_t *)xmalloc(((size_t)t.g.e + 1) * sizeof(int32_t));
                    c.g.pins = (int32_t *)xmalloc((size_t)(t.g.e ? t.g.off[t.g.e] : 0) *
                                                  sizeof(int32_t));
                    c.g.hw = (int32_t *)xmalloc((size_t)t.g.e * sizeof(int32_t));
                    c.g.off[0] = 0;
                    for (int32_t h = 0; h < t.g.e; h++) {
                        int32_t cnt = 0;
                        for (int32_t i = t.g.off[h]; i < t.g.off[h + 1]; i++)
                            cnt += side[t.g.pins[i]] == s;
                        if (cnt < 2) continue;
                        int32_t at = c.g.off[c.g.e];
                        for (int32_t i = t.g.off[h]; i < t.g.off[h + 1]; i++)
                            if (side[t.g.pins[i]] == s) c.g.pins[at++] = local[t.g.pins[i]];
                        c.g.hw[c.g.e] = t.g.hw[h];
                        c.g.off[c.g.e + 1] = at;
                        c.g.e++;
                    }
                    if (tail == cap) {
                        cap *= 2;
                        q = (task_t *)realloc(q, cap * sizeof(task_t));
                        if (!q) abort();
                    }
                    q[tail++] = c;
                }
                free(local);
                free(side);
            }
            free(t.g.off);
            free(t.g.pins);
            free(t.g.nw);
            free(t.g.hw);
            free(t.orig);
        }
        free(q);
    }

    if (part_out) memcpy(part_out, part, (size_t)n * sizeof(int32_t));
    if (cut_out) *cut_out = k > 1 ? oracle_cut(n, e, off, pins, nw, hw, k, part, NULL) : 0;
    free(part);
    return 0;
}
