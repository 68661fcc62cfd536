/*
 * CPU oracle for the online muon trigger's L1 seeds, causal N-fold count,
 * trigger fires and event windows.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is compared against.  It is used by the
 * tests, by the smoke check and by the benchmark's CPU-baseline leg, and by
 * nothing else; the product library neither links nor calls it, and this
 * file includes no header of the product library.
 *
 * What is computed (the paper: Bouhadef, Morganti, Terreni, "Parallel
 * Neutrino Triggers using GPUs for an Underwater Telescope", GPUHEP2014):
 *
 *   hits k = 0..n-1 with PMT p_k, time t_k (int64 ns), charge q_k (0.01 pe);
 *   floor_id[P]; thr[P*P] (row-major, integer ns); parameters
 *   Q (charge threshold), tau (floor-coincidence window), W (causal window
 *   cap), N (fold threshold), H (half event window).
 *
 *   seed  (Sec. 4.2 trigger list: charge over threshold QTRIG and floor
 *          coincidence FC; Sec. 3 charge trigger):
 *     S_k = q_k >= Q  or  (tau >= 0 and there is a hit m with p_m != p_k,
 *           floor_id[p_m] == floor_id[p_k] and |t_k - t_m| <= tau)
 *   fold  (Sec. 3: space-time correlation of hits within less than 3 us):
 *     for S_k:  fold_k = 1 + #{ m != k : S_m and |t_k - t_m| <= min(thr[p_k][p_m], W) }
 *   fires (N-fold trigger): F = { k : S_k and fold_k >= N }, ordered by (t, p, k)
 *   events (Sec. 2: a 6 us window centred on the trigger seed goes to the
 *           Event Manager; Sec. 4.2: hits within +-3 us of a trigger seed are
 *           tagged): each fire opens [t-H, t+H]; walking F in order, a fire
 *           whose window starts at or before the current event's end extends
 *           it, otherwise it opens a new event.
 *   level 0 (optional; Sec. 3: a level-0 trigger of N hits in a fixed time
 *           window TW, N7TW1000, N7TW500 for the 84-PMT tower; Sec. 4.1:
 *           DN7TW1000 counts hits of different PMTs): with N = l0_n > 0,
 *     L_k = there is a hit i with t_i <= t_k < t_i + TW whose window
 *           [t_i, t_i + TW) holds >= N hits (>= N distinct PMTs for DN);
 *           the seed rule then runs on the hits that pass: S_k requires L_k,
 *           and a floor partner m requires L_m
 *   seed menu (optional; Sec. 4.1 trigger list: SC, two adjacent PMTs within
 *           20 ns; FC, two PMTs of one floor within 100 ns; AFC, two PMTs on
 *           consecutive floors within 250 ns; Sec. 5: the candidate selection
 *           [SC and AFC] or [FC and AFC]): with partner m != k on another PMT
 *           (passing level 0 when it is on),
 *     FC_k  floor_id equal, |t_k - t_m| <= tau_f (t_floor_ns, the rule above)
 *     SC_k  floor_id equal and adj_id equal, |t_k - t_m| <= tau_sc (t_adj_ns)
 *     AFC_k |floor_id difference| = 1, |t_k - t_m| <= tau_afc (t_afloor_ns)
 *           (a negative window turns its rule off; adj_id NULL: no two PMTs
 *           adjacent); seed_mode 0: S_k = Q_k or FC_k or SC_k or AFC_k;
 *           seed_mode 1: S_k = Q_k or ((SC_k or FC_k) and AFC_k)
 *   tagged hits (Sec. 4.2: the hits within +-3 us of a trigger seed are
 *           marked for storage): T = { k : |t_k - t_f| <= H for some f in F },
 *           ordered by (t, p, k)
 *
 * Two forms:  "strict" evaluates every pair (O(n^2));  "blocked" evaluates
 * the very same pair tests, restricted to hits in the same or adjacent time
 * blocks of width B >= the largest window the test can accept (tau for
 * seeds, W for folds), which is complete because any accepted pair has
 * |dt| <= B and therefore lies in the same or an adjacent block.
 *
 * Readings of points the paper leaves open are listed with the test
 * fixtures: all windows inclusive; the fold counts the seed itself; a floor
 * partner must be a different PMT and need not be a seed; same-PMT seed
 * pairs count when the table allows (thr[p][p]); the table row is the seed
 * being counted; equal times order by (pmt, input index); slices are
 * self-contained and windows are not clipped.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint32_t q_seed;
    int32_t  t_floor_ns;
    uint32_t w_ns;
    uint32_t min_fold;
    uint32_t half_event_ns;
    uint32_t l0_n;           /* level-0 prefilter: hits (0 = off) ... */
    uint32_t l0_tw_ns;       /* ... within this window ... */
    uint32_t l0_distinct;    /* ... counting distinct PMTs when set */
    int32_t  t_adj_ns;       /* SC window (adjacent PMTs); < 0 off */
    int32_t  t_afloor_ns;    /* AFC window (consecutive floors); < 0 off */
    uint32_t seed_mode;      /* 0: any enabled rule; 1: Q or ((SC or FC) and AFC) */
} orc_params;

typedef struct {
    int64_t  t_ns;
    uint32_t hit_index;
    uint32_t fold;
    uint16_t pmt_id;
    uint16_t pad[3];
} orc_fire;

typedef struct {
    int64_t  t_trig, t_begin, t_end;
    uint32_t n_fire, max_fold;
} orc_event;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_ENOMEM = -3, ORC_EOVERFLOW = -5 };

static int64_t absdiff(int64_t a, int64_t b) { return a > b ? a - b : b - a; }

/* Input validation: every PMT index below P, fewer than 2^32 hits, time span
 * below 2^31 ns, and event windows representable in int64. */
int orc_validate(uint64_t n, const uint16_t *pmt, const int64_t *t, uint32_t n_pmt,
                 const orc_params *prm)
{
    if (n >= (1ull << 32)) return ORC_ERANGE;
    if (n == 0) return ORC_OK;
    int64_t lo = t[0], hi = t[0];
    for (uint64_t k = 0; k < n; ++k) {
        if (pmt[k] >= n_pmt) return ORC_ERANGE;
        if (t[k] < lo) lo = t[k];
        if (t[k] > hi) hi = t[k];
    }
    if ((uint64_t)hi - (uint64_t)lo >= (1ull << 31)) return ORC_ERANGE;
    if (lo < INT64_MIN + (int64_t)prm->half_event_ns) return ORC_ERANGE;
    if (hi > INT64_MAX - (int64_t)prm->half_event_ns) return ORC_ERANGE;
    return ORC_OK;
}

/* ---------------------------------------------------------------- strict */

/* Partner rules of hit k met by hit m: bit 0 FC, bit 1 SC, bit 2 AFC. */
static unsigned partner_bits(const uint16_t *pmt, const int64_t *t, const int32_t *floor_id,
                             const int32_t *adj_id, const orc_params *prm, uint64_t k, uint64_t m)
{
    if (m == k || pmt[m] == pmt[k]) return 0;
    const int64_t dt = absdiff(t[k], t[m]);
    const int64_t fk = floor_id[pmt[k]], fm = floor_id[pmt[m]];
    unsigned b = 0;
    if (prm->t_floor_ns >= 0 && fm == fk && dt <= prm->t_floor_ns) b |= 1u;
    if (prm->t_adj_ns >= 0 && adj_id && fm == fk && adj_id[pmt[m]] == adj_id[pmt[k]] && dt <= prm->t_adj_ns)
        b |= 2u;
    if (prm->t_afloor_ns >= 0 && (fm - fk == 1 || fk - fm == 1) && dt <= prm->t_afloor_ns) b |= 4u;
    return b;
}

static int seed_of(int charge, unsigned bits, const orc_params *prm)
{
    const int fc = bits & 1u, sc = (bits >> 1) & 1u, afc = (bits >> 2) & 1u;
    if (prm->seed_mode == 1) return charge || ((sc || fc) && afc);
    return charge || fc || sc || afc;
}

/* Widest partner window (< 0 when no partner rule is on). */
static int64_t partner_reach(const orc_params *prm)
{
    int64_t r = prm->t_floor_ns;
    if (prm->t_adj_ns > r) r = prm->t_adj_ns;
    if (prm->t_afloor_ns > r) r = prm->t_afloor_ns;
    return r;
}

static void seeds_strict(uint64_t n, const uint16_t *pmt, const int64_t *t, const uint16_t *q,
                         const int32_t *floor_id, const int32_t *adj_id, const uint8_t *l0, const orc_params *prm,
                         uint8_t *seed)
{
    const int any_rule = partner_reach(prm) >= 0;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        if (l0 && !l0[k]) { seed[k] = 0; continue; }
        unsigned bits = 0;
        for (uint64_t m = 0; any_rule && m < n; ++m)
            if (!l0 || l0[m]) bits |= partner_bits(pmt, t, floor_id, adj_id, prm, (uint64_t)k, m);
        seed[k] = (uint8_t)seed_of(q[k] >= prm->q_seed, bits, prm);
    }
}

static uint32_t pair_limit(const uint32_t *thr, uint32_t n_pmt, uint16_t pk, uint16_t pm, uint32_t w)
{
    uint32_t lim = thr[(uint64_t)pk * n_pmt + pm];
    return lim < w ? lim : w;
}

static void folds_strict(uint64_t n, const uint16_t *pmt, const int64_t *t, const uint8_t *seed,
                         uint32_t n_pmt, const uint32_t *thr, const orc_params *prm, uint32_t *fold)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        if (!seed[k]) { fold[k] = 0; continue; }
        uint32_t c = 1;
        for (uint64_t m = 0; m < n; ++m) {
            if ((int64_t)m == k || !seed[m]) continue;
            if (absdiff(t[k], t[m]) <= (int64_t)pair_limit(thr, n_pmt, pmt[k], pmt[m], prm->w_ns)) ++c;
        }
        fold[k] = c;
    }
}

/* --------------------------------------------------------------- blocked */

/* Group the indices of the selected hits by time block b = (t - t_lo) / B.
 * start[b]..start[b+1] lists block b's members in input order. */
typedef struct { uint64_t nb; uint64_t *start; uint32_t *member; int64_t t_lo; uint64_t width; } blocks;

static int make_blocks(uint64_t n, const int64_t *t, const uint8_t *sel, uint64_t width, blocks *B)
{
    int64_t lo = 0, hi = 0; int any = 0;
    for (uint64_t k = 0; k < n; ++k) {
        if (sel && !sel[k]) continue;
        if (!any) { lo = hi = t[k]; any = 1; }
        if (t[k] < lo) lo = t[k];
        if (t[k] > hi) hi = t[k];
    }
    uint64_t span = any ? (uint64_t)(hi - lo) : 0;
    uint64_t cnt = 0;
    for (uint64_t k = 0; k < n; ++k) cnt += (!sel || sel[k]);
    /* never more blocks than members: a wider block is still complete */
    uint64_t minw = cnt ? (span + cnt) / cnt : 1;
    if (width < minw) width = minw;
    if (width < 1) width = 1;
    B->t_lo = lo; B->width = width;
    B->nb = span / width + 1;
    B->start = (uint64_t *)calloc(B->nb + 1, sizeof(uint64_t));
    B->member = (uint32_t *)malloc((cnt ? cnt : 1) * sizeof(uint32_t));
    if (!B->start || !B->member) { free(B->start); free(B->member); return ORC_ENOMEM; }
    for (uint64_t k = 0; k < n; ++k)
        if (!sel || sel[k]) B->start[(uint64_t)(t[k] - lo) / width + 1]++;
    for (uint64_t b = 0; b < B->nb; ++b) B->start[b + 1] += B->start[b];
    uint64_t *fill = (uint64_t *)malloc((B->nb + 1) * sizeof(uint64_t));
    if (!fill) { free(B->start); free(B->member); return ORC_ENOMEM; }
    memcpy(fill, B->start, (B->nb + 1) * sizeof(uint64_t));
    for (uint64_t k = 0; k < n; ++k)
        if (!sel || sel[k]) B->member[fill[(uint64_t)(t[k] - lo) / width]++] = (uint32_t)k;
    free(fill);
    return ORC_OK;
}

static void free_blocks(blocks *B) { free(B->start); free(B->member); }

static int seeds_blocked(uint64_t n, const uint16_t *pmt, const int64_t *t, const uint16_t *q,
                         const int32_t *floor_id, const int32_t *adj_id, const uint8_t *l0, const orc_params *prm,
                         uint8_t *seed)
{
    for (uint64_t k = 0; k < n; ++k) seed[k] = seed_of(q[k] >= prm->q_seed, 0u, prm) && (!l0 || l0[k]);
    const int64_t reach = partner_reach(prm);
    if (reach < 0 || n == 0) return ORC_OK;
    blocks B;
    int rc = make_blocks(n, t, NULL, (uint64_t)reach, &B);
    if (rc) return rc;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        if (seed[k] || (l0 && !l0[k])) continue;
        uint64_t b = (uint64_t)(t[k] - B.t_lo) / B.width;
        uint64_t b0 = b ? b - 1 : 0, b1 = b + 1 < B.nb ? b + 1 : b;
        unsigned bits = 0;
        for (uint64_t bb = b0; bb <= b1; ++bb)
            for (uint64_t i = B.start[bb]; i < B.start[bb + 1]; ++i) {
                uint32_t m = B.member[i];
                if (l0 && !l0[m]) continue;
                bits |= partner_bits(pmt, t, floor_id, adj_id, prm, (uint64_t)k, m);
            }
        seed[k] = (uint8_t)seed_of(0, bits, prm);
    }
    free_blocks(&B);
    return ORC_OK;
}

static int folds_blocked(uint64_t n, const uint16_t *pmt, const int64_t *t, const uint8_t *seed,
                         uint32_t n_pmt, const uint32_t *thr, const orc_params *prm, uint32_t *fold)
{
    for (uint64_t k = 0; k < n; ++k) fold[k] = 0;
    if (n == 0) return ORC_OK;
    blocks B;
    int rc = make_blocks(n, t, seed, prm->w_ns, &B);
    if (rc) return rc;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        if (!seed[k]) continue;
        uint64_t b = (uint64_t)(t[k] - B.t_lo) / B.width;
        uint64_t b0 = b ? b - 1 : 0, b1 = b + 1 < B.nb ? b + 1 : b;
        uint32_t c = 1;
        for (uint64_t bb = b0; bb <= b1; ++bb)
            for (uint64_t i = B.start[bb]; i < B.start[bb + 1]; ++i) {
                uint32_t m = B.member[i];
                if ((int64_t)m == k) continue;
                if (absdiff(t[k], t[m]) <= (int64_t)pair_limit(thr, n_pmt, pmt[k], pmt[m], prm->w_ns)) ++c;
            }
        fold[k] = c;
    }
    free_blocks(&B);
    return ORC_OK;
}

/* --------------------------------------------------------------- level 0 */

/* Size of the window [t0, t0 + tw) over the candidates idx[0..nc): its hits,
 * or its distinct PMTs when distinct is set (seen[] has room for nc). */
static uint64_t window_count(const uint16_t *pmt, const int64_t *t, int64_t t0, int64_t tw,
                             const uint32_t *idx, uint64_t nc, int distinct, uint16_t *seen)
{
    uint64_t c = 0;
    for (uint64_t u = 0; u < nc; ++u) {
        const uint32_t m = idx[u];
        if (t[m] < t0 || t[m] - t0 >= tw) continue;
        if (distinct) {
            int dup = 0;
            for (uint64_t v = 0; v < c; ++v)
                if (seen[v] == pmt[m]) { dup = 1; break; }
            if (dup) continue;
            seen[c] = pmt[m];
        }
        ++c;
    }
    return c;
}

/* L_k for every hit.  strict: every hit is a candidate window start and a
 * candidate member; blocked: the same tests restricted to time blocks of
 * width >= TW (a window [t_i, t_i + TW) lies in t_i's block and the next; a
 * window holding t_k starts in t_k's block or the one before). */
static int level0(int strict, uint64_t n, const uint16_t *pmt, const int64_t *t, const orc_params *prm,
                  uint8_t *pass)
{
    const int64_t tw = prm->l0_tw_ns;
    const uint64_t need = prm->l0_n;
    const int distinct = prm->l0_distinct != 0;
    uint8_t *ok = (uint8_t *)calloc(n ? n : 1, 1);
    uint32_t *all = NULL;
    uint16_t *seen = NULL;
    blocks B;
    B.start = NULL; B.member = NULL;
    int rc = ORC_OK;
    if (!ok) return ORC_ENOMEM;
    if (strict) {
        all = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
        seen = (uint16_t *)malloc((n ? n : 1) * sizeof(uint16_t));
        if (!all || !seen) { rc = ORC_ENOMEM; goto out; }
        for (uint64_t k = 0; k < n; ++k) all[k] = (uint32_t)k;
        /* window starting at hit i */
        for (uint64_t i = 0; i < n; ++i) ok[i] = window_count(pmt, t, t[i], tw, all, n, distinct, seen) >= need;
        for (uint64_t k = 0; k < n; ++k) {
            pass[k] = 0;
            for (uint64_t i = 0; i < n && !pass[k]; ++i)
                if (ok[i] && t[i] <= t[k] && t[k] - t[i] < tw) pass[k] = 1;
        }
    } else {
        rc = make_blocks(n, t, NULL, (uint64_t)(tw > 0 ? tw : 1), &B);
        if (rc) goto out;
        uint64_t most = 1;
        for (uint64_t b = 0; b < B.nb; ++b) {
            const uint64_t e = b + 2 <= B.nb ? B.start[b + 2] : B.start[B.nb];
            if (e - B.start[b] > most) most = e - B.start[b];
        }
        seen = (uint16_t *)malloc(most * sizeof(uint16_t));
        if (!seen) { rc = ORC_ENOMEM; goto out; }
        for (uint64_t i = 0; i < n; ++i) {
            const uint64_t b = (uint64_t)(t[i] - B.t_lo) / B.width;
            const uint64_t e = b + 2 <= B.nb ? B.start[b + 2] : B.start[B.nb];
            ok[i] = window_count(pmt, t, t[i], tw, B.member + B.start[b], e - B.start[b], distinct, seen) >= need;
        }
        for (uint64_t k = 0; k < n; ++k) {
            const uint64_t b = (uint64_t)(t[k] - B.t_lo) / B.width;
            const uint64_t b0 = b ? b - 1 : 0;
            pass[k] = 0;
            for (uint64_t u = B.start[b0]; u < B.start[b + 1] && !pass[k]; ++u) {
                const uint32_t i = B.member[u];
                if (ok[i] && t[i] <= t[k] && t[k] - t[i] < tw) pass[k] = 1;
            }
        }
    }
out:
    free(ok); free(all); free(seen);
    if (B.start || B.member) free_blocks(&B);
    return rc;
}

/* ------------------------------------------------------- fires and events */

static int fire_cmp(const void *a, const void *b)
{
    const orc_fire *x = (const orc_fire *)a, *y = (const orc_fire *)b;
    if (x->t_ns != y->t_ns) return x->t_ns < y->t_ns ? -1 : 1;
    if (x->pmt_id != y->pmt_id) return x->pmt_id < y->pmt_id ? -1 : 1;
    if (x->hit_index != y->hit_index) return x->hit_index < y->hit_index ? -1 : 1;
    return 0;
}

/* Fires: every seed whose fold reaches N, ordered by (t, pmt, input index). */
static uint64_t collect_fires(uint64_t n, const uint16_t *pmt, const int64_t *t, const uint8_t *seed,
                              const uint32_t *fold, uint32_t min_fold, orc_fire *out)
{
    uint64_t c = 0;
    for (uint64_t k = 0; k < n; ++k) {
        if (!seed[k] || fold[k] < min_fold) continue;
        orc_fire f;
        memset(&f, 0, sizeof f);
        f.t_ns = t[k]; f.hit_index = (uint32_t)k; f.fold = fold[k]; f.pmt_id = pmt[k];
        out[c++] = f;
    }
    qsort(out, c, sizeof(orc_fire), fire_cmp);
    return c;
}

/* Events: walk the ordered fires; a fire whose window [t-H, t+H] starts at
 * or before the current event's end joins it, otherwise it opens a new one. */
uint64_t orc_events(const orc_fire *f, uint64_t nf, uint32_t half_event_ns, orc_event *ev)
{
    const int64_t H = half_event_ns;
    uint64_t ne = 0;
    for (uint64_t i = 0; i < nf; ++i) {
        if (ne > 0 && f[i].t_ns - H <= ev[ne - 1].t_end) {
            orc_event *e = &ev[ne - 1];
            e->t_end = f[i].t_ns + H;
            e->n_fire += 1;
            if (f[i].fold > e->max_fold) e->max_fold = f[i].fold;
        } else {
            orc_event e;
            e.t_trig = f[i].t_ns; e.t_begin = f[i].t_ns - H; e.t_end = f[i].t_ns + H;
            e.n_fire = 1; e.max_fold = f[i].fold;
            ev[ne++] = e;
        }
    }
    return ne;
}

/* Tagged hits (Sec. 4.2: once the trigger fires, the hits within +-3 us of a
 * trigger seed are marked for storage; Sec. 2: the 6 us window of tower data
 * centred on the trigger seed is what goes to storage).  Hit k is tagged when
 * some fire f has |t_k - t_f| <= H.  fires must be ordered by time (as
 * collect_fires leaves them).  out[] (room for n) receives the tagged hits'
 * input indices ordered by (t, pmt, input index); returns their number, or
 * UINT64_MAX when out of memory. */
uint64_t orc_tag(uint64_t n, const uint16_t *pmt, const int64_t *t, const orc_fire *f, uint64_t nf,
                 uint32_t half_event_ns, uint32_t *out)
{
    const int64_t H = half_event_ns;
    orc_fire *rec = (orc_fire *)malloc((n ? n : 1) * sizeof(orc_fire));
    if (!rec) return UINT64_MAX;
    uint64_t c = 0;
    for (uint64_t k = 0; k < n; ++k) {
        /* the first fire at or after t_k - H; hit k is tagged when it is also at
         * or before t_k + H */
        uint64_t lo = 0, hi = nf;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (f[mid].t_ns < t[k] - H) lo = mid + 1; else hi = mid;
        }
        if (lo < nf && f[lo].t_ns <= t[k] + H) {
            memset(&rec[c], 0, sizeof rec[c]);
            rec[c].t_ns = t[k]; rec[c].pmt_id = pmt[k]; rec[c].hit_index = (uint32_t)k;
            ++c;
        }
    }
    qsort(rec, c, sizeof(orc_fire), fire_cmp);   /* the fires' order: (t, pmt, index) */
    for (uint64_t i = 0; i < c; ++i) out[i] = rec[i].hit_index;
    free(rec);
    return c;
}

/* Whole path.  form 0 = strict, 1 = blocked.  seed_out / fold_out are [n]
 * (by input index).  fires / events need room for up to n records.  Returns
 * ORC_OK or the validation error (outputs then hold zero counts). */
int orc_run(int form, uint64_t n, const uint16_t *pmt, const int64_t *t, const uint16_t *q,
            uint32_t n_pmt, const int32_t *floor_id, const int32_t *adj_id, const uint32_t *thr,
            const orc_params *prm,
            uint8_t *seed_out, uint32_t *fold_out,
            orc_fire *fires, uint64_t *n_fires, orc_event *events, uint64_t *n_events,
            int n_threads)
{
    *n_fires = 0; *n_events = 0;
    if (!prm || n_pmt == 0 || (n && (!pmt || !t || !q))) return ORC_EINVAL;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int rc = orc_validate(n, pmt, t, n_pmt, prm);
    if (rc) return rc;
    uint8_t *l0 = NULL;
    if (prm->l0_n > 0 && n) {
        l0 = (uint8_t *)malloc(n);
        if (!l0) return ORC_ENOMEM;
        rc = level0(form == 0, n, pmt, t, prm, l0);
        if (rc) { free(l0); return rc; }
    }
    if (form == 0) {
        seeds_strict(n, pmt, t, q, floor_id, adj_id, l0, prm, seed_out);
        folds_strict(n, pmt, t, seed_out, n_pmt, thr, prm, fold_out);
    } else {
        rc = seeds_blocked(n, pmt, t, q, floor_id, adj_id, l0, prm, seed_out);
        if (!rc) rc = folds_blocked(n, pmt, t, seed_out, n_pmt, thr, prm, fold_out);
        if (rc) { free(l0); return rc; }
    }
    free(l0);
    *n_fires = collect_fires(n, pmt, t, seed_out, fold_out, prm->min_fold, fires);
    *n_events = orc_events(fires, *n_fires, prm->half_event_ns, events);
    return ORC_OK;
}

/* Sampled check at any size: seed flag and fold of the hits listed in ks,
 * each from the definition evaluated on the hits within W + tau of it (one
 * pass over the slice per sample; every partner a test can accept lies in
 * that neighbourhood).  fold is 0 for a non-seed. */
int orc_point(uint64_t n, const uint16_t *pmt, const int64_t *t, const uint16_t *q,
              uint32_t n_pmt, const int32_t *floor_id, const uint32_t *thr, const orc_params *prm,
              const uint64_t *ks, uint64_t nk, uint8_t *seed_k, uint32_t *fold_k, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int rc = orc_validate(n, pmt, t, n_pmt, prm);
    if (rc) return rc;
    /* sampled checks cover the rule without level 0 and the seed menu */
    if (prm->l0_n || prm->t_adj_ns >= 0 || prm->t_afloor_ns >= 0 || prm->seed_mode) return ORC_EINVAL;
    const int64_t tau = prm->t_floor_ns;
    const int64_t reach = (int64_t)prm->w_ns + (tau > 0 ? tau : 0);
    int fail = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < (int64_t)nk; ++s) {
        uint64_t k = ks[s];
        if (k >= n) { fail = 1; continue; }
        uint64_t cap = 1024, L = 0;
        uint64_t *near = (uint64_t *)malloc(cap * sizeof(uint64_t));
        for (uint64_t m = 0; m < n && near; ++m) {
            if (absdiff(t[m], t[k]) > reach) continue;
            if (L == cap) { cap *= 2; near = (uint64_t *)realloc(near, cap * sizeof(uint64_t)); if (!near) break; }
            near[L++] = m;
        }
        if (!near) { fail = 1; continue; }
        /* seed flag of a neighbour m (within W of k): its floor partners lie within tau of it */
        uint8_t sk = 0; uint32_t fk = 0;
        for (uint64_t a = 0; a < L; ++a) {
            uint64_t m = near[a];
            if (m != k && absdiff(t[m], t[k]) > (int64_t)prm->w_ns) continue;
            int s_m = q[m] >= prm->q_seed;
            if (!s_m && tau >= 0)
                for (uint64_t b = 0; b < L && !s_m; ++b) {
                    uint64_t r = near[b];
                    if (pmt[r] != pmt[m] && floor_id[pmt[r]] == floor_id[pmt[m]] && absdiff(t[r], t[m]) <= tau)
                        s_m = 1;
                }
            if (m == k) { sk = (uint8_t)s_m; continue; }
            if (s_m && absdiff(t[k], t[m]) <= (int64_t)pair_limit(thr, n_pmt, pmt[k], pmt[m], prm->w_ns)) ++fk;
        }
        seed_k[s] = sk;
        fold_k[s] = sk ? fk + 1 : 0;
        free(near);
    }
    return fail ? ORC_EINVAL : ORC_OK;
}
