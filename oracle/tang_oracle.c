/*
 * Linear-scan oracle for 5-field packet classification.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no code, header or table with the GPU library.
 *
 * What it computes (Sec. 2.1, the problem statement): a rule has prefix conditions on
 * SIP and DIP, inclusive ranges on SP and DP, and an exact-or-wildcard protocol; the
 * answer for a packet is the highest-priority rule that matches it. Priorities follow
 * the worked example of Table 1 / Sec. 4.2: a lower number wins. Equal priorities are
 * broken by the lower id, so (priority, id) is a total order and exactly one answer
 * exists. No match gives 0xFFFFFFFF.
 *
 * A prefix of length l keeps the top l bits and zero-fills the rest (the "11*" -> 110
 * example of Sec. 4.3); l = 0 keeps nothing (a C shift by 32 is undefined, so it is
 * special-cased).
 *
 * Method: sort the live rules by (priority, id), then scan each packet's rule list in
 * that order and stop at the first match, which is then the highest-priority match (the
 * rules of a bucket are checked in turn in Sec. 5.1.1). Packets are split over POSIX
 * threads.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Same byte layout as the inputs the tests hand in (28-byte rule, 16-byte header). */
typedef struct {
    uint32_t sip, dip, priority, id;
    uint16_t sp_lo, sp_hi, dp_lo, dp_hi;
    uint8_t sip_len, dip_len, proto, proto_mask;
} orc_rule;

typedef struct {
    uint32_t sip, dip;
    uint16_t sp, dp;
    uint8_t proto, pad[3];
} orc_hdr;

static uint32_t orc_prefix_mask(unsigned len) {
    if (len == 0) return 0u;
    if (len >= 32) return 0xFFFFFFFFu;
    return 0xFFFFFFFFu << (32u - len);
}

/* Rules in (priority, id) order, structure of arrays. */
typedef struct {
    size_t n;
    uint32_t *sval, *smask, *dval, *dmask, *id;
    uint16_t *splo, *sphi, *dplo, *dphi;
    uint8_t *proto, *pmask;
} orc_table;

static int orc_cmp(const void* a, const void* b) {
    const orc_rule* x = *(const orc_rule* const*)a;
    const orc_rule* y = *(const orc_rule* const*)b;
    if (x->priority != y->priority) return x->priority < y->priority ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

static int orc_match(const orc_table* t, size_t i, const orc_hdr* p) {
    if ((p->sip & t->smask[i]) != t->sval[i]) return 0;
    if ((p->dip & t->dmask[i]) != t->dval[i]) return 0;
    if (p->sp < t->splo[i] || p->sp > t->sphi[i]) return 0;
    if (p->dp < t->dplo[i] || p->dp > t->dphi[i]) return 0;
    if (t->pmask[i] != 0 && p->proto != t->proto[i]) return 0;
    return 1;
}

typedef struct {
    const orc_table* t;
    const orc_hdr* pkts;
    uint32_t* out;
    uint64_t* scanned; /* optional per-packet scan length */
    size_t lo, hi;
} orc_job;

static void* orc_worker(void* arg) {
    orc_job* j = (orc_job*)arg;
    for (size_t k = j->lo; k < j->hi; ++k) {
        uint32_t ans = 0xFFFFFFFFu;
        size_t i = 0;
        for (; i < j->t->n; ++i) {
            if (orc_match(j->t, i, &j->pkts[k])) { ans = j->t->id[i]; break; }
        }
        j->out[k] = ans;
        if (j->scanned) j->scanned[k] = (i < j->t->n) ? i + 1 : j->t->n;
    }
    return NULL;
}

static void orc_free(orc_table* t) {
    free(t->sval); free(t->smask); free(t->dval); free(t->dmask); free(t->id);
    free(t->splo); free(t->sphi); free(t->dplo); free(t->dphi);
    free(t->proto); free(t->pmask);
}

/*
 * rules[n_rules]: the ruleset; live (may be NULL = all live) marks which rules exist.
 * pkts[n_pkts] -> out[n_pkts] rule ids (0xFFFFFFFF = no match).
 * scanned (may be NULL): per packet, how many rules the early-exit scan tested.
 * threads <= 0 means 1. Returns 0, or -1 on allocation failure.
 */
int oracle_classify(const orc_rule* rules, size_t n_rules, const uint8_t* live,
                    const orc_hdr* pkts, size_t n_pkts, uint32_t* out,
                    uint64_t* scanned, int threads) {
    orc_table t;
    memset(&t, 0, sizeof t);
    const orc_rule** order = (const orc_rule**)malloc((n_rules ? n_rules : 1) * sizeof *order);
    if (!order) return -1;
    size_t m = 0;
    for (size_t i = 0; i < n_rules; ++i)
        if (!live || live[i]) order[m++] = &rules[i];
    qsort(order, m, sizeof *order, orc_cmp);

    size_t cap = m ? m : 1;
    t.n = m;
    t.sval = malloc(cap * 4); t.smask = malloc(cap * 4);
    t.dval = malloc(cap * 4); t.dmask = malloc(cap * 4); t.id = malloc(cap * 4);
    t.splo = malloc(cap * 2); t.sphi = malloc(cap * 2);
    t.dplo = malloc(cap * 2); t.dphi = malloc(cap * 2);
    t.proto = malloc(cap); t.pmask = malloc(cap);
    if (!t.sval || !t.smask || !t.dval || !t.dmask || !t.id || !t.splo || !t.sphi ||
        !t.dplo || !t.dphi || !t.proto || !t.pmask) {
        orc_free(&t); free(order); return -1;
    }
    for (size_t i = 0; i < m; ++i) {
        const orc_rule* r = order[i];
        t.smask[i] = orc_prefix_mask(r->sip_len);
        t.sval[i] = r->sip & t.smask[i];
        t.dmask[i] = orc_prefix_mask(r->dip_len);
        t.dval[i] = r->dip & t.dmask[i];
        t.splo[i] = r->sp_lo; t.sphi[i] = r->sp_hi;
        t.dplo[i] = r->dp_lo; t.dphi[i] = r->dp_hi;
        t.proto[i] = r->proto; t.pmask[i] = r->proto_mask;
        t.id[i] = r->id;
    }
    free(order);

    if (threads <= 0) threads = 1;
    if ((size_t)threads > n_pkts) threads = n_pkts ? (int)n_pkts : 1;
    pthread_t* th = malloc(sizeof *th * (size_t)threads);
    orc_job* jobs = malloc(sizeof *jobs * (size_t)threads);
    char* threaded = calloc((size_t)threads, 1);
    if (!th || !jobs || !threaded) {
        free(th); free(jobs); free(threaded); orc_free(&t); return -1;
    }
    size_t per = (n_pkts + (size_t)threads - 1) / (size_t)threads;
    for (int w = 0; w < threads; ++w) {
        jobs[w].t = &t; jobs[w].pkts = pkts; jobs[w].out = out; jobs[w].scanned = scanned;
        jobs[w].lo = (size_t)w * per;
        jobs[w].hi = jobs[w].lo + per > n_pkts ? n_pkts : jobs[w].lo + per;
        if (jobs[w].lo >= jobs[w].hi) continue;
        if (threads > 1 && pthread_create(&th[w], NULL, orc_worker, &jobs[w]) == 0)
            threaded[w] = 1;
        else
            orc_worker(&jobs[w]);
    }
    for (int w = 0; w < threads; ++w)
        if (threaded[w]) pthread_join(th[w], NULL);
    free(th); free(jobs); free(threaded); orc_free(&t);
    return 0;
}
