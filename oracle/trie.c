/*
 * Binary-trie longest-prefix match -- TEST ORACLE, not product code.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no code with the GPU library.
 *
 * The textbook one-bit-per-level trie: a rule (P, L, nh) is stored at the
 * node reached by walking the top L bits of P from the most significant bit;
 * a lookup walks the address's bits from the MSB and remembers the last next
 * hop it passed.  That is the definition of longest-prefix match (the rule
 * with the longest matching prefix wins, L = 0 matches every address) with no
 * other arithmetic.  Uncovered addresses get NO_ROUTE = 0xFFFF.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NO_ROUTE 0xFFFFu

typedef struct {
    int32_t child[2];
    int32_t nh; /* -1: no rule ends here */
} otnode;

typedef struct {
    otnode* nodes;
    size_t n, cap;
} otrie;

static int bit_at(uint64_t hi, uint64_t lo, int i) /* i = 0 is the MSB */
{
    return i < 64 ? (int)((hi >> (63 - i)) & 1u) : (int)((lo >> (127 - i)) & 1u);
}

static int32_t new_node(otrie* t)
{
    if (t->n == t->cap) {
        size_t cap = t->cap ? t->cap * 2 : 1024;
        otnode* p = (otnode*)realloc(t->nodes, cap * sizeof(otnode));
        if (!p) return -1;
        t->nodes = p;
        t->cap = cap;
    }
    t->nodes[t->n].child[0] = t->nodes[t->n].child[1] = -1;
    t->nodes[t->n].nh = -1;
    return (int32_t)t->n++;
}

void oracle_trie_free(otrie* t)
{
    if (!t) return;
    free(t->nodes);
    free(t);
}

/* prefixes: n records {hi, lo}; returns NULL on a bad length or no memory.
 * A rule given twice keeps the later next hop (inputs are unique anyway). */
otrie* oracle_trie_new(const uint64_t* prefixes, const uint8_t* lengths,
                       const uint16_t* next_hops, size_t n)
{
    otrie* t = (otrie*)calloc(1, sizeof(otrie));
    if (!t || new_node(t) < 0) { oracle_trie_free(t); return NULL; }
    for (size_t r = 0; r < n; ++r) {
        int L = lengths[r];
        if (L > 128) { oracle_trie_free(t); return NULL; }
        uint64_t hi = prefixes[2 * r], lo = prefixes[2 * r + 1];
        int32_t cur = 0;
        for (int i = 0; i < L; ++i) {
            int b = bit_at(hi, lo, i);
            int32_t nx = t->nodes[cur].child[b];
            if (nx < 0) {
                nx = new_node(t);
                if (nx < 0) { oracle_trie_free(t); return NULL; }
                t->nodes[cur].child[b] = nx;
            }
            cur = nx;
        }
        t->nodes[cur].nh = next_hops[r];
    }
    return t;
}

size_t oracle_trie_nodes(const otrie* t) { return t ? t->n : 0; }

static uint16_t lookup_one(const otrie* t, uint64_t hi, uint64_t lo)
{
    const otnode* nd = t->nodes;
    uint16_t best = nd[0].nh >= 0 ? (uint16_t)nd[0].nh : (uint16_t)ORACLE_NO_ROUTE;
    int32_t cur = 0;
    for (int i = 0; i < 128; ++i) {
        int32_t nx = nd[cur].child[bit_at(hi, lo, i)];
        if (nx < 0) break;
        cur = nx;
        if (nd[cur].nh >= 0) best = (uint16_t)nd[cur].nh;
    }
    return best;
}

typedef struct {
    const otrie* t;
    const uint64_t* addrs;
    uint16_t* out;
    size_t b, e;
} job;

static void* run(void* arg)
{
    job* j = (job*)arg;
    for (size_t i = j->b; i < j->e; ++i)
        j->out[i] = lookup_one(j->t, j->addrs[2 * i], j->addrs[2 * i + 1]);
    return NULL;
}

/* addrs: q records {hi, lo}; out: q next hops.  Returns 0, or -1 on error. */
int oracle_trie_lookup(const otrie* t, const uint64_t* addrs, size_t q,
                       uint16_t* out, int nthreads)
{
    if (!t) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((size_t)nthreads > q) nthreads = q ? (int)q : 1;
    pthread_t th[256];
    job jobs[256];
    size_t per = (q + (size_t)nthreads - 1) / (size_t)nthreads;
    int spawned[256];
    for (int k = 0; k < nthreads; ++k) {
        spawned[k] = 0;
        size_t b = (size_t)k * per, e = b + per;
        if (b > q) b = q;
        if (e > q) e = q;
        jobs[k].t = t; jobs[k].addrs = addrs; jobs[k].out = out;
        jobs[k].b = b; jobs[k].e = e;
        if (k == nthreads - 1 || pthread_create(&th[k], NULL, run, &jobs[k]) != 0) {
            run(&jobs[k]); /* last chunk (or a failed spawn) runs here */
        } else {
            spawned[k] = 1;
        }
    }
    for (int k = 0; k < nthreads; ++k)
        if (spawned[k]) pthread_join(th[k], NULL);
    return 0;
}
