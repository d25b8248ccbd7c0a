/*
 * ac_oracle.c -- plain single-threaded Aho-Corasick.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the GPU scan is checked
 * against.  Only the tests, the smoke entry point and the benchmark's CPU
 * baseline may load it; the product library never calls it and shares no
 * code, header or table with it.
 *
 * It follows the paper's description of Aho-Corasick (section III.A,
 * Figures 1 and 2) in the paper's own terms:
 *
 *   Stage 1 builds the string-matching machine from the keywords:
 *     - the goto function g: a keyword trie; states are numbered 0, 1, 2, ...
 *       in the order they are created while the keywords are inserted in
 *       input order (with keywords HIS, HERS, SHE inserted in that order this
 *       reproduces the state numbers of the paper's Figure 2 walk);
 *       g(0, a) = 0 for every symbol a that leaves the root on no edge;
 *     - the failure function f, computed breadth first: depth-1 states fail
 *       to the root (the paper's Figure 1 leaves those edges out), and for a
 *       child s = g(r, a) one follows failure links from f(r) until a state
 *       t with g(t, a) defined is found, then f(s) = g(t, a);
 *     - the output function: out(s) = the keywords ending at s together with
 *       out(f(s)), so overlapping keywords are all reported (the paper's
 *       SHE / HERS example in "SHERS").
 *   Stage 2 reads the text once: for each symbol, while g(s, a) is undefined
 *   take the failure transition and read the same symbol again, then move to
 *   g(s, a) and report every keyword in out(s) with the current position.
 *
 * Conventions (the paper does not fix them):
 *   - a pattern's id is its 0-based index in the input list; duplicates each
 *     keep their own id and are all reported;
 *   - a match is reported at the 0-based index of its last symbol ("end");
 *   - out(s) is kept sorted by id, so matches come out ordered by (end, id);
 *   - an empty pattern or a symbol >= sigma is rejected.
 *
 * The representation is deliberately the paper's partial goto function plus
 * failure links (not a completed transition table).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_EMPTY (-2)
#define OR_E_SYMBOL (-3)
#define OR_E_NOMEM (-5)

typedef struct {
    uint32_t *ids;
    uint32_t len, cap;
} idlist;

typedef struct {
    uint32_t sigma;
    uint32_t n_states, cap_states;
    int32_t *go;      /* go[s*sigma + a]: g(s,a), -1 = undefined */
    int32_t *fail;    /* f(s) */
    uint32_t *depth;  /* length of the string spelled by s */
    idlist *out;      /* out(s), sorted by pattern id */
} oracle_machine;

static int push_id(idlist *l, uint32_t id) {
    if (l->len == l->cap) {
        uint32_t nc = l->cap ? 2 * l->cap : 2;
        uint32_t *p = (uint32_t *)realloc(l->ids, (size_t)nc * sizeof(uint32_t));
        if (!p) return OR_E_NOMEM;
        l->ids = p;
        l->cap = nc;
    }
    l->ids[l->len++] = id;
    return OR_OK;
}

static int new_state(oracle_machine *m, uint32_t depth) {
    if (m->n_states == m->cap_states) {
        uint32_t nc = m->cap_states ? 2 * m->cap_states : 64;
        int32_t *g = (int32_t *)realloc(m->go, (size_t)nc * m->sigma * sizeof(int32_t));
        if (!g) return -1;
        m->go = g;
        int32_t *f = (int32_t *)realloc(m->fail, (size_t)nc * sizeof(int32_t));
        if (!f) return -1;
        m->fail = f;
        uint32_t *d = (uint32_t *)realloc(m->depth, (size_t)nc * sizeof(uint32_t));
        if (!d) return -1;
        m->depth = d;
        idlist *o = (idlist *)realloc(m->out, (size_t)nc * sizeof(idlist));
        if (!o) return -1;
        m->out = o;
        m->cap_states = nc;
    }
    uint32_t s = m->n_states++;
    for (uint32_t a = 0; a < m->sigma; ++a) m->go[(size_t)s * m->sigma + a] = -1;
    m->fail[s] = 0;
    m->depth[s] = depth;
    m->out[s].ids = NULL;
    m->out[s].len = m->out[s].cap = 0;
    return (int)s;
}

void oracle_free(oracle_machine *m) {
    if (!m) return;
    if (m->out)
        for (uint32_t s = 0; s < m->n_states; ++s) free(m->out[s].ids);
    free(m->out);
    free(m->go);
    free(m->fail);
    free(m->depth);
    free(m);
}

/* Stage 1.  Pattern i = sym[off[i] .. off[i+1]). */
int oracle_build(const uint8_t *sym, const uint64_t *off, uint32_t n_patterns,
                 uint32_t sigma, oracle_machine **out) {
    if (!out || !off || sigma == 0 || sigma > 256) return OR_E_INVALID;
    *out = NULL;
    if (n_patterns == 0) return OR_E_INVALID;
    for (uint32_t i = 0; i < n_patterns; ++i) {
        if (off[i + 1] <= off[i]) return OR_E_EMPTY;
        for (uint64_t k = off[i]; k < off[i + 1]; ++k)
            if (sym[k] >= sigma) return OR_E_SYMBOL;
    }
    oracle_machine *m = (oracle_machine *)calloc(1, sizeof(oracle_machine));
    if (!m) return OR_E_NOMEM;
    m->sigma = sigma;
    if (new_state(m, 0) != 0) { oracle_free(m); return OR_E_NOMEM; }

    /* goto function: insert every keyword, creating states as needed */
    for (uint32_t i = 0; i < n_patterns; ++i) {
        int32_t s = 0;
        for (uint64_t k = off[i]; k < off[i + 1]; ++k) {
            uint8_t a = sym[k];
            int32_t t = m->go[(size_t)s * sigma + a];
            if (t < 0) {
                t = new_state(m, m->depth[s] + 1);
                if (t < 0) { oracle_free(m); return OR_E_NOMEM; }
                m->go[(size_t)s * sigma + a] = t;
            }
            s = t;
        }
        if (push_id(&m->out[s], i) != OR_OK) { oracle_free(m); return OR_E_NOMEM; }
    }
    /* the root loops to itself on every symbol it has no edge for */
    for (uint32_t a = 0; a < sigma; ++a)
        if (m->go[a] < 0) m->go[a] = 0;

    /* failure and output functions, breadth first from the root */
    int32_t *queue = (int32_t *)malloc((size_t)m->n_states * sizeof(int32_t));
    if (!queue) { oracle_free(m); return OR_E_NOMEM; }
    size_t head = 0, tail = 0;
    for (uint32_t a = 0; a < sigma; ++a) {
        int32_t s = m->go[a];
        if (s != 0) {
            m->fail[s] = 0;
            queue[tail++] = s;
        }
    }
    while (head < tail) {
        int32_t r = queue[head++];
        for (uint32_t a = 0; a < sigma; ++a) {
            int32_t s = m->go[(size_t)r * sigma + a];
            if (s < 0) continue;
            queue[tail++] = s;
            int32_t t = m->fail[r];
            while (m->go[(size_t)t * sigma + a] < 0) t = m->fail[t];
            m->fail[s] = m->go[(size_t)t * sigma + a];
        }
    }
    /* out(s) = own(s) merged with out(f(s)); f(s) is shallower, so it is
       complete when states are visited in breadth-first order */
    for (size_t q = 0; q < tail; ++q) {
        int32_t s = queue[q];
        idlist *own = &m->out[s];
        const idlist *inh = &m->out[m->fail[s]];
        if (inh->len == 0) continue;
        idlist merged = {NULL, 0, 0};
        uint32_t x = 0, y = 0;
        while (x < own->len || y < inh->len) {
            uint32_t v;
            if (y >= inh->len || (x < own->len && own->ids[x] < inh->ids[y]))
                v = own->ids[x++];
            else
                v = inh->ids[y++];
            if (push_id(&merged, v) != OR_OK) {
                free(merged.ids);
                free(queue);
                oracle_free(m);
                return OR_E_NOMEM;
            }
        }
        free(own->ids);
        *own = merged;
    }
    free(queue);
    *out = m;
    return OR_OK;
}

/* Stage 2.  Writes up to cap matches (pid[k], end[k]) in (end, pid) order
   and returns the total number of matches. */
int64_t oracle_scan(const oracle_machine *m, const uint8_t *text, uint64_t n,
                    uint32_t *pid, uint32_t *end, uint64_t cap) {
    if (!m) return OR_E_INVALID;
    const uint32_t sigma = m->sigma;
    int64_t total = 0;
    int32_t s = 0;
    for (uint64_t e = 0; e < n; ++e) {
        uint8_t a = text[e];
        if (a >= sigma) return OR_E_SYMBOL;
        while (m->go[(size_t)s * sigma + a] < 0) s = m->fail[s];
        s = m->go[(size_t)s * sigma + a];
        const idlist *o = &m->out[s];
        for (uint32_t k = 0; k < o->len; ++k) {
            if ((uint64_t)total < cap) {
                pid[total] = o->ids[k];
                end[total] = (uint32_t)e;
            }
            ++total;
        }
    }
    return total;
}

/* Per-pattern occurrence counts (counts has n_patterns entries, zeroed here). */
int oracle_count(const oracle_machine *m, const uint8_t *text, uint64_t n,
                 uint64_t *counts, uint32_t n_patterns) {
    if (!m) return OR_E_INVALID;
    memset(counts, 0, (size_t)n_patterns * sizeof(uint64_t));
    const uint32_t sigma = m->sigma;
    int32_t s = 0;
    for (uint64_t e = 0; e < n; ++e) {
        uint8_t a = text[e];
        if (a >= sigma) return OR_E_SYMBOL;
        while (m->go[(size_t)s * sigma + a] < 0) s = m->fail[s];
        s = m->go[(size_t)s * sigma + a];
        const idlist *o = &m->out[s];
        for (uint32_t k = 0; k < o->len; ++k) counts[o->ids[k]]++;
    }
    return OR_OK;
}

/* The sequence of moves the machine makes on the text: state[k] is the
   state entered by move k and kind[k] is 'g' (goto) or 'f' (failure).
   Returns the number of moves (writes at most cap). */
int64_t oracle_trace(const oracle_machine *m, const uint8_t *text, uint64_t n,
                     int32_t *state, uint8_t *kind, uint64_t cap) {
    if (!m) return OR_E_INVALID;
    const uint32_t sigma = m->sigma;
    int64_t k = 0;
    int32_t s = 0;
    for (uint64_t e = 0; e < n; ++e) {
        uint8_t a = text[e];
        if (a >= sigma) return OR_E_SYMBOL;
        while (m->go[(size_t)s * sigma + a] < 0) {
            s = m->fail[s];
            if ((uint64_t)k < cap) { state[k] = s; kind[k] = 'f'; }
            ++k;
        }
        s = m->go[(size_t)s * sigma + a];
        if ((uint64_t)k < cap) { state[k] = s; kind[k] = 'g'; }
        ++k;
    }
    return k;
}

/* Accessors used by the tests to pin the machine itself. */
uint32_t oracle_num_states(const oracle_machine *m) { return m ? m->n_states : 0; }
int32_t oracle_goto(const oracle_machine *m, uint32_t s, uint32_t a) {
    return (m && s < m->n_states && a < m->sigma) ? m->go[(size_t)s * m->sigma + a] : -2;
}
int32_t oracle_fail(const oracle_machine *m, uint32_t s) {
    return (m && s < m->n_states) ? m->fail[s] : -2;
}
uint32_t oracle_depth(const oracle_machine *m, uint32_t s) {
    return (m && s < m->n_states) ? m->depth[s] : 0;
}
/* Copies up to cap ids of out(s); returns |out(s)|. */
int64_t oracle_output(const oracle_machine *m, uint32_t s, uint32_t *ids, uint64_t cap) {
    if (!m || s >= m->n_states) return OR_E_INVALID;
    const idlist *o = &m->out[s];
    for (uint32_t k = 0; k < o->len && k < cap; ++k) ids[k] = o->ids[k];
    return o->len;
}
