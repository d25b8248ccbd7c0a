/*
 * naive.c -- checkers that pin the Aho-Corasick oracle without using it.
 *
 * TEST INFRASTRUCTURE ONLY (see ac_oracle.c).  Neither function here knows
 * about automata:
 *
 *   naive_scan   the definition of the result, written out: for every end
 *                position e and every pattern i (in that order), report
 *                (i, e) when the |p_i| symbols ending at e equal p_i.  This
 *                is the set of all occurrences the paper's single-pass
 *                matcher must report (sections I and III.A), in (end, id)
 *                order.  O(n * total pattern length): tiny inputs only.
 *
 *   kmer_count   per-pattern occurrence counts by hashing: for each distinct
 *                pattern length L, a rolling base-sigma code of the last L
 *                symbols is looked up in a hash table of pattern codes.  An
 *                independent exact method that runs at full workload sizes
 *                (sigma^L must fit in 64 bits: L <= 31 for DNA, 14 for a
 *                20-letter alphabet).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t naive_scan(const uint8_t *text, uint64_t n, const uint8_t *sym,
                   const uint64_t *off, uint32_t n_patterns,
                   uint32_t *pid, uint32_t *end, uint64_t cap) {
    int64_t total = 0;
    for (uint64_t e = 0; e < n; ++e) {
        for (uint32_t i = 0; i < n_patterns; ++i) {
            uint64_t L = off[i + 1] - off[i];
            if (L == 0 || L > e + 1) continue;
            if (memcmp(text + (e + 1 - L), sym + off[i], (size_t)L) == 0) {
                if ((uint64_t)total < cap) {
                    pid[total] = i;
                    end[total] = (uint32_t)e;
                }
                ++total;
            }
        }
    }
    return total;
}

typedef struct {
    uint64_t code;
    uint32_t first; /* index into the chain array */
    uint32_t used;
} slot;

static uint64_t mix(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

/* counts[i] = number of end positions e with text[e-L+1..e] == p_i. */
int kmer_count(const uint8_t *text, uint64_t n, const uint8_t *sym,
               const uint64_t *off, uint32_t n_patterns, uint32_t sigma,
               uint64_t *counts) {
    memset(counts, 0, (size_t)n_patterns * sizeof(uint64_t));
    uint64_t maxL = 0;
    for (uint32_t i = 0; i < n_patterns; ++i) {
        uint64_t L = off[i + 1] - off[i];
        if (L > maxL) maxL = L;
    }
    /* next[i]: next pattern with the same (length, code), chained per slot */
    uint32_t *next = (uint32_t *)malloc((size_t)n_patterns * sizeof(uint32_t) + 4);
    if (!next) return -5;
    for (uint64_t L = 1; L <= maxL; ++L) {
        uint32_t members = 0;
        for (uint32_t i = 0; i < n_patterns; ++i)
            if (off[i + 1] - off[i] == L) ++members;
        if (!members) continue;
        /* sigma^L must not overflow: check by repeated multiplication */
        uint64_t top = 1; /* sigma^(L-1) */
        for (uint64_t k = 1; k < L; ++k) {
            if (top > UINT64_MAX / sigma / sigma) { free(next); return -4; }
            top *= sigma;
        }
        uint64_t nslots = 1;
        while (nslots < 2ULL * members) nslots <<= 1;
        slot *tab = (slot *)calloc((size_t)nslots, sizeof(slot));
        if (!tab) { free(next); return -5; }
        for (uint32_t i = 0; i < n_patterns; ++i) {
            if (off[i + 1] - off[i] != L) continue;
            uint64_t c = 0;
            for (uint64_t k = off[i]; k < off[i + 1]; ++k) c = c * sigma + sym[k];
            uint64_t h = mix(c) & (nslots - 1);
            while (tab[h].used && tab[h].code != c) h = (h + 1) & (nslots - 1);
            if (!tab[h].used) {
                tab[h].used = 1;
                tab[h].code = c;
                tab[h].first = i;
                next[i] = UINT32_MAX;
            } else {
                /* append to keep the chain in id order (not needed for counts) */
                uint32_t j = tab[h].first;
                while (next[j] != UINT32_MAX) j = next[j];
                next[j] = i;
                next[i] = UINT32_MAX;
            }
        }
        if (n >= L) {
            uint64_t c = 0;
            for (uint64_t e = 0; e < n; ++e) {
                if (e >= L) c -= (uint64_t)text[e - L] * top;
                c = c * sigma + text[e];
                if (e + 1 < L) continue;
                uint64_t h = mix(c) & (nslots - 1);
                while (tab[h].used && tab[h].code != c) h = (h + 1) & (nslots - 1);
                if (tab[h].used)
                    for (uint32_t j = tab[h].first; j != UINT32_MAX; j = next[j]) counts[j]++;
            }
        }
        free(tab);
    }
    free(next);
    return 0;
}
