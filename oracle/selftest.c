/*
 * Self-test driver of the CPU oracle, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by the test suite (test infrastructure only).
 *
 * It drives every entry point of skiplist.c -- batches with invalid queries
 * and the reserved key, both bulk loads, export, range search, interception,
 * the structural self-check and its planted faults -- against a brute-force
 * sorted array of pairs, so that the sanitizers see every code path run.
 * Exit status 0 when every answer agreed; the sanitizers abort on a memory or
 * undefined-behaviour error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_list orc_list;
orc_list *orc_create(int32_t max_height, int32_t log2_inv_p, uint64_t seed);
void orc_destroy(orc_list *s);
uint64_t orc_size(const orc_list *s);
int32_t orc_height_rule(uint64_t key, uint64_t seed, int32_t log2_inv_p, int32_t max_height);
int32_t orc_execute_batch(orc_list *s, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals,
                          uint64_t n, uint64_t *out_vals, uint8_t *out_status);
int32_t orc_bulk_load(orc_list *s, const uint64_t *keys, const uint64_t *vals, uint64_t n);
int32_t orc_bulk_load_sorted(orc_list *s, const uint64_t *keys, const uint64_t *vals, uint64_t n);
uint64_t orc_export(const orc_list *s, uint64_t *keys, uint64_t *vals, uint64_t cap);
uint64_t orc_range_batch(const orc_list *s, const uint64_t *lo, const uint64_t *hi, uint64_t n,
                         uint64_t *counts, uint64_t *keys, uint64_t *vals, uint64_t cap);
int32_t orc_interception(const orc_list *s, uint64_t q, uint64_t *key);
int32_t orc_check(const orc_list *s);
int32_t orc_debug_plant(orc_list *s, int32_t kind);
void orc_debug_restore(orc_list *s);

#define KMAX UINT64_MAX
#define CAP 8192

/* brute force: sorted arrays of pairs */
static uint64_t bk[CAP], bv[CAP];
static uint64_t bn;

static uint64_t rng_state;
static uint64_t rnd(void)
{
    /* xorshift64* (Vigna) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * UINT64_C(2685821657736338717);
}

static uint64_t lower(uint64_t k)
{
    uint64_t lo = 0, hi = bn;
    while (lo < hi) {
        const uint64_t m = (lo + hi) / 2;
        if (bk[m] < k) lo = m + 1; else hi = m;
    }
    return lo;
}

static int fail(const char *what, uint64_t a, uint64_t b)
{
    fprintf(stderr, "selftest: %s (%llu, %llu)\n", what, (unsigned long long)a, (unsigned long long)b);
    return 1;
}

static int run(uint64_t seed, int32_t l2p)
{
    const uint64_t hseed = UINT64_C(0x9E3779B97F4A7C15) ^ seed;
    orc_list *s = orc_create(24, l2p, hseed);
    if (!s) return fail("create", 0, 0);
    rng_state = seed * 2 + 1;
    bn = 0;
    /* bulk load with duplicates (last wins) and the reserved key (skipped) */
    enum { NL = 600 };
    uint64_t lk[NL], lv[NL];
    for (int i = 0; i < NL; i++) {
        lk[i] = rnd() % 3000;
        lv[i] = rnd();
    }
    lk[7] = KMAX;
    if (orc_bulk_load(s, lk, lv, NL) != 0) return fail("bulk_load", 0, 0);
    for (int i = 0; i < NL; i++) {
        if (lk[i] == KMAX) continue;
        const uint64_t p = lower(lk[i]);
        if (p < bn && bk[p] == lk[i]) {
            bv[p] = lv[i];
        } else {
            memmove(bk + p + 1, bk + p, (bn - p) * 8);
            memmove(bv + p + 1, bv + p, (bn - p) * 8);
            bk[p] = lk[i];
            bv[p] = lv[i];
            bn++;
        }
    }
    if (orc_size(s) != bn) return fail("size after load", orc_size(s), bn);
    /* batches */
    enum { NB = 1500 };
    uint8_t ops[NB], st[NB];
    uint64_t ks[NB], vs[NB], ov[NB];
    for (int b = 0; b < 6; b++) {
        for (int i = 0; i < NB; i++) {
            const uint64_t r = rnd();
            ops[i] = (uint8_t)(r % 100 < 2 ? 7 : r % 3);
            ks[i] = (r >> 8) % 100 < 1 ? KMAX : rnd() % 4000;
            vs[i] = rnd();
        }
        if (orc_execute_batch(s, ops, ks, vs, NB, ov, st) != 0) return fail("execute", b, 0);
        for (int i = 0; i < NB; i++) {
            if (ops[i] > 2 || ks[i] == KMAX) {
                if (st[i] != 255 || ov[i] != 0) return fail("invalid answer", i, st[i]);
                continue;
            }
            const uint64_t p = lower(ks[i]);
            const int hit = p < bn && bk[p] == ks[i];
            if (st[i] != (hit ? 1 : 0) || ov[i] != (hit ? bv[p] : 0)) return fail("answer", ks[i], st[i]);
            if (ops[i] == 1) {
                if (hit) {
                    bv[p] = vs[i];
                } else {
                    if (bn == CAP) return fail("brute force full", bn, 0);
                    memmove(bk + p + 1, bk + p, (bn - p) * 8);
                    memmove(bv + p + 1, bv + p, (bn - p) * 8);
                    bk[p] = ks[i];
                    bv[p] = vs[i];
                    bn++;
                }
            } else if (ops[i] == 2 && hit) {
                memmove(bk + p, bk + p + 1, (bn - p - 1) * 8);
                memmove(bv + p, bv + p + 1, (bn - p - 1) * 8);
                bn--;
            }
        }
        if (orc_check(s) != 0) return fail("check", b, (uint64_t)orc_check(s));
    }
    /* export */
    static uint64_t ek[CAP], ev[CAP];
    if (orc_export(s, ek, ev, CAP) != bn) return fail("export size", 0, 0);
    for (uint64_t i = 0; i < bn; i++)
        if (ek[i] != bk[i] || ev[i] != bv[i]) return fail("export", i, ek[i]);
    /* ranges, including empty and reversed ones */
    enum { NR = 300 };
    uint64_t lo[NR], hi[NR], cnt[NR];
    for (int i = 0; i < NR; i++) {
        lo[i] = rnd() % 4200;
        hi[i] = i % 17 == 0 ? lo[i] - 1 : lo[i] + rnd() % 200;
    }
    hi[1] = KMAX;
    static uint64_t rk[NR * 256], rv[NR * 256];
    const uint64_t tot = orc_range_batch(s, lo, hi, NR, cnt, rk, rv, NR * 256);
    uint64_t off = 0;
    for (int i = 0; i < NR; i++) {
        uint64_t c = 0;
        for (uint64_t j = lower(lo[i]); lo[i] <= hi[i] && j < bn && bk[j] <= hi[i]; j++, c++)
            if (off + c < NR * 256 && (rk[off + c] != bk[j] || rv[off + c] != bv[j])) return fail("range pair", i, c);
        if (cnt[i] != c) return fail("range count", i, cnt[i]);
        off += c;
    }
    if (off != tot) return fail("range total", off, tot);
    /* interceptions: the largest key of height > 1 that is <= q */
    for (int i = 0; i < 500; i++) {
        const uint64_t q = i == 0 ? KMAX - 1 : rnd() % 4300;
        uint64_t want = 0;
        int have = 0;
        for (uint64_t j = 0; j < bn && bk[j] <= q; j++)
            if (orc_height_rule(bk[j], hseed, l2p, 24) > 1) {
                want = bk[j];
                have = 1;
            }
        uint64_t got = 0;
        if (orc_interception(s, q, &got) != have || (have && got != want)) return fail("interception", q, got);
    }
    /* planted faults are caught with their own codes, and undone */
    for (int32_t kind = 1; kind <= 4; kind++) {
        if (orc_debug_plant(s, kind) != 0) return fail("plant", (uint64_t)kind, 0);
        if (orc_check(s) != kind) return fail("planted fault missed", (uint64_t)kind, (uint64_t)orc_check(s));
        orc_debug_restore(s);
        if (orc_check(s) != 0) return fail("restore", (uint64_t)kind, 0);
    }
    if (orc_debug_plant(s, 2) != 0) return fail("plant before destroy", 0, 0);
    orc_destroy(s); /* destroy restores a planted fault first */
    /* the sorted bulk load gives the same set */
    orc_list *t = orc_create(24, l2p, hseed);
    if (!t || orc_bulk_load_sorted(t, bk, bv, bn) != 0) return fail("bulk_load_sorted", 0, 0);
    if (orc_check(t) != 0 || orc_export(t, ek, ev, CAP) != bn) return fail("sorted load", 0, 0);
    for (uint64_t i = 0; i < bn; i++)
        if (ek[i] != bk[i] || ev[i] != bv[i]) return fail("sorted export", i, 0);
    orc_destroy(t);
    return 0;
}

int main(void)
{
    for (uint64_t seed = 1; seed <= 6; seed++)
        if (run(seed, seed % 2 ? 1 : 2)) return 1;
    puts("selftest ok");
    return 0;
}
