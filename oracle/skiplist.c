/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, single-threaded Pugh skip list (the classic structure the paper
 * builds on, Section 1 and Section 2) that applies every query of a batch in
 * arrival order.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library; the GPU library never links it and
 * the two share no source.
 *
 * What it computes (paper Section 3.2, query semantics, and Definitions 1-2):
 *   the index is a finite map from uint64 keys to uint64 values;
 *   SEARCH k  -> (PRESENT, m[k]) if k is in the map, else (ABSENT, 0);
 *   INSERT k v-> same answer as SEARCH, then m[k] = v;
 *   DELETE k  -> same answer as SEARCH, then k leaves the map;
 *   a query whose op is not 0/1/2 or whose key is 2^64-1 -> (INVALID, 0)
 *   and no effect.
 * The answers of INSERT and DELETE are a reading: the paper returns 1/null
 * for delete and nothing for insert; returning the previous value pins more.
 *
 * Tower heights (paper Section 3.2: the height of a new node is drawn from a
 * geometric distribution) follow a deterministic rule so that any two
 * implementations agree without sharing random state:
 *   z = key XOR seed, then the splitmix64 output finalizer (Steele, Lea and
 *   Flood, OOPSLA 2014; Vigna's public-domain splitmix64),
 *   height = 1 + min(ctz(z) / log2_inv_p, max_height - 1), ctz(0) = 64.
 * so P(height >= h) = p^(h-1) with p = 2^-log2_inv_p.
 *
 * A test hook lets a caller force the height of an inserted key; it exists
 * only to reproduce hand-worked examples whose heights are given.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_MAX_LEVELS 64

enum { ORC_SEARCH = 0, ORC_INSERT = 1, ORC_DELETE = 2 };
enum { ORC_ABSENT = 0, ORC_PRESENT = 1, ORC_INVALID = 255 };

typedef struct orc_node {
    uint64_t key;
    uint64_t val;
    int32_t height;
    struct orc_node *fwd[]; /* fwd[0] is the storage-level successor */
} orc_node;

typedef struct orc_list {
    orc_node *head; /* sentinel, key -infinity, max_height forward pointers */
    int32_t max_height;
    int32_t log2_inv_p;
    uint64_t seed;
    uint64_t size;
    int32_t forced_height; /* 0 = use the rule; test hook */
    /* a planted structural fault (test hook, see orc_debug_plant) */
    int32_t plant;
    orc_node *pa, *pb;
} orc_list;

/* ---------------------------------------------------------------- heights */

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);
    z = (z ^ (z >> 27)) * UINT64_C(0x94D049BB133111EB);
    return z ^ (z >> 31);
}

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

int32_t orc_height_rule(uint64_t key, uint64_t seed, int32_t log2_inv_p,
                        int32_t max_height)
{
    uint64_t z = mix64(key ^ seed);
    int32_t tz = 0;
    if (z == 0) {
        tz = 64;
    } else {
        while (((z >> tz) & 1u) == 0) tz++;
    }
    int32_t extra = tz / log2_inv_p;
    if (extra > max_height - 1) extra = max_height - 1;
    return 1 + extra;
}

static int32_t node_height(const orc_list *s, uint64_t key)
{
    if (s->forced_height > 0) return s->forced_height;
    return orc_height_rule(key, s->seed, s->log2_inv_p, s->max_height);
}

/* ------------------------------------------------------------- life cycle */

static orc_node *new_node(int32_t h, uint64_t key, uint64_t val)
{
    orc_node *n = (orc_node *)malloc(sizeof(orc_node) + (size_t)h * sizeof(orc_node *));
    if (!n) return NULL;
    n->key = key;
    n->val = val;
    n->height = h;
    for (int32_t i = 0; i < h; i++) n->fwd[i] = NULL;
    return n;
}

orc_list *orc_create(int32_t max_height, int32_t log2_inv_p, uint64_t seed)
{
    if (max_height < 1 || max_height > ORC_MAX_LEVELS || log2_inv_p < 1 || log2_inv_p > 32)
        return NULL;
    orc_list *s = (orc_list *)calloc(1, sizeof(orc_list));
    if (!s) return NULL;
    s->max_height = max_height;
    s->log2_inv_p = log2_inv_p;
    s->seed = seed;
    s->head = new_node(max_height, 0, 0);
    if (!s->head) {
        free(s);
        return NULL;
    }
    return s;
}

void orc_debug_restore(orc_list *s);

void orc_destroy(orc_list *s)
{
    if (!s) return;
    if (s->plant) orc_debug_restore(s);
    orc_node *n = s->head->fwd[0];
    while (n) {
        orc_node *nx = n->fwd[0];
        free(n);
        n = nx;
    }
    free(s->head);
    free(s);
}

void orc_force_height(orc_list *s, int32_t h) { s->forced_height = h; }

uint64_t orc_size(const orc_list *s) { return s->size; }

/* ------------------------------------------------------------ the descent */

/* Standard Pugh descent: on every level advance while the successor's key is
 * smaller than k; update[l] is the last node visited on level l.  Returns the
 * level-0 successor of update[0] (the only candidate equal to k). */
static orc_node *descend(const orc_list *s, uint64_t k, orc_node **update)
{
    orc_node *x = s->head;
    for (int32_t l = s->max_height - 1; l >= 0; l--) {
        while (x->fwd[l] && x->fwd[l]->key < k) x = x->fwd[l];
        if (update) update[l] = x;
    }
    return x->fwd[0];
}

int32_t orc_find(const orc_list *s, uint64_t k, uint64_t *val)
{
    orc_node *n = descend(s, k, NULL);
    if (n && n->key == k) {
        if (val) *val = n->val;
        return 1;
    }
    if (val) *val = 0;
    return 0;
}

/* Returns 1 and the previous value when k was present (value replaced),
 * 0 when a new node was spliced in, -1 on allocation failure. */
int32_t orc_insert(orc_list *s, uint64_t k, uint64_t v, uint64_t *old)
{
    orc_node *update[ORC_MAX_LEVELS];
    orc_node *n = descend(s, k, update);
    if (n && n->key == k) {
        if (old) *old = n->val;
        n->val = v;
        return 1;
    }
    int32_t h = node_height(s, k);
    orc_node *m = new_node(h, k, v);
    if (!m) return -1;
    for (int32_t l = 0; l < h; l++) {
        m->fwd[l] = update[l]->fwd[l];
        update[l]->fwd[l] = m;
    }
    s->size++;
    if (old) *old = 0;
    return 0;
}

/* Returns 1 and the removed value when k was present, else 0. */
int32_t orc_erase(orc_list *s, uint64_t k, uint64_t *old)
{
    orc_node *update[ORC_MAX_LEVELS];
    orc_node *n = descend(s, k, update);
    if (!(n && n->key == k)) {
        if (old) *old = 0;
        return 0;
    }
    for (int32_t l = 0; l < n->height; l++) update[l]->fwd[l] = n->fwd[l];
    if (old) *old = n->val;
    free(n);
    s->size--;
    return 1;
}

/* ------------------------------------------------------------ batch level */

/* Applies n queries in arrival order (the serial execution that the paper's
 * batched processing must reproduce, Section 3.2.4).  out_vals/out_status
 * receive one answer per query.  Returns 0, or -1 on allocation failure. */
int32_t orc_execute_batch(orc_list *s, const uint8_t *ops, const uint64_t *keys,
                          const uint64_t *vals, uint64_t n, uint64_t *out_vals,
                          uint8_t *out_status)
{
    for (uint64_t i = 0; i < n; i++) {
        uint8_t op = ops[i];
        uint64_t k = keys[i];
        uint64_t prev = 0;
        int32_t hit;
        if (op > ORC_DELETE || k == UINT64_MAX) {
            out_vals[i] = 0;
            out_status[i] = ORC_INVALID;
            continue;
        }
        if (op == ORC_SEARCH) {
            hit = orc_find(s, k, &prev);
        } else if (op == ORC_INSERT) {
            hit = orc_insert(s, k, vals[i], &prev);
            if (hit < 0) return -1;
        } else {
            hit = orc_erase(s, k, &prev);
        }
        out_vals[i] = hit ? prev : 0;
        out_status[i] = hit ? ORC_PRESENT : ORC_ABSENT;
    }
    return 0;
}

/* Bulk load = inserting the pairs in array order into an empty list, so the
 * last occurrence of a duplicated key wins.  Returns 0, -1 on allocation
 * failure, -2 if the list is not empty. */
/* orc_execute_batch timed with the monotonic clock around the whole loop
 * (the CPU baseline of the benchmark): *elapsed_ns receives the time. */
int32_t orc_execute_batch_timed(orc_list *s, const uint8_t *ops, const uint64_t *keys, const uint64_t *vals,
                                uint64_t n, uint64_t *out_vals, uint8_t *out_status, uint64_t *elapsed_ns)
{
    struct timespec a, b;
    clock_gettime(CLOCK_MONOTONIC, &a);
    const int32_t r = orc_execute_batch(s, ops, keys, vals, n, out_vals, out_status);
    clock_gettime(CLOCK_MONOTONIC, &b);
    *elapsed_ns = (uint64_t)(b.tv_sec - a.tv_sec) * UINT64_C(1000000000) + (uint64_t)b.tv_nsec - (uint64_t)a.tv_nsec;
    return r;
}

int32_t orc_bulk_load(orc_list *s, const uint64_t *keys, const uint64_t *vals, uint64_t n)
{
    if (s->size != 0) return -2;
    for (uint64_t i = 0; i < n; i++) {
        if (keys[i] == UINT64_MAX) continue;
        if (orc_insert(s, keys[i], vals[i], NULL) < 0) return -1;
    }
    return 0;
}

/* Faster bulk path for large inputs whose keys are already strictly
 * increasing (the caller sorted and de-duplicated them): nodes are appended
 * at the tail of every level they reach.  The structure is the same one the
 * sequential inserts build, because heights depend only on the key.
 * Returns 0, -1 on allocation failure, -2 if not empty, -3 if not sorted. */
int32_t orc_bulk_load_sorted(orc_list *s, const uint64_t *keys, const uint64_t *vals,
                             uint64_t n)
{
    if (s->size != 0) return -2;
    orc_node *tail[ORC_MAX_LEVELS];
    for (int32_t l = 0; l < s->max_height; l++) tail[l] = s->head;
    for (uint64_t i = 0; i < n; i++) {
        if (keys[i] == UINT64_MAX) return -3;
        if (i > 0 && keys[i] <= keys[i - 1]) return -3;
        int32_t h = node_height(s, keys[i]);
        orc_node *m = new_node(h, keys[i], vals[i]);
        if (!m) return -1;
        for (int32_t l = 0; l < h; l++) {
            tail[l]->fwd[l] = m;
            tail[l] = m;
        }
        s->size++;
    }
    return 0;
}

/* Writes the map in key order (a walk of the storage level).  Returns the
 * number of pairs written (at most cap). */
uint64_t orc_export(const orc_list *s, uint64_t *keys, uint64_t *vals, uint64_t cap)
{
    uint64_t i = 0;
    for (orc_node *n = s->head->fwd[0]; n && i < cap; n = n->fwd[0], i++) {
        keys[i] = n->key;
        vals[i] = n->val;
    }
    return i;
}

/* Range search (the paper's range query of Section 3.2.5, SEARCH only): the
 * pairs with lo <= key <= hi, in key order -- the descent to the first key
 * >= lo, then the storage-level walk until a key passes hi.  Writes at most
 * cap of them and returns how many there are (none when lo > hi). */
uint64_t orc_range(const orc_list *s, uint64_t lo, uint64_t hi, uint64_t *keys, uint64_t *vals, uint64_t cap)
{
    uint64_t c = 0;
    if (lo > hi) return 0;
    for (orc_node *n = descend(s, lo, NULL); n && n->key <= hi; n = n->fwd[0], c++) {
        if (c < cap) {
            keys[c] = n->key;
            vals[c] = n->val;
        }
    }
    return c;
}

/* n range searches: counts[i] = size of range i; the results of all ranges
 * are concatenated in range order into keys/vals (at most cap pairs in
 * total).  Returns the total. */
uint64_t orc_range_batch(const orc_list *s, const uint64_t *lo, const uint64_t *hi, uint64_t n,
                         uint64_t *counts, uint64_t *keys, uint64_t *vals, uint64_t cap)
{
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; i++) {
        const uint64_t room = (keys && vals && total < cap) ? cap - total : 0;
        const uint64_t c = orc_range(s, lo[i], hi[i], room ? keys + total : NULL, room ? vals + total : NULL, room);
        counts[i] = c;
        total += c;
    }
    return total;
}

/* Number of keys present on level l (1-based: level 1 is the storage level). */
uint64_t orc_level_count(const orc_list *s, int32_t level)
{
    if (level < 1 || level > s->max_height) return 0;
    uint64_t c = 0;
    for (orc_node *n = s->head->fwd[level - 1]; n; n = n->fwd[level - 1]) c++;
    return c;
}

uint64_t orc_level_keys(const orc_list *s, int32_t level, uint64_t *out, uint64_t cap)
{
    if (level < 1 || level > s->max_height) return 0;
    uint64_t c = 0;
    for (orc_node *n = s->head->fwd[level - 1]; n && c < cap; n = n->fwd[level - 1]) out[c++] = n->key;
    return c;
}

/* Interception (Definition 4): the node with the largest key among those of
 * height > 1 whose key is <= q.  Found by descending to level 2 and taking
 * the last node visited there.  Returns 1 and its key, or 0 when no such node
 * exists (the descent ends at the head). */
int32_t orc_interception(const orc_list *s, uint64_t q, uint64_t *key)
{
    orc_node *x = s->head;
    for (int32_t l = s->max_height - 1; l >= 1; l--)
        while (x->fwd[l] && x->fwd[l]->key <= q) x = x->fwd[l];
    if (x == s->head) {
        if (key) *key = 0;
        return 0;
    }
    if (key) *key = x->key;
    return 1;
}

/* Structural self-check.  Returns 0 when every invariant holds:
 *   1 a level is not strictly increasing;
 *   2 a node on level l is missing from level l-1;
 *   3 a node's height differs from the height rule (unless forced);
 *   4 the level-1 count differs from size;
 *   5 a node's forward pointer on a level at or above its height is set. */
int32_t orc_check(const orc_list *s)
{
    uint64_t cnt = 0;
    for (orc_node *n = s->head->fwd[0]; n; n = n->fwd[0]) {
        if (n->fwd[0] && !(n->key < n->fwd[0]->key)) return 1;
        if (s->forced_height == 0 &&
            n->height != orc_height_rule(n->key, s->seed, s->log2_inv_p, s->max_height))
            return 3;
        cnt++;
    }
    if (cnt != s->size) return 4;
    for (int32_t l = 1; l < s->max_height; l++) {
        orc_node *below = s->head->fwd[l - 1];
        for (orc_node *n = s->head->fwd[l]; n; n = n->fwd[l]) {
            if (n->height <= l) return 5;
            if (n->fwd[l] && !(n->key < n->fwd[l]->key)) return 1;
            while (below && below->key < n->key) below = below->fwd[l - 1];
            if (below != n) return 2;
        }
    }
    return 0;
}

/* ------------------------------------------------------------ test hooks */

/* Plants one structural fault so that the tests can show orc_check rejects
 * it (test infrastructure only); orc_debug_restore undoes it:
 *   1  two adjacent nodes of height 1 swap keys: level 1 is out of order
 *      (check code 1)
 *   2  the first node of height >= 2 is unlinked from level 1 only, the size
 *      adjusted: a level-2 key is missing one level below (code 2)
 *   3  the recorded height of the first height-1 node is raised by one: it
 *      differs from the height rule (code 3)
 *   4  the size is off by one (code 4)
 * Returns 0 when planted, -1 when no node fits or a fault is already
 * planted. */
int32_t orc_debug_plant(orc_list *s, int32_t kind)
{
    if (s->plant) return -1;
    orc_node *prev = s->head;
    for (orc_node *n = s->head->fwd[0]; n; prev = n, n = n->fwd[0]) {
        if (kind == 1 && n->height == 1 && n->fwd[0] && n->fwd[0]->height == 1) {
            const uint64_t k = n->key;
            n->key = n->fwd[0]->key;
            n->fwd[0]->key = k;
            s->pa = n;
            s->plant = 1;
            return 0;
        }
        if (kind == 2 && n->height >= 2) {
            prev->fwd[0] = n->fwd[0];
            s->size--;
            s->pa = prev;
            s->pb = n;
            s->plant = 2;
            return 0;
        }
        if (kind == 3 && n->height == 1) {
            n->height = 2;
            s->pa = n;
            s->plant = 3;
            return 0;
        }
    }
    if (kind == 4) {
        s->size++;
        s->plant = 4;
        return 0;
    }
    return -1;
}

void orc_debug_restore(orc_list *s)
{
    if (s->plant == 1) {
        const uint64_t k = s->pa->key;
        s->pa->key = s->pa->fwd[0]->key;
        s->pa->fwd[0]->key = k;
    } else if (s->plant == 2) {
        s->pa->fwd[0] = s->pb;
        s->size++;
    } else if (s->plant == 3) {
        s->pa->height = 1;
    } else if (s->plant == 4) {
        s->size--;
    }
    s->plant = 0;
    s->pa = s->pb = NULL;
}
