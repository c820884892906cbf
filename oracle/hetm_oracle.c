/*
 * hetm_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, single-threaded CPU statement of what one Speculative HeTM
 * (SHeTM) synchronization round computes on the GPU side, written from the
 * paper "HeTM: Transactional Memory for Heterogeneous Systems" (Castro,
 * Romano, Ilic, Khan):
 *
 *   - execution phase (§IV-C.1): the batch of GPU transactions, replayed one
 *     at a time in the order the GPU recorded, against the GPU replica, with
 *     the read-set / write-set granule bitmaps of the committed attempts
 *     (§IV-B "GPU instrumentation"; writes recorded in both bitmaps, §IV-C.2);
 *   - validation (§IV-C.2): a host log entry conflicts iff its word's granule
 *     is set in the read-set bitmap; the round conflicts iff any entry does;
 *   - apply (§IV-C.2): every entry is applied, even after a conflict, iff its
 *     timestamp is fresher than the word's TS entry;
 *   - merge (§IV-C.3): the dirty granules of the write-set bitmap are copied
 *     GPU->host on success and host->GPU on conflict (CPU-wins, §IV-E).
 *
 * There is no blocking, fusion or reordering beyond what those passages
 * state.  Only the tests, the smoke check and the CPU baseline of the
 * benchmark load this file; the product library never links it and the two
 * share no code.  It is built with plain gcc.
 *
 * Error codes (a documented contract shared by value, not by header):
 *   0 ok, -1 invalid argument, -3 timestamp order violated.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK      0
#define ORC_EINVAL -1
#define ORC_EORDER -3

#define TS_LIMIT (1ull << 63)

/* ---------------------------------------------------------------- bitmaps */

static void bit_set(uint32_t *bm, uint64_t i) { bm[i / 32] |= 1u << (i % 32); }
static int bit_get(const uint32_t *bm, uint64_t i) { return (bm[i / 32] >> (i % 32)) & 1u; }

/* Records one accessed word in the granule bitmaps: the read-set bitmap
 * gets every word read or written (so WS is a subset of RS, §IV-C.2), the
 * write-set bitmap only written words. */
static void note_read(uint32_t *RS, uint64_t G, uint64_t w) { bit_set(RS, w / G); }
static void note_write(uint32_t *RS, uint32_t *WS, uint64_t G, uint64_t w)
{
    bit_set(RS, w / G);
    bit_set(WS, w / G);
}

/* order[] must be a permutation of 0..n-1 */
static int check_permutation(const uint32_t *order, uint64_t n)
{
    uint8_t *seen = calloc(n ? n : 1, 1);
    if (!seen) return ORC_EINVAL;
    int rc = ORC_OK;
    for (uint64_t p = 0; p < n; p++) {
        if (order[p] >= n || seen[order[p]]) { rc = ORC_EINVAL; break; }
        seen[order[p]] = 1;
    }
    free(seen);
    return rc;
}

/* --------------------------------------------------- execution: programs */

/*
 * OPLIST program (the synthetic read / read-update transactions of §V-A):
 * transaction t reads words idx[off[t]..off[t+1]) in order, then for the
 * first nw[t] of them writes (value read + tid[t]) mod 2^32.  All reads come
 * before all writes, so no read sees the transaction's own write.
 *
 * Replays the batch serially in the given commit order against S, storing
 * every read value of t at results[off[t] + j].
 */
int orc_replay_oplist(uint32_t *S, uint64_t N, uint64_t G,
                      const uint32_t *off, const uint32_t *idx, const uint8_t *nw,
                      const uint32_t *tid, uint64_t n, const uint32_t *order,
                      uint32_t *results, uint32_t *RS, uint32_t *WS)
{
    if (G == 0 || check_permutation(order, n)) return ORC_EINVAL;
    for (uint64_t t = 0; t < n; t++) {
        if (off[t + 1] < off[t] || nw[t] > off[t + 1] - off[t]) return ORC_EINVAL;
        for (uint32_t k = off[t]; k < off[t + 1]; k++)
            if (idx[k] >= N) return ORC_EINVAL;
    }
    for (uint64_t p = 0; p < n; p++) {
        uint32_t t = order[p];
        uint32_t L = off[t + 1] - off[t];
        const uint32_t *a = idx + off[t];
        uint32_t *r = results + off[t];
        for (uint32_t j = 0; j < L; j++) {           /* phase 1: reads */
            r[j] = S[a[j]];
            note_read(RS, G, a[j]);
        }
        for (uint32_t j = 0; j < nw[t]; j++) {       /* phase 2: writes */
            S[a[j]] = r[j] + tid[t];
            note_write(RS, WS, G, a[j]);
        }
    }
    return ORC_OK;
}

/*
 * TRANSFER program (bank transfers over int64 accounts): read both balances;
 * if src != dst and the source balance covers the amount, move it.
 * results[t] = source balance read, results[n+t] = destination balance read,
 * results[2n+t] = 1 if the transfer was applied else 0.
 */
int orc_replay_transfer(int64_t *S, uint64_t N, uint64_t G,
                        const uint32_t *src, const uint32_t *dst, const uint32_t *amt,
                        uint64_t n, const uint32_t *order, int64_t *results,
                        uint32_t *RS, uint32_t *WS)
{
    if (G == 0 || check_permutation(order, n)) return ORC_EINVAL;
    for (uint64_t t = 0; t < n; t++)
        if (src[t] >= N || dst[t] >= N) return ORC_EINVAL;
    for (uint64_t p = 0; p < n; p++) {
        uint32_t t = order[p];
        int64_t bs = S[src[t]];
        int64_t bd = S[dst[t]];
        note_read(RS, G, src[t]);
        note_read(RS, G, dst[t]);
        int applied = src[t] != dst[t] && bs >= (int64_t)amt[t];
        if (applied) {
            S[src[t]] = bs - (int64_t)amt[t];
            S[dst[t]] = bd + (int64_t)amt[t];
            note_write(RS, WS, G, src[t]);
            note_write(RS, WS, G, dst[t]);
        }
        results[t] = bs;
        results[n + t] = bd;
        results[2 * n + t] = applied;
    }
    return ORC_OK;
}

/*
 * CACHE program: an 8-way set-associative object cache laid out in 32-bit
 * STMR words, after the cache of §V-D (per-way LRU stamp, per-set stamp
 * bumped by every PUT), one 128-word record per set:
 *
 *   words  0..15  keys of ways 0..7 (u64, low word first; 0 = empty way)
 *   words 16..23  LRU stamps of ways 0..7
 *   word  24      set PUT stamp
 *   words 32..95  values, way w at 32 + 8w (8 words; word 7 is a checksum)
 *
 * set(key) = (mix64(key) mod nsets) with its low bit replaced by the key's
 * low bit, so key parity partitions the sets.
 *
 * GET reads the set PUT stamp and the 8 keys; on a hit it reads the way's
 * value and writes the way's stamp := tid.  Result: 0x100|way on a hit, 0 on
 * a miss, then the 8 value words (zeros on a miss).
 * PUT reads the set PUT stamp, the 8 keys and the 8 stamps; the victim is the
 * way holding the key, else the way with the smallest stamp (lowest way on a
 * tie).  It writes key, value, the way's stamp := tid and the set PUT stamp
 * := tid.  Result: 0x200 | (0x100 if the key was present) | victim, then the
 * 8 value words written.
 */
#define C_SET_WORDS 128u
#define C_KEY(w)    (2u * (w))
#define C_STAMP(w)  (16u + (w))
#define C_SETSTAMP  24u
#define C_VAL(w)    (32u + 8u * (w))

uint64_t orc_mix64(uint64_t z)      /* splitmix64 finalizer (Steele et al.) */
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t orc_cache_set(uint64_t key, uint64_t nsets)
{
    return (orc_mix64(key) & (nsets - 1) & ~1ull) | (key & 1ull);
}

/* value words of a PUT of key by tid: 7 mixed words and an XOR checksum */
void orc_cache_value(uint64_t key, uint32_t tid, uint32_t v[8])
{
    uint32_t chk = (uint32_t)orc_mix64(key);
    for (uint32_t i = 0; i < 7; i++) {
        v[i] = (uint32_t)orc_mix64(key ^ ((uint64_t)tid << 32) ^ i);
        chk ^= v[i];
    }
    v[7] = chk;
}

static uint64_t load_key(const uint32_t *set, uint32_t w)
{
    return (uint64_t)set[C_KEY(w)] | ((uint64_t)set[C_KEY(w) + 1] << 32);
}

/* One cache operation on replica S; a NULL RS skips bitmap recording.
 * Writes the 9 result words to res. */
static void cache_op(uint32_t *S, uint64_t nsets, uint64_t G, uint64_t key, int is_put,
                     uint32_t tid, uint32_t *res, uint32_t *RS, uint32_t *WS)
{
    uint64_t base = orc_cache_set(key, nsets) * C_SET_WORDS;
    uint32_t *set = S + base;
    if (RS) note_read(RS, G, base + C_SETSTAMP);
    int hit = -1;
    for (uint32_t w = 0; w < 8; w++) {
        if (RS) { note_read(RS, G, base + C_KEY(w)); note_read(RS, G, base + C_KEY(w) + 1); }
        if (hit < 0 && load_key(set, w) == key) hit = (int)w;
    }
    if (!is_put) {
        memset(res, 0, 9 * sizeof(uint32_t));
        if (hit >= 0) {
            res[0] = 0x100u | (uint32_t)hit;
            for (uint32_t i = 0; i < 8; i++) {
                res[1 + i] = set[C_VAL(hit) + i];
                if (RS) note_read(RS, G, base + C_VAL(hit) + i);
            }
            set[C_STAMP(hit)] = tid;
            if (RS) note_write(RS, WS, G, base + C_STAMP(hit));
        }
        return;
    }
    uint32_t victim = 0;
    for (uint32_t w = 0; w < 8; w++) {
        if (RS) note_read(RS, G, base + C_STAMP(w));
        if (set[C_STAMP(w)] < set[C_STAMP(victim)]) victim = w;
    }
    if (hit >= 0) victim = (uint32_t)hit;
    uint32_t v[8];
    orc_cache_value(key, tid, v);
    set[C_KEY(victim)] = (uint32_t)key;
    set[C_KEY(victim) + 1] = (uint32_t)(key >> 32);
    for (uint32_t i = 0; i < 8; i++) set[C_VAL(victim) + i] = v[i];
    set[C_STAMP(victim)] = tid;
    set[C_SETSTAMP] = tid;
    if (RS) {
        note_write(RS, WS, G, base + C_KEY(victim));
        note_write(RS, WS, G, base + C_KEY(victim) + 1);
        for (uint32_t i = 0; i < 8; i++) note_write(RS, WS, G, base + C_VAL(victim) + i);
        note_write(RS, WS, G, base + C_STAMP(victim));
        note_write(RS, WS, G, base + C_SETSTAMP);
    }
    res[0] = 0x200u | (hit >= 0 ? 0x100u : 0u) | victim;
    for (uint32_t i = 0; i < 8; i++) res[1 + i] = v[i];
}

int orc_replay_cache(uint32_t *S, uint64_t N, uint64_t G,
                     const uint64_t *key, const uint8_t *op, const uint32_t *tid,
                     uint64_t n, const uint32_t *order, uint32_t *results,
                     uint32_t *RS, uint32_t *WS)
{
    uint64_t nsets = N / C_SET_WORDS;
    if (G == 0 || nsets < 2 || (nsets & (nsets - 1)) || N % C_SET_WORDS) return ORC_EINVAL;
    if (check_permutation(order, n)) return ORC_EINVAL;
    for (uint64_t t = 0; t < n; t++)
        if (key[t] == 0 || op[t] > 1) return ORC_EINVAL;
    for (uint64_t p = 0; p < n; p++) {
        uint32_t t = order[p];
        cache_op(S, nsets, G, key[t], op[t], tid[t], results + 9ull * t, RS, WS);
    }
    return ORC_OK;
}

/* ---------------------------------------------------- host side replay */

/*
 * The host runs its own transactions and logs the <word, value, timestamp>
 * of every word each committed transaction updated (§IV-B "CPU
 * instrumentation"); timestamps totally order the updates of each word.
 * These helpers replay host transactions serially in the order given (the
 * caller sorts them by their commit timestamps ts[]) on replica H and emit
 * the log that replay produces, so a host TM's concurrent result and log
 * can be checked against it.
 * Entry layout, W = 8: {u32 word, u32 pad, u64 value, u64 ts};
 * W = 4: {u32 word, u32 value, u64 ts}.  Return the number of entries.
 */
typedef struct { uint32_t word; uint32_t value; uint64_t ts; } orc_entry4;
typedef struct { uint32_t word; uint32_t pad; uint64_t value; uint64_t ts; } orc_entry8;

uint64_t orc_host_transfers(int64_t *H, uint64_t N, const uint32_t *src, const uint32_t *dst,
                            const uint32_t *amt, const uint64_t *ts, uint64_t n, orc_entry8 *log)
{
    uint64_t m = 0;
    for (uint64_t t = 0; t < n; t++) {
        if (src[t] >= N || dst[t] >= N) continue;
        int64_t bs = H[src[t]], bd = H[dst[t]];
        if (src[t] == dst[t] || bs < (int64_t)amt[t]) continue;
        H[src[t]] = bs - (int64_t)amt[t];
        H[dst[t]] = bd + (int64_t)amt[t];
        log[m++] = (orc_entry8){src[t], 0, (uint64_t)H[src[t]], ts[t]};
        log[m++] = (orc_entry8){dst[t], 0, (uint64_t)H[dst[t]], ts[t]};
    }
    return m;
}

uint64_t orc_host_cache_puts(uint32_t *H, uint64_t N, const uint64_t *key, const uint64_t *ts, uint64_t n,
                             orc_entry4 *log)
{
    uint64_t nsets = N / C_SET_WORDS, m = 0;
    for (uint64_t t = 0; t < n; t++) {
        uint64_t base = orc_cache_set(key[t], nsets) * C_SET_WORDS;
        uint32_t res[9];
        cache_op(H, nsets, 1, key[t], 1, (uint32_t)ts[t], res, NULL, NULL);
        uint32_t v = res[0] & 7u;
        uint32_t written[12] = {C_KEY(v), C_KEY(v) + 1, C_VAL(v) + 0, C_VAL(v) + 1,
                                C_VAL(v) + 2, C_VAL(v) + 3, C_VAL(v) + 4, C_VAL(v) + 5,
                                C_VAL(v) + 6, C_VAL(v) + 7, C_STAMP(v), C_SETSTAMP};
        for (uint32_t i = 0; i < 12; i++)
            log[m++] = (orc_entry4){(uint32_t)(base + written[i]), H[base + written[i]], ts[t]};
    }
    return m;
}

/* ----------------------------------------------------------- validation */

static uint64_t entry_word(const void *log, int W, uint64_t k)
{
    return W == 4 ? ((const orc_entry4 *)log)[k].word : ((const orc_entry8 *)log)[k].word;
}
static uint64_t entry_ts(const void *log, int W, uint64_t k)
{
    return W == 4 ? ((const orc_entry4 *)log)[k].ts : ((const orc_entry8 *)log)[k].ts;
}

/*
 * Validation (§IV-C.2): T^CPU can be serialized before T^GPU iff no word the
 * CPU wrote lies in a granule the GPU read (writes included).  flag bit k is
 * set iff entry k's word's granule is set in RS; *conflict = OR of all flags.
 * flags (nullable) holds ceil(n/32) words and is fully overwritten.
 */
int orc_validate(const void *log, int W, uint64_t n, const uint32_t *RS, uint64_t G,
                 uint64_t N, uint32_t *flags, uint32_t *conflict)
{
    if ((W != 4 && W != 8) || G == 0) return ORC_EINVAL;
    for (uint64_t k = 0; k < n; k++)
        if (entry_word(log, W, k) >= N) return ORC_EINVAL;
    if (flags) memset(flags, 0, ((n + 31) / 32) * sizeof(uint32_t));
    uint32_t any = 0;
    for (uint64_t k = 0; k < n; k++) {
        if (bit_get(RS, entry_word(log, W, k) / G)) {
            if (flags) bit_set(flags, k);
            any = 1;
        }
    }
    *conflict = any;
    return ORC_OK;
}

/* -------------------------------------------------------------- apply */

/*
 * Apply (§IV-C.2): the whole log is applied, also after a conflict.  Entries
 * arrive in arbitrary order, so an entry overwrites word w only if its
 * timestamp is fresher than TS[w]; TS[w] then takes that timestamp.  The
 * outcome is the entry with the largest timestamp per word.
 *
 * Timestamps must totally order the updates of one word (§IV-B), so the
 * result is undetermined when the timestamp that would win a word is
 * carried by two or more entries -- two of this chunk, or one of this chunk
 * and the winner an earlier chunk of the same round left in TS.  Ties below
 * a word's winning timestamp do not change the result and pass.
 *
 * A chunk is checked whole before anything of it is applied; a chunk that
 * fails a check applies nothing (S and TS unchanged):
 *   word < N (else -1);  floor < ts < 2^63 (else -3), where floor is the
 *   largest timestamp applied in earlier rounds;  no tie at a winning
 *   timestamp (else -3).
 * *max_ts receives the largest ts of the chunk (floor if it is empty).
 */
static int cmp_word_ts(const void *a, const void *b)
{
    const uint64_t *x = a, *y = b;           /* (word, ts) pairs */
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return x[1] < y[1] ? -1 : x[1] > y[1] ? 1 : 0;
}

int orc_apply(void *S, int W, uint64_t *TS, uint64_t N, const void *log, uint64_t n,
              uint64_t floor, uint64_t *max_ts)
{
    if (W != 4 && W != 8) return ORC_EINVAL;
    for (uint64_t k = 0; k < n; k++)
        if (entry_word(log, W, k) >= N) return ORC_EINVAL;
    uint64_t mx = floor;
    for (uint64_t k = 0; k < n; k++) {
        uint64_t ts = entry_ts(log, W, k);
        if (ts <= floor || ts >= TS_LIMIT) return ORC_EORDER;
        if (ts > mx) mx = ts;
    }
    /* the tie check: group the chunk's (word, ts) pairs by word; the last
     * pair of a group carries the word's largest ts m.  If m would win
     * (m > TS[w]) it must be carried by one entry only; if m equals TS[w]
     * it ties the winner of an earlier chunk. */
    uint64_t *pairs = malloc((n ? n : 1) * 2 * sizeof(uint64_t));
    if (!pairs) return ORC_EINVAL;
    for (uint64_t k = 0; k < n; k++) {
        pairs[2 * k] = entry_word(log, W, k);
        pairs[2 * k + 1] = entry_ts(log, W, k);
    }
    qsort(pairs, n, 2 * sizeof(uint64_t), cmp_word_ts);
    int rc = ORC_OK;
    for (uint64_t i = 0; i < n && rc == ORC_OK; i++) {
        int last_of_word = i + 1 == n || pairs[2 * (i + 1)] != pairs[2 * i];
        if (!last_of_word) continue;
        uint64_t w = pairs[2 * i], m = pairs[2 * i + 1];
        int dup = i > 0 && pairs[2 * (i - 1)] == w && pairs[2 * (i - 1) + 1] == m;
        if (m == TS[w] || (m > TS[w] && dup)) rc = ORC_EORDER;
    }
    free(pairs);
    if (rc != ORC_OK) return rc;
    for (uint64_t k = 0; k < n; k++) {         /* the freshness rule, entry by entry */
        uint64_t w = entry_word(log, W, k), ts = entry_ts(log, W, k);
        if (ts > TS[w]) {
            if (W == 4) ((uint32_t *)S)[w] = ((const orc_entry4 *)log)[k].value;
            else        ((uint64_t *)S)[w] = ((const orc_entry8 *)log)[k].value;
            TS[w] = ts;
        }
    }
    if (max_ts) *max_ts = mx;
    return ORC_OK;
}

/* -------------------------------------------------------------- merge */

/*
 * Merge (§IV-C.3), CPU-wins policy (§IV-E): for every granule g set in WS,
 * in ascending order, words [gG, min((g+1)G, N)) are copied from the GPU
 * replica S to the host replica H when the round had no conflict, and from
 * H to S when it had one.  ids (nullable) receives the ascending granule
 * ids; *n_dirty their count; *n_runs (nullable) the number of maximal runs
 * of consecutive ids.
 */
int orc_merge(uint32_t conflict, const uint32_t *WS, uint64_t G, uint64_t N, int W,
              void *S, void *H, uint32_t *ids, uint64_t *n_dirty, uint64_t *n_runs)
{
    if ((W != 4 && W != 8) || G == 0) return ORC_EINVAL;
    uint64_t nG = (N + G - 1) / G, d = 0, runs = 0;
    for (uint64_t g = 0; g < nG; g++) {
        if (!bit_get(WS, g)) continue;
        if (ids) ids[d] = (uint32_t)g;
        if (g == 0 || !bit_get(WS, g - 1)) runs++;
        d++;
        uint64_t lo = g * G, hi = lo + G < N ? lo + G : N;
        char *dst = (char *)(conflict ? S : H);
        const char *srcp = (const char *)(conflict ? H : S);
        memcpy(dst + lo * W, srcp + lo * W, (hi - lo) * W);
    }
    *n_dirty = d;
    if (n_runs) *n_runs = runs;
    return ORC_OK;
}
