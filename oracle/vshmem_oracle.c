/*
 * CPU oracle of the GPU-aware OpenSHMEM semantics on virtual PEs.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP implementation.
 *
 * Model.  Each virtual PE p owns a host byte array H[p] of `stride` bytes
 * (the symmetric heap slice of the paper's Section 2.1 and the GPU heap of
 * Section 6.1).  A symmetric object is named by its byte offset, the same on
 * every PE, so PE p's copy of object `o` is H[p][o].
 *
 * Operations are applied one at a time in a defined order: within one PE's
 * program, list order; across PEs, a deterministic scheduler that always
 * advances the lowest-numbered runnable PE.  A PE blocks at an unsatisfied
 * wait_until and at barrier_all.  If no PE can run and some have not
 * finished, the program deadlocks and the oracle reports it.
 *
 * The base meanings of put, get, the atomics, fence, quiet, wait and the
 * collectives are those of OpenSHMEM 1.x, which the paper keeps unchanged for
 * GPU-resident operands (Section 6.3, "RMA, atomics, synchronization, and
 * collectives"; operation list of Section 2.1).
 *
 * Built with plain gcc, -O2 -ffp-contract=off, no fast-math.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ types */
typedef struct {
    uint8_t op, scope, aux, flags;
    int32_t issuer, target;
    uint32_t result_idx;
    uint64_t src, dst, nbytes, value, cond, reserved;
} orc_desc;

enum {
    O_NOP = 0, O_PUT = 1, O_GET = 2, O_PUT_SIGNAL = 3,
    O_FETCH_ADD = 4, O_FETCH_XOR = 5, O_COMPARE_SWAP = 6,
    O_ADD = 7, O_XOR = 8, O_SET = 9, O_FETCH = 10, O_SWAP = 11,
    O_WAIT_UNTIL = 12, O_FENCE = 13, O_QUIET = 14, O_BARRIER_ALL = 15
};
enum { C_EQ = 0, C_NE, C_GT, C_GE, C_LT, C_LE };
enum { SIG_SET = 0, SIG_ADD = 1 };
enum {
    ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_RANGE = -2, ORC_ERR_CONFLICT = -3,
    ORC_ERR_DEADLOCK = -4, ORC_ERR_OP = -5, ORC_ERR_NOMEM = -6, ORC_ERR_SEARCH = -7
};
#define NO_RESULT 0xFFFFFFFFu

static void set_err(char *err, int errlen, const char *msg, long long a, long long b)
{
    if (err && errlen > 0) snprintf(err, (size_t)errlen, "%s (%lld, %lld)", msg, a, b);
}

/* -------------------------------------------------- int64 cells of a heap */
static uint64_t load64(const uint8_t *heap, uint64_t stride, int pe, uint64_t off)
{
    uint64_t v;
    memcpy(&v, heap + (uint64_t)pe * stride + off, 8);
    return v;
}

static void store64(uint8_t *heap, uint64_t stride, int pe, uint64_t off, uint64_t v)
{
    memcpy(heap + (uint64_t)pe * stride + off, &v, 8);
}

/* ------------------------------------------------------- conflict checker
 * Two accesses conflict when they touch a common byte, at least one of them
 * is a plain write, neither is ordered before the other, and they are not
 * both atomic.  Ordering follows the paper's Section 6.4: fence orders later
 * operations of a PE after its earlier ones, quiet completes them, a barrier
 * orders everything before it before everything after it, and an observed
 * signal (wait_until on a location written by put-with-signal or an atomic)
 * orders the writer's fenced operations before the waiter's later ones.
 * Atomicity alone does not order anything (Section 6.3).
 *
 * Bookkeeping uses vector clocks: seg[i] counts PE i's fence/quiet/barrier
 * points; vc[j*npes+i] is the number of PE i's segments that PE j knows to
 * be complete.  An access of PE i in segment s is ordered before the current
 * operation of PE j iff s < (i == j ? seg[j] : vc[j][i]).
 */
enum { A_READ = 0, A_WRITE = 1, A_ATOMIC = 2 };

typedef struct { int32_t pe; uint8_t kind; uint64_t seg, lo, hi; } access_rec;

typedef struct {
    access_rec *v;
    size_t n, cap, last_prune;
} access_log;

typedef struct { int32_t pe; uint64_t off; uint64_t *clock; } sig_clock;

typedef struct {
    int npes;
    uint64_t *seg;          /* npes */
    uint64_t *vc;           /* npes*npes */
    access_log *logs;       /* one per target PE */
    sig_clock *sigs;
    size_t nsig, capsig;
} checker;

static int checker_init(checker *c, int npes)
{
    memset(c, 0, sizeof(*c));
    c->npes = npes;
    c->seg = calloc((size_t)npes, sizeof(uint64_t));
    c->vc = calloc((size_t)npes * (size_t)npes, sizeof(uint64_t));
    c->logs = calloc((size_t)npes, sizeof(access_log));
    if (!c->seg || !c->vc || !c->logs) return ORC_ERR_NOMEM;
    return ORC_OK;
}

static void checker_free(checker *c)
{
    if (c->logs)
        for (int p = 0; p < c->npes; ++p) free(c->logs[p].v);
    for (size_t i = 0; i < c->nsig; ++i) free(c->sigs[i].clock);
    free(c->sigs);
    free(c->logs);
    free(c->vc);
    free(c->seg);
}

static int ordered_before(const checker *c, const access_rec *r, int j)
{
    if (r->pe == j) return r->seg < c->seg[j];
    return r->seg < c->vc[(size_t)j * c->npes + r->pe];
}

static void prune_log(checker *c, access_log *lg)
{
    size_t k = 0;
    for (size_t i = 0; i < lg->n; ++i) {
        int all = 1;
        for (int j = 0; j < c->npes && all; ++j)
            if (!ordered_before(c, &lg->v[i], j)) all = 0;
        if (!all) lg->v[k++] = lg->v[i];
    }
    lg->n = k;
    lg->last_prune = k;
}

/* Record an access by PE `who` to bytes [lo,hi) of PE `pe`; fail on conflict. */
static int access(checker *c, int who, int pe, uint64_t lo, uint64_t hi, int kind,
                  char *err, int errlen)
{
    if (hi <= lo) return ORC_OK;
    access_log *lg = &c->logs[pe];
    for (size_t i = 0; i < lg->n; ++i) {
        const access_rec *r = &lg->v[i];
        if (!(lo < r->hi && r->lo < hi)) continue;
        if (kind == A_READ && r->kind == A_READ) continue;
        if (kind == A_ATOMIC && r->kind == A_ATOMIC) continue;
        if (ordered_before(c, r, who)) continue;
        set_err(err, errlen, "conflicting accesses within one epoch on PE/offset", pe, (long long)lo);
        return ORC_ERR_CONFLICT;
    }
    if (lg->n == lg->cap) {
        size_t nc = lg->cap ? 2 * lg->cap : 64;
        access_rec *nv = realloc(lg->v, nc * sizeof(access_rec));
        if (!nv) return ORC_ERR_NOMEM;
        lg->v = nv;
        lg->cap = nc;
    }
    access_rec r = { who, (uint8_t)kind, c->seg[who], lo, hi };
    lg->v[lg->n++] = r;
    if (lg->n > 1024 && lg->n > 2 * lg->last_prune) prune_log(c, lg);
    return ORC_OK;
}

static uint64_t *sig_clock_of(checker *c, int pe, uint64_t off, int create)
{
    for (size_t i = 0; i < c->nsig; ++i)
        if (c->sigs[i].pe == pe && c->sigs[i].off == off) return c->sigs[i].clock;
    if (!create) return NULL;
    if (c->nsig == c->capsig) {
        size_t nc = c->capsig ? 2 * c->capsig : 16;
        sig_clock *ns = realloc(c->sigs, nc * sizeof(sig_clock));
        if (!ns) return NULL;
        c->sigs = ns;
        c->capsig = nc;
    }
    uint64_t *clk = calloc((size_t)c->npes, sizeof(uint64_t));
    if (!clk) return NULL;
    c->sigs[c->nsig].pe = pe;
    c->sigs[c->nsig].off = off;
    c->sigs[c->nsig].clock = clk;
    c->nsig++;
    return clk;
}

/* A release by PE `who` through location (pe, off): joins who's knowledge,
 * with its own completed segments, into the location's clock. */
static int release_through(checker *c, int who, int pe, uint64_t off)
{
    uint64_t *clk = sig_clock_of(c, pe, off, 1);
    if (!clk) return ORC_ERR_NOMEM;
    for (int k = 0; k < c->npes; ++k) {
        uint64_t v = (k == who) ? c->seg[who] : c->vc[(size_t)who * c->npes + k];
        if (v > clk[k]) clk[k] = v;
    }
    return ORC_OK;
}

static void acquire_from(checker *c, int who, int pe, uint64_t off)
{
    uint64_t *clk = sig_clock_of(c, pe, off, 0);
    if (!clk) return;
    for (int k = 0; k < c->npes; ++k) {
        if (k == who) continue;
        uint64_t *mine = &c->vc[(size_t)who * c->npes + k];
        if (clk[k] > *mine) *mine = clk[k];
    }
}

static void barrier_join(checker *c)
{
    for (int i = 0; i < c->npes; ++i) c->seg[i]++;
    for (int j = 0; j < c->npes; ++j)
        for (int i = 0; i < c->npes; ++i)
            c->vc[(size_t)j * c->npes + i] = c->seg[i];
    for (int p = 0; p < c->npes; ++p) {
        c->logs[p].n = 0;
        c->logs[p].last_prune = 0;
    }
}

/* ---------------------------------------------------------- the operations */
static int cmp_holds(uint64_t x, int cmp, uint64_t v, int is_unsigned)
{
    if (is_unsigned) {
        switch (cmp) {
        case C_EQ: return x == v;
        case C_NE: return x != v;
        case C_GT: return x > v;
        case C_GE: return x >= v;
        case C_LT: return x < v;
        case C_LE: return x <= v;
        }
    } else {
        int64_t a = (int64_t)x, b = (int64_t)v;
        switch (cmp) {
        case C_EQ: return a == b;
        case C_NE: return a != b;
        case C_GT: return a > b;
        case C_GE: return a >= b;
        case C_LT: return a < b;
        case C_LE: return a <= b;
        }
    }
    return 0;
}

static int in_heap(uint64_t stride, uint64_t off, uint64_t n)
{
    return off <= stride && n <= stride - off;
}

/*
 * Apply one non-blocking operation of PE `me`.
 *   put   (Section 2.1): H[target][dst, dst+n) <- H[me][src, src+n)
 *   get   (Section 2.1): H[me][dst, dst+n)     <- H[target][src, src+n)
 *   put-with-signal (Sections 4.3 and 7): the put, then the signal word at
 *         H[target][cond] is set to `value` or increased by it; the signal
 *         is never observable before the data.
 *   atomics (Section 2.1; atomicity without ordering, Section 6.3) on the
 *         int64 at H[target][src], two's-complement wrap:
 *         fetch_add: r = x; x = r + v     fetch_xor: r = x; x = r ^ v
 *         compare_swap: r = x; if r == cond: x = v
 *         add / xor: as above without the fetch; set: x = v;
 *         fetch: r = x; swap: r = x; x = v.
 *   fence / quiet (Section 6.4): no state change; they end the PE's segment.
 * The memcpy below is the plain definition of a put/get: the conflict rule
 * guarantees source and destination do not overlap.
 */
static int apply(uint8_t *heap, int npes, uint64_t stride, const orc_desc *d, uint64_t *results,
                 uint64_t nresults, checker *ck, char *err, int errlen)
{
    int me = d->issuer, t = d->target;
    if (me < 0 || me >= npes) { set_err(err, errlen, "issuer PE out of range", me, 0); return ORC_ERR_RANGE; }
    switch (d->op) {
    case O_NOP:
        return ORC_OK;
    case O_PUT:
    case O_GET:
    case O_PUT_SIGNAL: {
        if (t < 0 || t >= npes) { set_err(err, errlen, "target PE out of range", t, 0); return ORC_ERR_RANGE; }
        int rpe = (d->op == O_GET) ? t : me;    /* PE whose bytes are read */
        int wpe = (d->op == O_GET) ? me : t;    /* PE whose bytes are written */
        if (!in_heap(stride, d->src, d->nbytes) || !in_heap(stride, d->dst, d->nbytes)) {
            set_err(err, errlen, "RMA range outside the heap", (long long)d->src, (long long)d->dst);
            return ORC_ERR_RANGE;
        }
        if (ck) {
            int rc = access(ck, me, rpe, d->src, d->src + d->nbytes, A_READ, err, errlen);
            if (rc) return rc;
            rc = access(ck, me, wpe, d->dst, d->dst + d->nbytes, A_WRITE, err, errlen);
            if (rc) return rc;
        }
        if (d->nbytes)
            memmove(heap + (uint64_t)wpe * stride + d->dst, heap + (uint64_t)rpe * stride + d->src, d->nbytes);
        if (d->op == O_PUT_SIGNAL) {
            if (!in_heap(stride, d->cond, 8) || (d->cond & 7)) {
                set_err(err, errlen, "signal word outside the heap or misaligned", (long long)d->cond, 0);
                return ORC_ERR_RANGE;
            }
            if (ck) {
                ck->seg[me]++;   /* the data is ordered before the signal */
                int rc = access(ck, me, t, d->cond, d->cond + 8, A_ATOMIC, err, errlen);
                if (rc) return rc;
                rc = release_through(ck, me, t, d->cond);
                if (rc) return rc;
            }
            uint64_t s = load64(heap, stride, t, d->cond);
            s = (d->aux == SIG_ADD) ? s + d->value : d->value;
            store64(heap, stride, t, d->cond, s);
        }
        return ORC_OK;
    }
    case O_FETCH_ADD: case O_FETCH_XOR: case O_COMPARE_SWAP: case O_ADD: case O_XOR:
    case O_SET: case O_FETCH: case O_SWAP: {
        if (t < 0 || t >= npes) { set_err(err, errlen, "target PE out of range", t, 0); return ORC_ERR_RANGE; }
        if (!in_heap(stride, d->src, 8) || (d->src & 7)) {
            set_err(err, errlen, "atomic word outside the heap or misaligned", (long long)d->src, 0);
            return ORC_ERR_RANGE;
        }
        if (ck) {
            int rc = access(ck, me, t, d->src, d->src + 8, A_ATOMIC, err, errlen);
            if (rc) return rc;
            rc = release_through(ck, me, t, d->src);
            if (rc) return rc;
        }
        uint64_t x = load64(heap, stride, t, d->src), r = x, v = d->value;
        switch (d->op) {
        case O_FETCH_ADD: case O_ADD: x = r + v; break;
        case O_FETCH_XOR: case O_XOR: x = r ^ v; break;
        case O_COMPARE_SWAP: if (r == d->cond) x = v; break;
        case O_SET: case O_SWAP: x = v; break;
        case O_FETCH: break;
        }
        store64(heap, stride, t, d->src, x);
        int fetching = !(d->op == O_ADD || d->op == O_XOR || d->op == O_SET);
        if (fetching && d->result_idx != NO_RESULT) {
            if (d->result_idx >= nresults) { set_err(err, errlen, "result index out of range", d->result_idx, 0); return ORC_ERR_RANGE; }
            results[d->result_idx] = r;
        }
        return ORC_OK;
    }
    case O_FENCE:
    case O_QUIET:
        if (ck) ck->seg[me]++;
        return ORC_OK;
    default:
        set_err(err, errlen, "unknown operation code", d->op, 0);
        return ORC_ERR_OP;
    }
}

/*
 * Run a multi-PE program.  descs[] holds every PE's operations; PE p's
 * program is the subsequence with issuer == p, in list order.  barrier_all
 * (Section 6.3, device collectives; a barrier implies quiet, Section 6.3
 * "Remote visibility is only guaranteed after an explicit quiet/barrier")
 * is a rendezvous of all PEs.  wait_until (Section 2.1, point-to-point
 * synchronization) blocks PE p until the int64 (or uint64 when flags bit 0
 * is set) at H[p][src] satisfies `aux` against `value`.
 *
 * results[] receives the fetched value of every fetching atomic with a
 * result index.  check != 0 enables the conflict checker.
 * Returns ORC_OK or a negative ORC_ERR_* code with a message in err.
 */
int orc_run_program(uint8_t *heap, int npes, uint64_t stride, const orc_desc *descs, uint64_t n,
                    uint64_t *results, uint64_t nresults, int check, char *err, int errlen)
{
    if (!heap || npes <= 0 || (!descs && n)) return ORC_ERR_ARG;
    uint64_t **prog = calloc((size_t)npes, sizeof(uint64_t *));
    uint64_t *plen = calloc((size_t)npes, sizeof(uint64_t));
    uint64_t *pc = calloc((size_t)npes, sizeof(uint64_t));
    int *at_barrier = calloc((size_t)npes, sizeof(int));
    int rc = ORC_OK;
    checker ck;
    int ck_ok = 0;
    if (!prog || !plen || !pc || !at_barrier) { rc = ORC_ERR_NOMEM; goto done; }
    for (uint64_t i = 0; i < n; ++i) {
        int p = descs[i].issuer;
        if (p < 0 || p >= npes) { set_err(err, errlen, "issuer PE out of range", p, (long long)i); rc = ORC_ERR_RANGE; goto done; }
        plen[p]++;
    }
    for (int p = 0; p < npes; ++p) {
        prog[p] = malloc((plen[p] ? plen[p] : 1) * sizeof(uint64_t));
        if (!prog[p]) { rc = ORC_ERR_NOMEM; goto done; }
        plen[p] = 0;
    }
    for (uint64_t i = 0; i < n; ++i) {
        int p = descs[i].issuer;
        prog[p][plen[p]++] = i;
    }
    if (check) {
        rc = checker_init(&ck, npes);
        ck_ok = 1;
        if (rc) goto done;
    }
    for (;;) {
        int finished = 0, waiting_barrier = 0;
        for (int p = 0; p < npes; ++p) {
            if (pc[p] >= plen[p]) finished++;
            else if (at_barrier[p]) waiting_barrier++;
        }
        if (waiting_barrier == npes) {           /* every PE arrived: release */
            for (int p = 0; p < npes; ++p) { at_barrier[p] = 0; pc[p]++; }
            if (check) barrier_join(&ck);
            continue;
        }
        if (finished == npes) break;
        int advanced = 0;
        for (int p = 0; p < npes && !advanced; ++p) {   /* lowest runnable PE */
            if (pc[p] >= plen[p] || at_barrier[p]) continue;
            const orc_desc *d = &descs[prog[p][pc[p]]];
            if (d->op == O_BARRIER_ALL) {
                at_barrier[p] = 1;
                advanced = 1;
            } else if (d->op == O_WAIT_UNTIL) {
                if (!in_heap(stride, d->src, 8) || (d->src & 7)) {
                    set_err(err, errlen, "wait word outside the heap or misaligned", (long long)d->src, 0);
                    rc = ORC_ERR_RANGE;
                    goto done;
                }
                uint64_t x = load64(heap, stride, p, d->src);
                if (!cmp_holds(x, d->aux, d->value, d->flags & 1)) continue;   /* blocked */
                if (check) {
                    rc = access(&ck, p, p, d->src, d->src + 8, A_ATOMIC, err, errlen);
                    if (rc) goto done;
                    acquire_from(&ck, p, p, d->src);
                }
                pc[p]++;
                advanced = 1;
            } else {
                rc = apply(heap, npes, stride, d, results, nresults, check ? &ck : NULL, err, errlen);
                if (rc) goto done;
                pc[p]++;
                advanced = 1;
            }
        }
        if (!advanced) {
            set_err(err, errlen, "deadlock: no PE can run; finished PEs / PEs", finished, npes);
            rc = ORC_ERR_DEADLOCK;
            goto done;
        }
    }
done:
    if (ck_ok) checker_free(&ck);
    if (prog)
        for (int p = 0; p < npes; ++p) free(prog[p]);
    free(prog);
    free(plen);
    free(pc);
    free(at_barrier);
    return rc;
}

/* ------------------------------------------------- host-memory operands
 * Host-initiated put and get (Tier 0 of Section 7: the host issues OpenSHMEM
 * operations on GPU-resident symmetric objects, Section 6.3).  The local
 * operand is a private buffer of the issuing host, not a heap object:
 *   put: H[pe][dst, dst+n) <- buf[0, n)
 *   get: buf[0, n)         <- H[pe][src, src+n)
 * A heap-to-heap host operation is an ordinary put/get of PE 0 (the PE the
 * host acts for) and goes through orc_run_program.
 */
int orc_host_put(uint8_t *heap, int npes, uint64_t stride, int pe, uint64_t dst, const uint8_t *buf, uint64_t n)
{
    if (pe < 0 || pe >= npes || (!buf && n)) return ORC_ERR_ARG;
    if (!in_heap(stride, dst, n)) return ORC_ERR_RANGE;
    memcpy(heap + (uint64_t)pe * stride + dst, buf, n);
    return ORC_OK;
}

int orc_host_get(const uint8_t *heap, int npes, uint64_t stride, int pe, uint64_t src, uint8_t *buf, uint64_t n)
{
    if (pe < 0 || pe >= npes || (!buf && n)) return ORC_ERR_ARG;
    if (!in_heap(stride, src, n)) return ORC_ERR_RANGE;
    memcpy(buf, heap + (uint64_t)pe * stride + src, n);
    return ORC_OK;
}

/* --------------------------------------------------------------- teams */
/* Team member k is PE start + k*stride_pe (OpenSHMEM strided teams). */
static int team_pe(int start, int stride_pe, int k) { return start + k * stride_pe; }

static int team_ok(int npes, int start, int stride_pe, int size)
{
    if (size <= 0 || start < 0 || stride_pe <= 0) return 0;
    return team_pe(start, stride_pe, size - 1) < npes;
}

/*
 * broadcast (team collective named in Section 4.3): every member's
 * H[p][dst, dst+n) receives H[root][src, src+n); the root's own destination
 * is written too.  `root` is a team index.
 */
int orc_broadcast(uint8_t *heap, int npes, uint64_t stride, int start, int stride_pe, int size,
                  uint64_t dst, uint64_t src, uint64_t n, int root)
{
    if (!team_ok(npes, start, stride_pe, size) || root < 0 || root >= size) return ORC_ERR_ARG;
    if (!in_heap(stride, dst, n) || !in_heap(stride, src, n)) return ORC_ERR_RANGE;
    const uint8_t *s = heap + (uint64_t)team_pe(start, stride_pe, root) * stride + src;
    uint8_t *tmp = malloc(n ? n : 1);
    if (!tmp) return ORC_ERR_NOMEM;
    memcpy(tmp, s, n);
    for (int k = 0; k < size; ++k)
        memcpy(heap + (uint64_t)team_pe(start, stride_pe, k) * stride + dst, tmp, n);
    free(tmp);
    return ORC_OK;
}

/*
 * fcollect (concatenation of every member's block): for every members p and
 * q, H[p][dst + q*n, +n) receives H[q][src, +n).
 */
int orc_fcollect(uint8_t *heap, int npes, uint64_t stride, int start, int stride_pe, int size,
                 uint64_t dst, uint64_t src, uint64_t n)
{
    if (!team_ok(npes, start, stride_pe, size)) return ORC_ERR_ARG;
    if (!in_heap(stride, dst, n * (uint64_t)size) || !in_heap(stride, src, n)) return ORC_ERR_RANGE;
    uint8_t *all = malloc(n * (uint64_t)size + 1);
    if (!all) return ORC_ERR_NOMEM;
    for (int q = 0; q < size; ++q)
        memcpy(all + (uint64_t)q * n, heap + (uint64_t)team_pe(start, stride_pe, q) * stride + src, n);
    for (int p = 0; p < size; ++p)
        memcpy(heap + (uint64_t)team_pe(start, stride_pe, p) * stride + dst, all, n * (uint64_t)size);
    free(all);
    return ORC_OK;
}

/*
 * alltoall (team collective named in Section 4.3): for every members p, q,
 * H[p][dst + q*n, +n) receives H[q][src + p*n, +n)  (a block transpose).
 */
int orc_alltoall(uint8_t *heap, int npes, uint64_t stride, int start, int stride_pe, int size,
                 uint64_t dst, uint64_t src, uint64_t n)
{
    if (!team_ok(npes, start, stride_pe, size)) return ORC_ERR_ARG;
    uint64_t tot = n * (uint64_t)size;
    if (!in_heap(stride, dst, tot) || !in_heap(stride, src, tot)) return ORC_ERR_RANGE;
    uint8_t *snap = malloc(tot * (uint64_t)size + 1);
    if (!snap) return ORC_ERR_NOMEM;
    for (int q = 0; q < size; ++q)
        memcpy(snap + (uint64_t)q * tot, heap + (uint64_t)team_pe(start, stride_pe, q) * stride + src, tot);
    for (int p = 0; p < size; ++p)
        for (int q = 0; q < size; ++q)
            memcpy(heap + (uint64_t)team_pe(start, stride_pe, p) * stride + dst + (uint64_t)q * n,
                   snap + (uint64_t)q * tot + (uint64_t)p * n, n);
    free(snap);
    return ORC_OK;
}

/* ------------------------------------------------------------ reductions
 * Reductions to all (thread-collaborative reductions, Section 4.4 case
 * study 3): for every element k, r = TREE(x_0k, ..., x_{P-1}k) over the team
 * in team order, and every member's destination element k receives r.
 *
 * TREE is the documented order: L = [x_0 .. x_{P-1}]; while |L| > 1, replace
 * L by [op(L[0],L[1]), op(L[2],L[3]), ...] and, when |L| is odd, carry its
 * last element unchanged; the result is the single remaining element.
 *
 * Types: int64 (wrapping add), fp32 (IEEE round-to-nearest-even adds) and
 * bf16 (each input widened exactly to fp32, reduced in fp32, the result
 * rounded once to bf16 with round-to-nearest-even).  max uses
 * op(a, b) = (b > a) ? b : a, so a tie keeps the left (lower-PE) operand.
 */
enum { DT_INT64 = 0, DT_FP32 = 1, DT_BF16 = 2 };
enum { RO_SUM = 0, RO_MAX = 1 };

static int64_t op_i64(int rop, int64_t a, int64_t b)
{
    if (rop == RO_SUM) return (int64_t)((uint64_t)a + (uint64_t)b);
    return (b > a) ? b : a;
}

static float op_f32(int rop, float a, float b)
{
    if (rop == RO_SUM) return a + b;
    return (b > a) ? b : a;
}

static float bf16_widen(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

static uint16_t bf16_round(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
        return (uint16_t)((u >> 16) | 0x0040u);          /* NaN stays NaN (quiet) */
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

/* TREE over L[0..m) in place; returns L[0]. */
static int64_t tree_i64(int rop, int64_t *L, int m)
{
    while (m > 1) {
        int h = 0;
        for (int j = 0; 2 * j + 1 < m; ++j) L[h++] = op_i64(rop, L[2 * j], L[2 * j + 1]);
        if (m & 1) L[h++] = L[m - 1];
        m = h;
    }
    return L[0];
}

static float tree_f32(int rop, float *L, int m)
{
    while (m > 1) {
        int h = 0;
        for (int j = 0; 2 * j + 1 < m; ++j) L[h++] = op_f32(rop, L[2 * j], L[2 * j + 1]);
        if (m & 1) L[h++] = L[m - 1];
        m = h;
    }
    return L[0];
}

/* Element size of a reduction datatype. */
static uint64_t dt_size(int dt) { return dt == DT_INT64 ? 8 : (dt == DT_FP32 ? 4 : 2); }

/*
 * Reduce `nreduce` elements of type `dt` found at H[q][src] on every member
 * q; write the result to H[p][dst] on every member p.  Elements listed in
 * `only` (when non-NULL, `nonly` indices) are the only ones computed and are
 * written to out[] instead of the heap: this computes sampled outputs one
 * by one for checks at large sizes.
 */
int orc_reduce(uint8_t *heap, int npes, uint64_t stride, int start, int stride_pe, int size,
               int dt, int rop, uint64_t dst, uint64_t src, uint64_t nreduce,
               const uint64_t *only, uint64_t nonly, void *out)
{
    if (!team_ok(npes, start, stride_pe, size) || dt < DT_INT64 || dt > DT_BF16 || rop < RO_SUM || rop > RO_MAX)
        return ORC_ERR_ARG;
    uint64_t es = dt_size(dt);
    if (!in_heap(stride, src, nreduce * es)) return ORC_ERR_RANGE;
    if (!only && !in_heap(stride, dst, nreduce * es)) return ORC_ERR_RANGE;
    int64_t *Li = malloc((size_t)size * sizeof(int64_t));
    float *Lf = malloc((size_t)size * sizeof(float));
    if (!Li || !Lf) { free(Li); free(Lf); return ORC_ERR_NOMEM; }
    /* Read every source element before writing any destination: dst may alias src. */
    uint64_t count = only ? nonly : nreduce;
    uint8_t *res = malloc(count * es + 1);
    if (!res) { free(Li); free(Lf); return ORC_ERR_NOMEM; }
    for (uint64_t e = 0; e < count; ++e) {
        uint64_t k = only ? only[e] : e;
        if (k >= nreduce) { free(Li); free(Lf); free(res); return ORC_ERR_RANGE; }
        for (int q = 0; q < size; ++q) {
            const uint8_t *p = heap + (uint64_t)team_pe(start, stride_pe, q) * stride + src + k * es;
            if (dt == DT_INT64) memcpy(&Li[q], p, 8);
            else if (dt == DT_FP32) memcpy(&Lf[q], p, 4);
            else { uint16_t h; memcpy(&h, p, 2); Lf[q] = bf16_widen(h); }
        }
        if (dt == DT_INT64) { int64_t r = tree_i64(rop, Li, size); memcpy(res + e * es, &r, 8); }
        else if (dt == DT_FP32) { float r = tree_f32(rop, Lf, size); memcpy(res + e * es, &r, 4); }
        else { uint16_t r = bf16_round(tree_f32(rop, Lf, size)); memcpy(res + e * es, &r, 2); }
    }
    if (only) {
        memcpy(out, res, count * es);
    } else {
        for (int p = 0; p < size; ++p)
            memcpy(heap + (uint64_t)team_pe(start, stride_pe, p) * stride + dst, res, nreduce * es);
    }
    free(res);
    free(Li);
    free(Lf);
    return ORC_OK;
}

/* fp32 -> bf16 rounding used by the reductions, exported for its own pin. */
uint16_t orc_bf16_round(float f) { return bf16_round(f); }

/* ------------------------------------------------------------------- GUPS
 * Random-access atomics (Section 4.4 case study 2: remote atomic updates).
 * table[] is the whole distributed table in global-index order (the caller
 * maps global index g to its home PE).  Update u, in update order, is
 * fetch_add(value) when is_add[u] and fetch_xor(value) otherwise; its fetched
 * value goes to fetched[u] when fetched is non-NULL.
 */
int orc_gups(int64_t *table, uint64_t nentries, const uint64_t *idx, const uint64_t *val,
             const uint8_t *is_add, uint64_t nupd, uint64_t *fetched)
{
    for (uint64_t u = 0; u < nupd; ++u) {
        uint64_t g = idx[u];
        if (g >= nentries) return ORC_ERR_RANGE;
        uint64_t r = (uint64_t)table[g];
        table[g] = (int64_t)(is_add[u] ? r + val[u] : r ^ val[u]);
        if (fetched) fetched[u] = r;
    }
    return ORC_OK;
}

/* ------------------------------------------------------- witness replay
 * Atomicity does not imply ordering (Section 6.3), so a GPU may apply the
 * atomics on one word in any order.  Given, for every update, the word it
 * hit, its kind (0 = fetch_add, 1 = fetch_xor, 2 = fetch with no change) and
 * operand, and the value the GPU says it fetched, decide whether some
 * serial order of the updates explains every fetched value and the word's
 * final value.  Starting from the initial value x, repeatedly apply an unused
 * update whose fetched value equals x; when candidates with different
 * effects exist, search depth first (bounded by `budget` steps).
 *
 * addr[u] indexes init[]/final[]; returns the number of words for which no
 * such order exists (0 = all valid), or ORC_ERR_SEARCH if the budget ran out.
 */
static uint64_t apply_kind(int kind, uint64_t x, uint64_t v)
{
    return kind == 0 ? x + v : (kind == 1 ? x ^ v : x);
}

typedef struct { uint64_t *ids; uint64_t n; } group_t;

static int replay_group(const uint8_t *kind, const uint64_t *val, const uint64_t *fetched,
                        const uint64_t *ids, uint64_t m, uint64_t init, uint64_t final,
                        uint64_t *budget)
{
    /* Depth-first search with an explicit stack of choice points. */
    uint8_t *used = calloc(m + 1, 1);
    uint64_t *stack = malloc((m + 1) * sizeof(uint64_t));      /* chosen position per depth */
    uint64_t *xs = malloc((m + 1) * sizeof(uint64_t));         /* x before each depth */
    if (!used || !stack || !xs) { free(used); free(stack); free(xs); return -1; }
    uint64_t depth = 0, x = init;
    uint64_t next_try = 0;
    int ok = 0;
    for (;;) {
        if (depth == m) {
            if (x == final) { ok = 1; break; }
            goto backtrack;
        }
        {
            uint64_t found = m;
            for (uint64_t j = next_try; j < m; ++j)
                if (!used[j] && fetched[ids[j]] == x) { found = j; break; }
            if (found == m) goto backtrack;
            if (*budget == 0) { ok = -2; break; }
            (*budget)--;
            used[found] = 1;
            stack[depth] = found;
            xs[depth] = x;
            x = apply_kind(kind[ids[found]], x, val[ids[found]]);
            depth++;
            next_try = 0;
            continue;
        }
    backtrack:
        if (depth == 0) { ok = 0; break; }
        depth--;
        used[stack[depth]] = 0;
        x = xs[depth];
        /* Skip alternatives with the same effect as the one just undone. */
        {
            uint64_t undone = stack[depth];
            uint64_t j = undone + 1;
            while (j < m && (used[j] || fetched[ids[j]] != x ||
                             (kind[ids[j]] == kind[ids[undone]] && val[ids[j]] == val[ids[undone]])))
                ++j;
            next_try = j;
        }
    }
    free(used);
    free(stack);
    free(xs);
    return ok;
}

static const uint64_t *g_sort_addr;
static int cmp_by_addr(const void *a, const void *b)
{
    uint64_t x = g_sort_addr[*(const uint64_t *)a], y = g_sort_addr[*(const uint64_t *)b];
    if (x != y) return x < y ? -1 : 1;
    uint64_t i = *(const uint64_t *)a, j = *(const uint64_t *)b;
    return i < j ? -1 : (i > j);
}

int64_t orc_witness_check(const uint64_t *addr, const uint8_t *kind, const uint64_t *val,
                          const uint64_t *fetched, uint64_t nupd, const uint64_t *init,
                          const uint64_t *final, uint64_t nwords, uint64_t budget)
{
    uint64_t *order = malloc((nupd + 1) * sizeof(uint64_t));
    if (!order) return ORC_ERR_NOMEM;
    for (uint64_t u = 0; u < nupd; ++u) {
        if (addr[u] >= nwords) { free(order); return ORC_ERR_RANGE; }
        order[u] = u;
    }
    g_sort_addr = addr;
    qsort(order, nupd, sizeof(uint64_t), cmp_by_addr);
    int64_t bad = 0;
    uint8_t *seen = calloc(nwords + 1, 1);
    if (!seen) { free(order); return ORC_ERR_NOMEM; }
    uint64_t i = 0;
    while (i < nupd) {
        uint64_t a = addr[order[i]], j = i;
        while (j < nupd && addr[order[j]] == a) ++j;
        seen[a] = 1;
        int r = replay_group(kind, val, fetched, order + i, j - i, init[a], final[a], &budget);
        if (r == -2) { free(order); free(seen); return ORC_ERR_SEARCH; }
        if (r != 1) bad++;
        i = j;
    }
    for (uint64_t a = 0; a < nwords; ++a)
        if (!seen[a] && init[a] != final[a]) bad++;    /* untouched words must not change */
    free(order);
    free(seen);
    return bad;
}
