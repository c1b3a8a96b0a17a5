/*
 * CPU oracle for the all-matches PFSM scan.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * links, calls or includes it, and the two share no code.
 *
 * What it computes is the plain definition of the PFSM's output
 * (Section III.B, match reporting rule; Fig. 2 is an instance of it):
 *
 *   M(x) = { (s, e, l) : 0 <= s <= e < n, some path from q0 that spells
 *            x[s..e] (epsilon edges interleaved freely) ends in a final
 *            state f, and l is a label of f }
 *
 * written out per start position s.  Restarting the matcher at every start
 * position is the acalculia remedy recalled in Section II; it yields the same
 * set as the PFSM's tagged reinitialisation (Section III.B), where a tag is
 * the start position and travels unmodified with the instance.  For start s
 * the set S of states reachable after x[s..e] is advanced one symbol at a
 * time (the PFSM's steps 3 and 4), closed under epsilon edges right after
 * each symbol, and every label of every final state in S is reported with
 * end e.  Empty matches (a final state in the epsilon closure of q0) are
 * never reported: every match consumes at least one symbol.
 *
 * Two optional shortcuts, each switchable so the tests can show that it does
 * not change the result:
 *   prune: drop states from which no final state is reachable (they cannot
 *          contribute a match); an instance ends when its set is empty.
 *   memo:  the first step of every start applies the same function to the
 *          same argument, closure(delta(closure({q0}), c)); it is computed
 *          once per byte value c.
 *
 * Work counters (metric numerators, not results):
 *   T = instance-steps: for every start, the number of symbols consumed while
 *       its set was non-empty (the symbol that empties it included);
 *   X = state activations: the sum over those steps of the size of the set
 *       after the step.
 *
 * Threads split the starts into contiguous segments; a segment's walks read
 * past the segment's end until their set empties or the input ends (lazy data
 * partitioning, Section III.D.2).  Output triples are int32 (start, end,
 * label), end inclusive, sorted by (start, end, label) without duplicates.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small growable arrays                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t *v;
    int64_t n, cap;
} vec32;

static int vpush(vec32 *a, int32_t x) {
    if (a->n == a->cap) {
        int64_t nc = a->cap ? a->cap * 2 : 64;
        int32_t *nv = (int32_t *)realloc(a->v, (size_t)nc * sizeof(int32_t));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ */
/* automaton view                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int is_dfa;
    int32_t n_states, q0;
    /* DFA */
    int32_t n_symbols;
    const int16_t *b2s;
    const int32_t *delta;
    /* NFA */
    const int32_t *row_ptr, *edge_class, *edge_dst;
    const uint32_t *class_bits;
    int32_t n_classes;
    /* labels */
    const int32_t *final_off, *final_labels;
    /* derived */
    uint8_t *coreach;       /* 1 when a final state is reachable (0 or more steps) */
    int prune, memo;
    vec32 first[256];       /* memo: closure(delta(closure({q0}), c)), pruned if prune */
    vec32 z;                /* closure({q0}) */
} fsm_t;

static int class_has(const fsm_t *a, int32_t k, uint8_t c) {
    return (a->class_bits[(int64_t)k * 8 + (c >> 5)] >> (c & 31)) & 1u;
}

static int class_nonempty(const fsm_t *a, int32_t k) {
    for (int w = 0; w < 8; w++)
        if (a->class_bits[(int64_t)k * 8 + w]) return 1;
    return 0;
}

static int dfa_symbol(const fsm_t *a, uint8_t c) {
    return a->b2s ? (int)a->b2s[c] : (int)c;
}

/* Reverse breadth-first search from the final states over every edge that
 * some byte (or epsilon) can take. */
static int compute_coreach(fsm_t *a) {
    int32_t N = a->n_states;
    a->coreach = (uint8_t *)calloc((size_t)N, 1);
    if (!a->coreach) return -1;
    int64_t n_edges;
    int32_t *rsrc, *rdst; /* reverse edge list: rdst <- rsrc */
    if (a->is_dfa) {
        int S = a->n_symbols;
        uint8_t *sym_used = (uint8_t *)calloc((size_t)S, 1);
        if (!sym_used) return -1;
        if (a->b2s) {
            for (int b = 0; b < 256; b++)
                if (a->b2s[b] >= 0) sym_used[a->b2s[b]] = 1;
        } else {
            for (int s = 0; s < S; s++) sym_used[s] = 1;
        }
        n_edges = (int64_t)N * S;
        rsrc = (int32_t *)malloc((size_t)n_edges * sizeof(int32_t));
        rdst = (int32_t *)malloc((size_t)n_edges * sizeof(int32_t));
        if (!rsrc || !rdst) return -1;
        int64_t m = 0;
        for (int32_t q = 0; q < N; q++)
            for (int s = 0; s < S; s++) {
                int32_t t = a->delta[(int64_t)q * S + s];
                if (t >= 0 && sym_used[s]) { rsrc[m] = t; rdst[m] = q; m++; }
            }
        n_edges = m;
        free(sym_used);
    } else {
        n_edges = a->row_ptr[N];
        rsrc = (int32_t *)malloc((size_t)(n_edges + 1) * sizeof(int32_t));
        rdst = (int32_t *)malloc((size_t)(n_edges + 1) * sizeof(int32_t));
        if (!rsrc || !rdst) return -1;
        int64_t m = 0;
        for (int32_t q = 0; q < N; q++)
            for (int32_t e = a->row_ptr[q]; e < a->row_ptr[q + 1]; e++) {
                int32_t k = a->edge_class[e];
                if (k < 0 || class_nonempty(a, k)) { rsrc[m] = a->edge_dst[e]; rdst[m] = q; m++; }
            }
        n_edges = m;
    }
    /* CSR of the reverse graph keyed by rsrc */
    int32_t *off = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    int32_t *adj = (int32_t *)malloc((size_t)(n_edges + 1) * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!off || !adj || !queue) return -1;
    for (int64_t i = 0; i < n_edges; i++) off[rsrc[i] + 1]++;
    for (int32_t q = 0; q < N; q++) off[q + 1] += off[q];
    int32_t *fill = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!fill) return -1;
    memcpy(fill, off, (size_t)N * sizeof(int32_t));
    for (int64_t i = 0; i < n_edges; i++) adj[fill[rsrc[i]]++] = rdst[i];
    int32_t head = 0, tail = 0;
    for (int32_t q = 0; q < N; q++)
        if (a->final_off[q + 1] > a->final_off[q]) { a->coreach[q] = 1; queue[tail++] = q; }
    while (head < tail) {
        int32_t q = queue[head++];
        for (int32_t i = off[q]; i < off[q + 1]; i++) {
            int32_t p = adj[i];
            if (!a->coreach[p]) { a->coreach[p] = 1; queue[tail++] = p; }
        }
    }
    free(rsrc); free(rdst); free(off); free(adj); free(queue); free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* per-thread NFA set machinery                                         */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t *mark; /* mark[q] == gen  <=>  q is in the set being built */
    uint32_t gen;
    vec32 cur, nxt, labs;
} setws_t;

static void ws_newset(setws_t *w, int32_t n_states) {
    if (++w->gen == 0) {
        memset(w->mark, 0, (size_t)n_states * sizeof(uint32_t));
        w->gen = 1;
    }
}

static int ws_add(setws_t *w, vec32 *set, int32_t q) {
    if (w->mark[q] == w->gen) return 0;
    w->mark[q] = w->gen;
    return vpush(set, q);
}

/* Close `set` (whose members are marked with the current generation) under
 * epsilon edges. */
static int eps_close(const fsm_t *a, setws_t *w, vec32 *set) {
    for (int64_t i = 0; i < set->n; i++) {
        int32_t q = set->v[i];
        for (int32_t e = a->row_ptr[q]; e < a->row_ptr[q + 1]; e++)
            if (a->edge_class[e] < 0)
                if (ws_add(w, set, a->edge_dst[e])) return -1;
    }
    return 0;
}

/* out = closure(delta(in, c)), then intersected with the co-reachable set
 * when pruning. */
static int nfa_step(const fsm_t *a, setws_t *w, const vec32 *in, uint8_t c, vec32 *out) {
    out->n = 0;
    ws_newset(w, a->n_states);
    for (int64_t i = 0; i < in->n; i++) {
        int32_t q = in->v[i];
        for (int32_t e = a->row_ptr[q]; e < a->row_ptr[q + 1]; e++) {
            int32_t k = a->edge_class[e];
            if (k >= 0 && class_has(a, k, c))
                if (ws_add(w, out, a->edge_dst[e])) return -1;
        }
    }
    if (eps_close(a, w, out)) return -1;
    if (a->prune) {
        int64_t m = 0;
        for (int64_t i = 0; i < out->n; i++)
            if (a->coreach[out->v[i]]) out->v[m++] = out->v[i];
        out->n = m;
    }
    return 0;
}

static int nfa_closure_q0(const fsm_t *a, setws_t *w, vec32 *out) {
    out->n = 0;
    ws_newset(w, a->n_states);
    if (ws_add(w, out, a->q0)) return -1;
    return eps_close(a, w, out);
}

/* ------------------------------------------------------------------ */
/* emission                                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    vec32 m;      /* triples, flattened */
    int64_t T, X;
    int err;
} chunk_out_t;

/* Emit (s, e, l) for every distinct label l of the final states in `set`,
 * in increasing label order. */
static int emit_set(const fsm_t *a, setws_t *w, const int32_t *states, int64_t n_set,
                    int64_t s, int64_t e, chunk_out_t *o) {
    w->labs.n = 0;
    for (int64_t i = 0; i < n_set; i++) {
        int32_t q = states[i];
        for (int32_t j = a->final_off[q]; j < a->final_off[q + 1]; j++)
            if (vpush(&w->labs, a->final_labels[j])) return -1;
    }
    if (w->labs.n == 0) return 0;
    qsort(w->labs.v, (size_t)w->labs.n, sizeof(int32_t), cmp_i32);
    for (int64_t i = 0; i < w->labs.n; i++) {
        if (i > 0 && w->labs.v[i] == w->labs.v[i - 1]) continue;
        if (vpush(&o->m, (int32_t)s) || vpush(&o->m, (int32_t)e) || vpush(&o->m, w->labs.v[i]))
            return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* per-start simulation                                                */
/* ------------------------------------------------------------------ */

static int run_dfa_start(const fsm_t *a, setws_t *w, const uint8_t *x, int64_t n, int64_t s,
                         chunk_out_t *o) {
    int32_t q = a->q0;
    for (int64_t e = s; e < n; e++) {
        o->T++;
        int sym = dfa_symbol(a, x[e]);
        if (sym < 0) return 0;
        q = a->delta[(int64_t)q * a->n_symbols + sym];
        if (q < 0) return 0;
        if (a->prune && !a->coreach[q]) return 0;
        o->X++;
        if (emit_set(a, w, &q, 1, s, e, o)) return -1;
    }
    return 0;
}

static int run_nfa_start(const fsm_t *a, setws_t *w, const uint8_t *x, int64_t n, int64_t s,
                         chunk_out_t *o) {
    vec32 *S = &w->cur, *N = &w->nxt;
    if (!a->memo) {
        if (nfa_closure_q0(a, w, S)) return -1;
    }
    for (int64_t e = s; e < n; e++) {
        o->T++;
        if (e == s && a->memo) {
            const vec32 *f = &a->first[x[e]];
            N->n = 0;
            for (int64_t i = 0; i < f->n; i++)
                if (vpush(N, f->v[i])) return -1;
        } else {
            if (nfa_step(a, w, S, x[e], N)) return -1;
        }
        o->X += N->n;
        if (N->n == 0) return 0;
        if (emit_set(a, w, N->v, N->n, s, e, o)) return -1;
        vec32 *t = S; S = N; N = t;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* threading                                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    const fsm_t *a;
    const uint8_t *x;
    int64_t n, s_lo, s_hi, chunk;
    int64_t n_chunks;
    int64_t next; /* atomic */
    chunk_out_t *outs;
} job_t;

static void *worker(void *arg) {
    job_t *j = (job_t *)arg;
    const fsm_t *a = j->a;
    setws_t w;
    memset(&w, 0, sizeof(w));
    if (!a->is_dfa) {
        w.mark = (uint32_t *)calloc((size_t)a->n_states, sizeof(uint32_t));
        if (!w.mark) return NULL;
    }
    for (;;) {
        int64_t c = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (c >= j->n_chunks) break;
        chunk_out_t *o = &j->outs[c];
        int64_t lo = j->s_lo + c * j->chunk;
        int64_t hi = lo + j->chunk < j->s_hi ? lo + j->chunk : j->s_hi;
        for (int64_t s = lo; s < hi && !o->err; s++) {
            int r = a->is_dfa ? run_dfa_start(a, &w, j->x, j->n, s, o)
                              : run_nfa_start(a, &w, j->x, j->n, s, o);
            if (r) o->err = 1;
        }
    }
    free(w.mark);
    free(w.cur.v); free(w.nxt.v); free(w.labs.v);
    return NULL;
}

static int build_first(fsm_t *a) {
    setws_t w;
    memset(&w, 0, sizeof(w));
    w.mark = (uint32_t *)calloc((size_t)a->n_states, sizeof(uint32_t));
    if (!w.mark) return -1;
    if (nfa_closure_q0(a, &w, &a->z)) return -1;
    for (int c = 0; c < 256; c++)
        if (nfa_step(a, &w, &a->z, (uint8_t)c, &a->first[c])) return -1;
    free(w.mark); free(w.cur.v); free(w.nxt.v); free(w.labs.v);
    return 0;
}

static void fsm_free(fsm_t *a) {
    free(a->coreach);
    for (int c = 0; c < 256; c++) free(a->first[c].v);
    free(a->z.v);
}

static int64_t run(fsm_t *a, const uint8_t *x, int64_t n, int64_t s_lo, int64_t s_hi,
                   int32_t n_threads, int32_t **out_ptr, int64_t *work) {
    *out_ptr = NULL;
    if (s_lo < 0) s_lo = 0;
    if (s_hi > n) s_hi = n;
    if (compute_coreach(a)) { fsm_free(a); return -2; }
    if (!a->is_dfa && a->memo && build_first(a)) { fsm_free(a); return -2; }
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    job_t j;
    memset(&j, 0, sizeof(j));
    j.a = a; j.x = x; j.n = n; j.s_lo = s_lo; j.s_hi = s_hi;
    int64_t span = s_hi > s_lo ? s_hi - s_lo : 0;
    j.chunk = span / ((int64_t)n_threads * 16) + 1;
    if (j.chunk < 256) j.chunk = 256;
    j.n_chunks = span ? (span + j.chunk - 1) / j.chunk : 0;
    j.outs = (chunk_out_t *)calloc((size_t)(j.n_chunks + 1), sizeof(chunk_out_t));
    if (!j.outs) { fsm_free(a); return -2; }
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < n_threads; t++)
        if (pthread_create(&th[t], NULL, worker, &j) == 0) started++;
        else break;
    worker(&j);
    for (int t = 1; t <= started; t++) pthread_join(th[t], NULL);
    int64_t total = 0, T = 0, X = 0;
    int err = 0;
    for (int64_t c = 0; c < j.n_chunks; c++) {
        total += j.outs[c].m.n / 3;
        T += j.outs[c].T;
        X += j.outs[c].X;
        err |= j.outs[c].err;
    }
    int32_t *res = NULL;
    if (!err) {
        res = (int32_t *)malloc((size_t)(total * 3 + 1) * sizeof(int32_t));
        if (!res) err = 1;
    }
    int64_t pos = 0;
    for (int64_t c = 0; c < j.n_chunks; c++) {
        if (!err) memcpy(res + pos, j.outs[c].m.v, (size_t)j.outs[c].m.n * sizeof(int32_t));
        pos += j.outs[c].m.n;
        free(j.outs[c].m.v);
    }
    free(j.outs);
    fsm_free(a);
    if (err) { free(res); return -2; }
    if (work) { work[0] = T; work[1] = X; }
    *out_ptr = res;
    return total;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                               */
/* ------------------------------------------------------------------ */

/* Returns the number of matches (>= 0), -1 for an invalid descriptor, -2 when
 * memory runs out.  *out_ptr receives a malloc'ed int32[3*count] array
 * (release it with pfsm_oracle_free).  work[0] = T, work[1] = X. */
int64_t pfsm_oracle_dfa(int32_t n_states, int32_t n_symbols, int32_t q0,
                        const int16_t *byte_to_symbol, const int32_t *delta,
                        const int32_t *final_off, const int32_t *final_labels,
                        const uint8_t *x, int64_t n, int64_t s_lo, int64_t s_hi,
                        int32_t prune, int32_t n_threads, int32_t **out_ptr, int64_t *work) {
    *out_ptr = NULL;
    if (n_states <= 0 || n_symbols <= 0 || q0 < 0 || q0 >= n_states) return -1;
    if (!byte_to_symbol && n_symbols != 256) return -1;
    if (byte_to_symbol)
        for (int b = 0; b < 256; b++)
            if (byte_to_symbol[b] >= n_symbols) return -1;
    for (int64_t i = 0; i < (int64_t)n_states * n_symbols; i++)
        if (delta[i] < -1 || delta[i] >= n_states) return -1;
    fsm_t a;
    memset(&a, 0, sizeof(a));
    a.is_dfa = 1; a.n_states = n_states; a.n_symbols = n_symbols; a.q0 = q0;
    a.b2s = byte_to_symbol; a.delta = delta;
    a.final_off = final_off; a.final_labels = final_labels;
    a.prune = prune;
    return run(&a, x, n, s_lo, s_hi, n_threads, out_ptr, work);
}

int64_t pfsm_oracle_nfa(int32_t n_states, int32_t q0, int32_t n_classes,
                        const int32_t *row_ptr, const int32_t *edge_class, const int32_t *edge_dst,
                        const uint32_t *class_bits, const int32_t *final_off,
                        const int32_t *final_labels, const uint8_t *x, int64_t n, int64_t s_lo,
                        int64_t s_hi, int32_t prune, int32_t memo, int32_t n_threads,
                        int32_t **out_ptr, int64_t *work) {
    *out_ptr = NULL;
    if (n_states <= 0 || q0 < 0 || q0 >= n_states || row_ptr[0] != 0) return -1;
    for (int32_t q = 0; q < n_states; q++)
        if (row_ptr[q + 1] < row_ptr[q]) return -1;
    for (int32_t e = 0; e < row_ptr[n_states]; e++)
        if (edge_dst[e] < 0 || edge_dst[e] >= n_states || edge_class[e] < -1 ||
            edge_class[e] >= n_classes)
            return -1;
    fsm_t a;
    memset(&a, 0, sizeof(a));
    a.is_dfa = 0; a.n_states = n_states; a.q0 = q0; a.n_classes = n_classes;
    a.row_ptr = row_ptr; a.edge_class = edge_class; a.edge_dst = edge_dst;
    a.class_bits = class_bits;
    a.final_off = final_off; a.final_labels = final_labels;
    a.prune = prune; a.memo = memo;
    return run(&a, x, n, s_lo, s_hi, n_threads, out_ptr, work);
}

void pfsm_oracle_free(int32_t *p) { free(p); }
