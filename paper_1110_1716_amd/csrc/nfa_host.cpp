// NFA half of the host library: descriptor validation, the union of the
// loaded automaton with added patterns (Section III.A), the read-only caches
// derived from it, device upload and the launch of the NFA scan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "host_common.h"
#include "pfsm_nfa.h"
#include "stream.h"

namespace pfsmk {

namespace {

constexpr int64_t kPairBudget = 32ll << 20;   // states stored by the byte-pair cache
constexpr int64_t kClosureBudget = 64ll << 20;

// One automaton put into the handle: the loaded one, or a pattern added
// later.  Its states occupy global ids [first, first + n).
struct Part {
    int32_t first = 0, n = 0, q0 = 0;
    bool added = false;
    bool cut = false;                // removed: no longer reachable from the start
    std::vector<int32_t> disabled;   // removed labels (sorted)
};

// Device copy of every derived table; replaced as a whole on add/remove.
struct NfaTables {
    DevBuf rec, edges, class_bits, cl_off, cl, lab, f1_off, f1, e1_off, e1, p_bits, p_off, p_st, pl_off, p_lab;
    int32_t n_states = 0;
    int32_t pair_on = 0;
};

bool class_nonempty(const std::vector<uint32_t> &bits, int k) {
    for (int w = 0; w < 8; ++w)
        if (bits[(size_t)k * 8 + w]) return true;
    return false;
}

bool class_has(const std::vector<uint32_t> &bits, int k, int b) {
    return (bits[(size_t)k * 8 + (b >> 5)] >> (b & 31)) & 1u;
}

}  // namespace

struct NfaHost {
    // the union, global ids
    int32_t N = 0;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> out;  // per state: (class or -1, dst)
    std::vector<uint32_t> class_bits;                           // [n_classes * 8]
    std::vector<std::vector<int32_t>> labels;                   // per state, sorted unique
    std::vector<Part> parts;
    std::unique_ptr<NfaTables> tab;
    int n_blocks = 0;
    int occ = 0, cus = 0;
    Knobs knobs;
    WorkspacePool pool;
};

void NfaDeleter::operator()(NfaHost *p) const { delete p; }

namespace {

int validate(const pfsm_nfa_desc *d) {
    if (!d) return fail(PFSM_EINVAL, "NULL descriptor");
    const int32_t N = d->n_states;
    if (N < 1 || N >= (1 << 29)) return fail(PFSM_EINVAL, "n_states must be in [1, 2^29)");
    if (d->q0 < 0 || d->q0 >= N) return fail(PFSM_EINVAL, "q0 out of range");
    if (d->n_classes < 0 || d->n_classes >= (1 << 22)) return fail(PFSM_EINVAL, "n_classes must be in [0, 2^22)");
    if (!d->row_ptr) return fail(PFSM_EINVAL, "row_ptr is NULL");
    if (d->row_ptr[0] != 0) return fail(PFSM_EINVAL, "row_ptr[0] must be 0");
    for (int32_t q = 0; q < N; ++q)
        if (d->row_ptr[q + 1] < d->row_ptr[q]) return fail(PFSM_EINVAL, "row_ptr decreases at state %d", q);
    const int32_t E = d->row_ptr[N];
    if (E > 0 && (!d->edge_class || !d->edge_dst)) return fail(PFSM_EINVAL, "edge arrays are NULL");
    for (int32_t e = 0; e < E; ++e) {
        if (d->edge_dst[e] < 0 || d->edge_dst[e] >= N)
            return fail(PFSM_EINVAL, "edge_dst[%d] = %d out of range", e, d->edge_dst[e]);
        if (d->edge_class[e] < -1 || d->edge_class[e] >= d->n_classes)
            return fail(PFSM_EINVAL, "edge_class[%d] = %d out of range", e, d->edge_class[e]);
    }
    if (d->n_classes > 0 && !d->class_bits) return fail(PFSM_EINVAL, "class_bits is NULL");
    if (!d->final_off) return fail(PFSM_EINVAL, "final_off is NULL");
    if (d->final_off[0] != 0) return fail(PFSM_EINVAL, "final_off[0] must be 0");
    for (int32_t q = 0; q < N; ++q)
        if (d->final_off[q + 1] < d->final_off[q]) return fail(PFSM_EINVAL, "final_off decreases at state %d", q);
    const int32_t nnz = d->final_off[N];
    if (nnz > 0 && !d->final_labels) return fail(PFSM_EINVAL, "final_labels is NULL");
    for (int32_t i = 0; i < nnz; ++i)
        if (d->final_labels[i] < 0) return fail(PFSM_EINVAL, "label %d is negative", d->final_labels[i]);
    return PFSM_OK;
}

// Append a descriptor's states to the union as a new part.
int append_part(NfaHost *h, const pfsm_nfa_desc *d, bool added) {
    const int64_t newN = (int64_t)h->N + d->n_states;
    if (newN >= (1 << 29)) return fail(PFSM_EINVAL, "too many states in the union");
    const int32_t cbase = (int32_t)(h->class_bits.size() / 8);
    if ((int64_t)cbase + d->n_classes >= (1 << 22)) return fail(PFSM_EINVAL, "too many byte classes in the union");
    Part p;
    p.first = h->N;
    p.n = d->n_states;
    p.q0 = h->N + d->q0;
    p.added = added;
    h->out.resize(newN);
    h->labels.resize(newN);
    for (int32_t q = 0; q < d->n_states; ++q) {
        auto &o = h->out[h->N + q];
        for (int32_t e = d->row_ptr[q]; e < d->row_ptr[q + 1]; ++e) {
            const int32_t k = d->edge_class[e];
            o.push_back({k < 0 ? -1 : k + cbase, h->N + d->edge_dst[e]});
        }
        auto &l = h->labels[h->N + q];
        l.assign(d->final_labels + d->final_off[q], d->final_labels + d->final_off[q + 1]);
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    h->class_bits.insert(h->class_bits.end(), d->class_bits, d->class_bits + (size_t)d->n_classes * 8);
    h->N = (int32_t)newN;
    h->parts.push_back(std::move(p));
    return PFSM_OK;
}

const Part &part_of(const NfaHost *h, int32_t q) {
    // parts are in id order
    size_t lo = 0, hi = h->parts.size();
    while (hi - lo > 1) {
        const size_t mid = (lo + hi) / 2;
        if (h->parts[mid].first <= q) lo = mid;
        else hi = mid;
    }
    return h->parts[lo];
}

// Labels currently reported by the handle.
std::vector<int32_t> active_labels(const NfaHost *h) {
    std::vector<int32_t> all;
    for (const Part &p : h->parts) {
        if (p.cut) continue;
        for (int32_t q = p.first; q < p.first + p.n; ++q)
            for (int32_t l : h->labels[q])
                if (!std::binary_search(p.disabled.begin(), p.disabled.end(), l)) all.push_back(l);
    }
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    return all;
}

// Build every derived table from the union and upload it.
int rebuild(NfaHost *h, hipStream_t s) {
    const int32_t N = h->N;
    const int n_classes = (int)(h->class_bits.size() / 8);
    std::vector<uint8_t> cls_ok(n_classes);
    std::vector<int> cls_single(n_classes, -1);
    std::vector<uint8_t> cls_any(n_classes, 0);
    for (int k = 0; k < n_classes; ++k) {
        cls_ok[k] = class_nonempty(h->class_bits, k);
        int cnt = 0, last = -1;
        for (int b = 0; b < 256; ++b)
            if (class_has(h->class_bits, k, b)) {
                ++cnt;
                last = b;
            }
        if (cnt == 1) cls_single[k] = last;
        cls_any[k] = cnt == 256;
    }
    // enabled labels per state
    std::vector<std::vector<int32_t>> en(N);
    for (const Part &p : h->parts)
        for (int32_t q = p.first; q < p.first + p.n; ++q)
            for (int32_t l : h->labels[q])
                if (!std::binary_search(p.disabled.begin(), p.disabled.end(), l)) en[q].push_back(l);
    // live: reverse reachability to a state with an enabled label
    std::vector<std::vector<int32_t>> rev(N);
    for (int32_t q = 0; q < N; ++q)
        for (auto &e : h->out[q])
            if (e.first < 0 || cls_ok[e.first]) rev[e.second].push_back(q);
    std::vector<uint8_t> live(N, 0);
    std::vector<int32_t> work;
    for (int32_t q = 0; q < N; ++q)
        if (!en[q].empty()) {
            live[q] = 1;
            work.push_back(q);
        }
    for (size_t i = 0; i < work.size(); ++i)
        for (int32_t p : rev[work[i]])
            if (!live[p]) {
                live[p] = 1;
                work.push_back(p);
            }
    // epsilon closures restricted to live states (for states with epsilon edges)
    std::vector<int32_t> mark(N, -1);
    auto closure = [&](const std::vector<int32_t> &seed, int32_t stamp, std::vector<int32_t> &outv, bool only_live) {
        outv.clear();
        std::vector<int32_t> stack;
        for (int32_t q : seed)
            if (mark[q] != stamp) {
                mark[q] = stamp;
                stack.push_back(q);
            }
        while (!stack.empty()) {
            const int32_t q = stack.back();
            stack.pop_back();
            if (!only_live || live[q]) outv.push_back(q);
            for (auto &e : h->out[q])
                if (e.first < 0 && mark[e.second] != stamp) {
                    mark[e.second] = stamp;
                    stack.push_back(e.second);
                }
        }
        std::sort(outv.begin(), outv.end());
    };
    int32_t stamp = 0;
    auto word = [&](int32_t q) { return (uint32_t)q | (en[q].empty() ? 0u : kTgtFinal); };
    std::vector<int32_t> list_of(N, -1);  // closure list index of a state, -1 = itself
    std::vector<int32_t> cl_off(1, 0);
    std::vector<uint32_t> cl;
    std::vector<int32_t> tmp;
    for (int32_t q = 0; q < N; ++q) {
        bool has_eps = false;
        for (auto &e : h->out[q]) has_eps |= e.first < 0;
        if (!has_eps || !live[q]) continue;
        closure({q}, stamp++, tmp, true);
        if (tmp.size() == 1 && tmp[0] == q) continue;
        list_of[q] = (int32_t)cl_off.size() - 1;
        for (int32_t d : tmp) cl.push_back(word(d));
        cl_off.push_back((int32_t)cl.size());
        if ((int64_t)cl.size() > kClosureBudget) return fail(PFSM_ENOMEM, "epsilon closures exceed the budget");
    }
    auto target = [&](int32_t d) { return list_of[d] < 0 ? word(d) : (kTgtList | (uint32_t)list_of[d]); };
    // packed records
    std::vector<NfaRec> rec(N);
    std::vector<uint32_t> edges;
    std::vector<int32_t> lab;
    for (int32_t q = 0; q < N; ++q) {
        NfaRec &r = rec[q];
        std::memset(&r, 0, sizeof r);
        r.lab_off = (int32_t)lab.size();
        lab.insert(lab.end(), en[q].begin(), en[q].end());
        if (en[q].size() >= (size_t)kNfaLabelsMax) return fail(PFSM_EINVAL, "too many labels on state %d", q);
        r.info = (live[q] ? kRecLive : 0) | (en[q].empty() ? 0 : kRecFinal) | ((uint32_t)en[q].size() << 8);
        if (!live[q]) continue;
        std::vector<std::pair<uint32_t, uint32_t>> es;
        for (auto &e : h->out[q]) {
            if (e.first < 0 || !cls_ok[e.first] || !live[e.second]) continue;
            uint32_t test;
            if (cls_single[e.first] >= 0) test = (uint32_t)cls_single[e.first];
            else if (cls_any[e.first]) test = 1u << 8;
            else test = (2u << 8) | ((uint32_t)e.first << 10);
            es.push_back({test, target(e.second)});
        }
        r.n_edges = (int32_t)es.size();
        if (es.size() <= 2) {
            r.info |= kRecInline;
            if (es.size() > 0) {
                r.e0_test = es[0].first;
                r.e0_tgt = es[0].second;
            }
            if (es.size() > 1) {
                r.e1_test = es[1].first;
                r.e1_tgt = es[1].second;
            }
        } else {
            r.edge_off = (int32_t)(edges.size() / 2);
            for (auto &e : es) {
                edges.push_back(e.first);
                edges.push_back(e.second);
            }
        }
    }
    // start set: closure of the loaded automaton's q0 and of every added,
    // not removed pattern's q0 (the ancillary initial state's epsilon edges)
    std::vector<int32_t> seeds;
    for (const Part &p : h->parts)
        if (!p.cut) seeds.push_back(p.q0);
    std::vector<int32_t> Z;
    closure(seeds, stamp++, Z, false);
    // set after symbol c from a source set, as sorted live states
    auto step_set = [&](const std::vector<int32_t> &src, int c, std::vector<int32_t> &dst) {
        std::vector<int32_t> tg;
        for (int32_t q : src)
            for (auto &e : h->out[q])
                if (e.first >= 0 && class_has(h->class_bits, e.first, c)) tg.push_back(e.second);
        closure(tg, stamp++, dst, true);
    };
    auto labels_of = [&](const std::vector<int32_t> &set, std::vector<int32_t> &outl) {
        outl.clear();
        for (int32_t q : set) outl.insert(outl.end(), en[q].begin(), en[q].end());
        std::sort(outl.begin(), outl.end());
        outl.erase(std::unique(outl.begin(), outl.end()), outl.end());
    };
    std::vector<std::vector<int32_t>> first1(256);
    std::vector<int32_t> f1_off(257, 0), e1_off(257, 0), e1;
    std::vector<uint32_t> f1;
    std::vector<int32_t> lt;
    for (int c = 0; c < 256; ++c) {
        step_set(Z, c, first1[c]);
        for (int32_t q : first1[c]) f1.push_back(word(q));
        f1_off[c + 1] = (int32_t)f1.size();
        labels_of(first1[c], lt);
        e1.insert(e1.end(), lt.begin(), lt.end());
        e1_off[c + 1] = (int32_t)e1.size();
    }
    // byte-pair cache
    std::vector<uint32_t> p_bits(2048, 0);
    std::vector<int32_t> p_off(65537, 0), pl_off(65537, 0), p_lab;
    std::vector<uint32_t> p_st;
    bool pair_on = h->knobs.pair_cache != 0;
    if (pair_on) {
        std::vector<int32_t> s2;
        for (int c1 = 0; c1 < 256 && pair_on; ++c1) {
            for (int c2 = 0; c2 < 256; ++c2) {
                const int p = c1 * 256 + c2;
                if (!first1[c1].empty()) {
                    step_set(first1[c1], c2, s2);
                    for (int32_t q : s2) p_st.push_back(word(q));
                    labels_of(s2, lt);
                    p_lab.insert(p_lab.end(), lt.begin(), lt.end());
                    if (!s2.empty() || !lt.empty()) p_bits[p >> 5] |= 1u << (p & 31);
                }
                p_off[p + 1] = (int32_t)p_st.size();
                pl_off[p + 1] = (int32_t)p_lab.size();
            }
            if ((int64_t)p_st.size() + (int64_t)p_lab.size() > kPairBudget) pair_on = false;  // ends the loop
        }
    }
    if (!pair_on) {
        p_st.clear();
        p_lab.clear();
        std::fill(p_off.begin(), p_off.end(), 0);
        std::fill(pl_off.begin(), pl_off.end(), 0);
        std::fill(p_bits.begin(), p_bits.end(), 0);
    }

    auto t = std::make_unique<NfaTables>();
    t->n_states = N;
    t->pair_on = pair_on ? 1 : 0;
    int rc;
    if ((rc = t->rec.upload(rec.data(), rec.size(), s))) return rc;
    if ((rc = t->edges.upload(edges.data(), edges.size(), s))) return rc;
    if ((rc = t->class_bits.upload(h->class_bits.data(), h->class_bits.size(), s))) return rc;
    if ((rc = t->cl_off.upload(cl_off.data(), cl_off.size(), s))) return rc;
    if ((rc = t->cl.upload(cl.data(), cl.size(), s))) return rc;
    if ((rc = t->lab.upload(lab.data(), lab.size(), s))) return rc;
    if ((rc = t->f1_off.upload(f1_off.data(), f1_off.size(), s))) return rc;
    if ((rc = t->f1.upload(f1.data(), f1.size(), s))) return rc;
    if ((rc = t->e1_off.upload(e1_off.data(), e1_off.size(), s))) return rc;
    if ((rc = t->e1.upload(e1.data(), e1.size(), s))) return rc;
    if ((rc = t->p_bits.upload(p_bits.data(), p_bits.size(), s))) return rc;
    if ((rc = t->p_off.upload(p_off.data(), p_off.size(), s))) return rc;
    if ((rc = t->p_st.upload(p_st.data(), p_st.size(), s))) return rc;
    if ((rc = t->pl_off.upload(pl_off.data(), pl_off.size(), s))) return rc;
    if ((rc = t->p_lab.upload(p_lab.data(), p_lab.size(), s))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    // Scans already issued on any stream keep reading the old tables: wait
    // for them before the old tables are released.
    HIP_TRY(hipDeviceSynchronize());
    h->tab = std::move(t);
    return PFSM_OK;
}

int grid_size(NfaHost *h) {
    int occ = 0, cus = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, nfa_kernel_fn(false), kNfaThreads, 0));
    int rc = device_cus(&cus);
    if (rc) return rc;
    if (occ < 1) return fail(PFSM_EINVAL, "NFA scan kernel does not fit on a compute unit");
    h->occ = occ;
    h->cus = cus;
    h->n_blocks = grid_blocks(occ, cus, h->knobs.wpc);
    return PFSM_OK;
}

}  // namespace

int nfa_load(const pfsm_nfa_desc *d, hipStream_t s, NfaPtr *out) {
    int rc = validate(d);
    if (rc) return rc;
    NfaPtr h(new (std::nothrow) NfaHost);
    if (!h) return fail(PFSM_ENOMEM, "handle");
    if ((rc = append_part(h.get(), d, false))) return rc;
    if ((rc = rebuild(h.get(), s))) return rc;
    if ((rc = grid_size(h.get()))) return rc;
    *out = std::move(h);
    return PFSM_OK;
}

int nfa_add_pattern(NfaHost *h, const pfsm_nfa_desc *p, hipStream_t s) {
    int rc = validate(p);
    if (rc) return rc;
    const std::vector<int32_t> have = active_labels(h);
    for (int32_t i = 0; i < p->final_off[p->n_states]; ++i)
        if (std::binary_search(have.begin(), have.end(), p->final_labels[i]))
            return fail(PFSM_EEXIST, "label %d is already present", p->final_labels[i]);
    if ((rc = append_part(h, p, true))) return rc;
    return rebuild(h, s);
}

int nfa_remove_pattern(NfaHost *h, int32_t label, hipStream_t s) {
    bool found = false;
    for (Part &p : h->parts) {
        if (p.cut || std::binary_search(p.disabled.begin(), p.disabled.end(), label)) continue;
        bool carries = false;
        for (int32_t q = p.first; q < p.first + p.n && !carries; ++q)
            carries = std::binary_search(h->labels[q].begin(), h->labels[q].end(), label);
        if (!carries) continue;
        found = true;
        if (p.added) {
            p.cut = true;
        } else {
            p.disabled.insert(std::upper_bound(p.disabled.begin(), p.disabled.end(), label), label);
        }
    }
    if (!found) return fail(PFSM_ENOENT, "no pattern carries label %d", label);
    return rebuild(h, s);
}

int nfa_grid_blocks(NfaHost *h) { return h->n_blocks; }

Knobs *nfa_knobs(NfaHost *h) { return &h->knobs; }

int nfa_occupancy(NfaHost *h) { return h->occ; }

int nfa_apply_knobs(NfaHost *h, bool tables, hipStream_t s) {
    h->n_blocks = grid_blocks(h->occ, h->cus, h->knobs.wpc);
    if (!tables) return PFSM_OK;
    HIP_TRY(hipDeviceSynchronize());
    return rebuild(h, s);
}

WorkspacePool *nfa_pool(NfaHost *h) { return &h->pool; }

namespace {

// The workspace of stream s with replay scratch sized for the current union.
int nfa_workspace(NfaHost *h, hipStream_t s, Workspace **out) {
    Workspace *w;
    int rc = h->pool.get(s, h->n_blocks, &w);
    if (rc) return rc;
    NfaTables *t = h->tab.get();
    const int64_t words_front = (int64_t)h->n_blocks * 2 * t->n_states;
    const int64_t words_bits = (int64_t)h->n_blocks * ((t->n_states + 31) / 32);
    if (w->big_states < t->n_states) {
        HIP_TRY(hipStreamSynchronize(s));
        if (w->big_front) HIP_TRY(hipFree(w->big_front));
        if (w->big_bits) HIP_TRY(hipFree(w->big_bits));
        w->big_front = w->big_bits = nullptr;
        w->big_states = 0;
        HIP_TRY(hipMalloc(&w->big_front, sizeof(uint32_t) * words_front));
        HIP_TRY(hipMalloc(&w->big_bits, sizeof(uint32_t) * words_bits));
        HIP_TRY(hipMemset(w->big_bits, 0, sizeof(uint32_t) * words_bits));
        HIP_TRY(hipDeviceSynchronize());
        w->big_states = t->n_states;
    }
    *out = w;
    return PFSM_OK;
}

// The scan's view of the current tables.
void nfa_table_args(NfaHost *h, NfaArgs &a) {
    NfaTables *t = h->tab.get();
    a.n_states = t->n_states;
    a.rec = t->rec.as<NfaRec>();
    a.edges = t->edges.as<uint32_t>();
    a.class_bits = t->class_bits.as<uint32_t>();
    a.cl_off = t->cl_off.as<int32_t>();
    a.cl = t->cl.as<uint32_t>();
    a.lab = t->lab.as<int32_t>();
    a.f1_off = t->f1_off.as<int32_t>();
    a.f1 = t->f1.as<uint32_t>();
    a.e1_off = t->e1_off.as<int32_t>();
    a.e1 = t->e1.as<int32_t>();
    a.pair_on = t->pair_on;
    a.p_bits = t->p_bits.as<uint32_t>();
    a.p_off = t->p_off.as<int32_t>();
    a.p_st = t->p_st.as<uint32_t>();
    a.pl_off = t->pl_off.as<int32_t>();
    a.p_lab = t->p_lab.as<int32_t>();
}

}  // namespace

int nfa_resume(NfaHost *h, const uint8_t *x, int64_t n, int32_t base, const CarrySet &in, int64_t *cnt,
               const int64_t *off, MatchOut *out, int64_t cap, const CarryOut &carry, int write, hipStream_t s) {
    Workspace *w;
    int rc = nfa_workspace(h, s, &w);
    if (rc) return rc;
    NfaResumeArgs r;
    std::memset(&r, 0, sizeof r);
    nfa_table_args(h, r.a);
    r.a.x = x;
    r.a.n = n;
    r.a.out = out;
    r.a.cap = cap;
    r.a.big_front = w->big_front;
    r.a.big_bits = w->big_bits;
    r.a.carry = carry;
    r.base = base;
    r.write = write;
    r.in = in;
    r.cnt = cnt;
    r.off = off;
    HIP_TRY(launch_nfa_resume(r, h->n_blocks, s));
    return PFSM_OK;
}

int nfa_launch(NfaHost *h, const uint8_t *x, int64_t n, const SegPlan *plan, int64_t seg, MatchOut *out,
               int64_t cap, int64_t *d_total, hipStream_t s, const int64_t *d_base, const CarryOut *carry) {
    Workspace *w;
    int rc = nfa_workspace(h, s, &w);
    if (rc) return rc;
    NfaArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = x;
    a.n = n;
    nfa_table_args(h, a);
    a.out = out;
    a.cap = cap;
    a.total = d_total;
    a.ctl = w->ctl;
    a.bstats = w->bstats;
    a.big_front = w->big_front;
    a.big_bits = w->big_bits;
    int grid = h->n_blocks;
    if (plan) {
        a.plan = *plan;
        a.seg = seg;
    } else {
        int rounds;
        plan_segments(n, h->n_blocks, h->knobs.segment > 0 ? h->knobs.segment : kNfaSegMax, kNfaSegFloor, &a.seg,
                      &rounds);
        const int64_t n_segs = (n + a.seg - 1) / a.seg;
        if ((rc = grow_lb(w, (int)n_segs))) return rc;
        a.n_segs = (int32_t)n_segs;
        a.plan.base_dev = d_base;
        grid = (int)std::min<int64_t>(n_segs, h->n_blocks);
    }
    if (carry) a.carry = *carry;
    // after any growth of the look-back words above
    a.lb = w->lb;
    a.lb_cap = w->lb_cap;
    void *args[] = {&a};
    HIP_TRY(hipLaunchKernel(nfa_kernel_fn(carry != nullptr), dim3(grid), dim3(kNfaThreads), args, 0, s));
    w->last_grid = grid;
    h->pool.mark(w);
    return PFSM_OK;
}

int nfa_scan_async(NfaHost *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap, int64_t *d_total,
                   hipStream_t s) {
    return nfa_launch(h, x, n, nullptr, 0, out, cap, d_total, s);
}

}  // namespace pfsmk
