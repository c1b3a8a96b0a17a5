// NFA half of the host library: descriptor validation, the union of the
// loaded automaton with added patterns (Section III.A), the read-only caches
// derived from it, device upload and the launch of the NFA scan.
//
// Edits are incremental.  A part (the loaded automaton or an added pattern)
// whose initial state has no incoming edge is split into components: the
// pieces of its graph that stay connected once that initial state is taken
// away (one signature chain each, for a union built under an ancillary
// initial state).  Every component owns fixed regions of the packed device
// arrays and its own contribution to the first-symbol and byte-pair tables.
// An added pattern appends its components; a removed label recomputes only
// the components that carry it (their tables can only shrink, so they are
// rewritten inside their regions); a removed added pattern drops its
// components' contributions.  The start tables are then reassembled from the
// contributions and every changed range is copied into the same device
// buffers, so table addresses stay fixed while the arrays have room.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <iterator>
#include <unordered_map>
#include <vector>

#include "dfa_defer.h"
#include "host_common.h"
#include "pfsm_nfa.h"
#include "stream.h"

namespace pfsmk {

namespace {

constexpr int64_t kPairBudget = 32ll << 20;   // states and labels stored by the byte-pair cache
constexpr int64_t kClosureBudget = 64ll << 20;

// One automaton put into the handle: the loaded one, or a pattern added
// later.  Its states occupy global ids [first, first + n).
struct Part {
    int32_t first = 0, n = 0, q0 = 0;
    bool added = false;
    bool cut = false;                // removed: no longer reachable from the start
    bool hub = false;                // q0 has no incoming edge: its components stand apart
    std::vector<int32_t> disabled;   // removed labels (sorted)
    std::vector<int32_t> comps;      // its components
    std::vector<int32_t> labs;       // labels its states carry (sorted unique)
};

// What a component adds to the start tables: the live states (as target
// words) and labels after the first symbol, for each byte that has any, and
// the same after the first two symbols, for each byte pair that has any.
struct Contrib {
    std::vector<int32_t> f1_b;                    // bytes, ascending
    std::vector<int32_t> f1_off, e1_off;          // [f1_b.size() + 1]
    std::vector<uint32_t> f1;
    std::vector<int32_t> e1;
    std::vector<int32_t> pr;                      // pair ids c1 * 256 + c2, ascending
    std::vector<int32_t> pr_st_off, pr_lab_off;   // [pr.size() + 1]
    std::vector<uint32_t> pr_st;
    std::vector<int32_t> pr_lab;
};

// A component and its regions of the packed arrays (element offsets).
struct Comp {
    int32_t part = 0;
    std::vector<int32_t> states;          // global ids, ascending
    int32_t list_at = 0, list_cap = 0;    // closure lists (one spare index)
    int32_t cl_at = 0, cl_cap = 0;        // closure list words
    int32_t edge_at = 0, edge_cap = 0;    // out-of-record edges, (test, target) pairs
    int32_t lab_at = 0, lab_cap = 0;      // label entries
    Contrib start;
};

// A packed device array and its host copy.  The host copy is the authority;
// after an edit its dirty range is copied into the device buffer, which is
// replaced (and the old one kept until the handle is freed) only when the
// array outgrows it.
template <typename T>
struct Packed {
    std::vector<T> host;
    void *dev = nullptr;
    size_t cap = 0;  // elements the device buffer holds
    size_t lo = SIZE_MAX, hi = 0;
    void dirty(size_t a, size_t b) {
        lo = std::min(lo, a);
        hi = std::max(hi, b);
    }
    void all_dirty() { dirty(0, host.size()); }
    T *ptr() const { return static_cast<T *>(dev); }
};

// A byte class as its 256-bit set, for sharing ids across the union.
struct ClassKey {
    uint32_t w[8];
    bool operator==(const ClassKey &o) const { return std::memcmp(w, o.w, sizeof w) == 0; }
};
struct ClassKeyHash {
    size_t operator()(const ClassKey &k) const {
        uint64_t x = 1469598103934665603ull;
        for (uint32_t v : k.w) x = (x ^ v) * 1099511628211ull;
        return (size_t)x;
    }
};

bool class_has(const std::vector<uint32_t> &bits, int k, int b) {
    return (bits[(size_t)k * 8 + (b >> 5)] >> (b & 31)) & 1u;
}

}  // namespace

struct NfaHost {
    // the union, global ids
    int32_t N = 0;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> out;  // per state: (class or -1, dst)
    std::vector<uint32_t> class_bits;                           // [n_classes * 8]
    std::vector<uint8_t> cls_ok;                                // class has a byte
    std::vector<int16_t> cls_single;                            // its only byte, or -1
    std::vector<uint8_t> cls_any;                               // class is every byte
    std::unordered_map<ClassKey, int32_t, ClassKeyHash> class_id;  // byte set: its class id
    std::vector<std::vector<int32_t>> labels;                   // per state, sorted unique
    std::vector<int32_t> comp_of;                               // per state: component, -1 = a hub q0
    std::vector<Part> parts;
    std::vector<Comp> comps;
    // packed arrays (layout in pfsm_dev.h, NfaArgs)
    Packed<NfaRec> rec;
    Packed<uint32_t> edges, cl, f1, p_bits, p_st, cls;
    Packed<int32_t> cl_off, lab, f1_off, e1_off, e1, p_lab;
    Packed<PairRange> p_rng;
    int32_t n_lists = 0;  // closure list indices in use (cl_off has one more entry)
    int32_t pair_on = 0;  // the byte-pair cache is in use
    uint64_t layout_epoch = 0;
    std::vector<void *> retired;  // device buffers replaced by larger ones
    std::unordered_map<int32_t, int32_t> enabled;  // label: parts in the union that report it
    // byte-pair cache bookkeeping: per pair, the components that reach it
    // and the capacities of its regions
    std::vector<std::vector<int32_t>> pair_reach;
    std::vector<int32_t> st_cap, lab_cap;
    int64_t pair_words = 0;    // entries in use (states and labels)
    int64_t pair_garbage = 0;  // entries left behind by moved lists
    std::vector<uint32_t> a_st;
    std::vector<int32_t> a_lb;
    // closure scratch
    std::vector<int32_t> mark;
    int32_t stamp = 0;
    int n_blocks = 0;
    int occ = 0, cus = 0;
    Knobs knobs;
    WorkspacePool pool;

    ~NfaHost() {
        void *bufs[] = {rec.dev, edges.dev, cl.dev, f1.dev, p_bits.dev, p_st.dev, cls.dev, cl_off.dev,
                        lab.dev, f1_off.dev, e1_off.dev, e1.dev, p_rng.dev, p_lab.dev};
        for (void *p : bufs)
            if (p) (void)hipFree(p);
        for (void *p : retired) (void)hipFree(p);
    }
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

// Append a descriptor's states to the union as a new part, and split the
// part into components.
int append_part(NfaHost *h, const pfsm_nfa_desc *d, bool added) {
    const int64_t newN = (int64_t)h->N + d->n_states;
    if (newN >= (1 << 29)) return fail(PFSM_EINVAL, "too many states in the union");
    // byte classes: one id per distinct byte set across the union
    std::vector<int32_t> cmap(d->n_classes);
    for (int32_t k = 0; k < d->n_classes; ++k) {
        ClassKey key;
        std::memcpy(key.w, d->class_bits + (size_t)k * 8, sizeof key.w);
        auto it = h->class_id.find(key);
        if (it == h->class_id.end()) {
            const int32_t id = (int32_t)(h->class_bits.size() / 8);
            if (id >= (1 << 22)) return fail(PFSM_EINVAL, "too many byte classes in the union");
            h->class_bits.insert(h->class_bits.end(), key.w, key.w + 8);
            int cnt = 0, last = -1;
            for (int bb = 0; bb < 256; ++bb)
                if (class_has(h->class_bits, id, bb)) {
                    ++cnt;
                    last = bb;
                }
            h->cls_ok.push_back(cnt > 0);
            h->cls_single.push_back((int16_t)(cnt == 1 ? last : -1));
            h->cls_any.push_back(cnt == 256);
            it = h->class_id.emplace(key, id).first;
        }
        cmap[k] = it->second;
    }
    const int32_t first = h->N;
    Part p;
    p.first = first;
    p.n = d->n_states;
    p.q0 = first + d->q0;
    p.added = added;
    h->out.resize(newN);
    h->labels.resize(newN);
    h->comp_of.resize(newN, -1);
    h->mark.resize(newN, -1);
    for (int32_t q = 0; q < d->n_states; ++q) {
        auto &o = h->out[first + q];
        for (int32_t e = d->row_ptr[q]; e < d->row_ptr[q + 1]; ++e) {
            const int32_t k = d->edge_class[e];
            o.push_back({k < 0 ? -1 : cmap[k], first + d->edge_dst[e]});
        }
        auto &l = h->labels[first + q];
        l.assign(d->final_labels + d->final_off[q], d->final_labels + d->final_off[q + 1]);
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    for (int32_t q = first; q < (int32_t)newN; ++q) p.labs.insert(p.labs.end(), h->labels[q].begin(), h->labels[q].end());
    std::sort(p.labs.begin(), p.labs.end());
    p.labs.erase(std::unique(p.labs.begin(), p.labs.end()), p.labs.end());
    for (int32_t l : p.labs) ++h->enabled[l];
    h->N = (int32_t)newN;
    // components: union-find over the part's edges, without q0 when nothing
    // enters it
    p.hub = true;
    for (int32_t q = first; q < (int32_t)newN && p.hub; ++q)
        for (auto &e : h->out[q])
            if (e.second == p.q0) {
                p.hub = false;
                break;
            }
    std::vector<int32_t> uf(d->n_states);
    std::iota(uf.begin(), uf.end(), 0);
    auto find = [&](int32_t a) {
        while (uf[a] != a) a = uf[a] = uf[uf[a]];
        return a;
    };
    for (int32_t q = first; q < (int32_t)newN; ++q) {
        if (p.hub && q == p.q0) continue;
        for (auto &e : h->out[q]) {
            const int32_t a = find(q - first), b = find(e.second - first);
            if (a != b) uf[std::max(a, b)] = std::min(a, b);
        }
    }
    std::vector<int32_t> root_comp(d->n_states, -1);
    const int32_t pi = (int32_t)h->parts.size();
    for (int32_t q = first; q < (int32_t)newN; ++q) {
        if (p.hub && q == p.q0) continue;
        const int32_t r = find(q - first);
        if (root_comp[r] < 0) {
            root_comp[r] = (int32_t)h->comps.size();
            h->comps.emplace_back();
            h->comps.back().part = pi;
            p.comps.push_back(root_comp[r]);
        }
        h->comps[root_comp[r]].states.push_back(q);
        h->comp_of[q] = root_comp[r];
    }
    h->parts.push_back(std::move(p));
    return PFSM_OK;
}

// The tables of one component, from its part's enabled labels.  `place`:
// the component is new and its regions go at the ends of the arrays;
// otherwise they are rewritten inside the regions it already has.
int compute_comp(NfaHost *h, int32_t ci, bool place) {
    Comp &c = h->comps[ci];
    const Part &p = h->parts[c.part];
    const std::vector<int32_t> &S = c.states;
    const int32_t n = (int32_t)S.size();
    auto loc = [&](int32_t q) { return (int32_t)(std::lower_bound(S.begin(), S.end(), q) - S.begin()); };
    // enabled labels and liveness (reverse search inside the component)
    std::vector<std::vector<int32_t>> en(n);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t l : h->labels[S[i]])
            if (!std::binary_search(p.disabled.begin(), p.disabled.end(), l)) en[i].push_back(l);
    std::vector<std::vector<int32_t>> rev(n);
    for (int32_t i = 0; i < n; ++i)
        for (auto &e : h->out[S[i]])
            if (e.first < 0 || h->cls_ok[e.first]) rev[loc(e.second)].push_back(i);
    std::vector<uint8_t> live(n, 0);
    std::vector<int32_t> work;
    for (int32_t i = 0; i < n; ++i)
        if (!en[i].empty()) {
            live[i] = 1;
            work.push_back(i);
        }
    for (size_t k = 0; k < work.size(); ++k)
        for (int32_t j : rev[work[k]])
            if (!live[j]) {
                live[j] = 1;
                work.push_back(j);
            }
    auto is_live = [&](int32_t q) { return h->comp_of[q] == ci && live[loc(q)]; };
    // epsilon closure of a seed set (global ids), sorted; only_live keeps
    // live states only
    auto closure = [&](const std::vector<int32_t> &seed, std::vector<int32_t> &outv, bool only_live) {
        if (++h->stamp == INT32_MAX) {
            std::fill(h->mark.begin(), h->mark.end(), -1);
            h->stamp = 0;
        }
        const int32_t st = h->stamp;
        outv.clear();
        std::vector<int32_t> stack;
        for (int32_t q : seed)
            if (h->mark[q] != st) {
                h->mark[q] = st;
                stack.push_back(q);
            }
        while (!stack.empty()) {
            const int32_t q = stack.back();
            stack.pop_back();
            if (!only_live || is_live(q)) outv.push_back(q);
            for (auto &e : h->out[q])
                if (e.first < 0 && h->mark[e.second] != st) {
                    h->mark[e.second] = st;
                    stack.push_back(e.second);
                }
        }
        std::sort(outv.begin(), outv.end());
    };
    auto word = [&](int32_t q) { return (uint32_t)q | (en[loc(q)].empty() ? 0u : kTgtFinal); };
    // closure lists of live states with epsilon edges
    std::vector<int32_t> list_of(n, -1), l_off(1, 0);
    std::vector<uint32_t> l_words;
    std::vector<int32_t> tmp;
    const int32_t list_at = place ? h->n_lists : c.list_at;
    for (int32_t i = 0; i < n; ++i) {
        bool has_eps = false;
        for (auto &e : h->out[S[i]]) has_eps |= e.first < 0;
        if (!has_eps || !live[i]) continue;
        closure({S[i]}, tmp, true);
        if (tmp.size() == 1 && tmp[0] == S[i]) continue;
        list_of[i] = list_at + (int32_t)l_off.size() - 1;
        for (int32_t d : tmp) l_words.push_back(word(d));
        l_off.push_back((int32_t)l_words.size());
        if ((int64_t)l_words.size() + (int64_t)h->cl.host.size() > kClosureBudget)
            return fail(PFSM_ENOMEM, "epsilon closures exceed the budget");
    }
    auto target = [&](int32_t d) {
        const int32_t j = loc(d);
        return list_of[j] < 0 ? word(d) : (kTgtList | (uint32_t)list_of[j]);
    };
    // records, out-of-record edges, labels
    const int32_t n_lists = (int32_t)l_off.size() - 1;
    int32_t n_edge = 0, n_lab = 0;
    std::vector<NfaRec> recs(n);
    std::vector<uint32_t> e_words;
    std::vector<int32_t> labs;
    const int32_t edge_at = place ? (int32_t)(h->edges.host.size() / 2) : c.edge_at;
    const int32_t lab_at = place ? (int32_t)h->lab.host.size() : c.lab_at;
    for (int32_t i = 0; i < n; ++i) {
        NfaRec &r = recs[i];
        std::memset(&r, 0, sizeof r);
        r.lab_off = lab_at + n_lab;
        labs.insert(labs.end(), en[i].begin(), en[i].end());
        n_lab += (int32_t)en[i].size();
        if (en[i].size() >= (size_t)kNfaLabelsMax) return fail(PFSM_EINVAL, "too many labels on state %d", S[i]);
        r.info = (live[i] ? kRecLive : 0) | (en[i].empty() ? 0 : kRecFinal) | ((uint32_t)en[i].size() << 8);
        if (!live[i]) continue;
        std::vector<std::pair<uint32_t, uint32_t>> es;
        for (auto &e : h->out[S[i]]) {
            if (e.first < 0 || !h->cls_ok[e.first] || !is_live(e.second)) continue;
            uint32_t test;
            if (h->cls_single[e.first] >= 0) test = (uint32_t)h->cls_single[e.first];
            else if (h->cls_any[e.first]) test = 1u << 8;
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
            r.edge_off = edge_at + n_edge;
            for (auto &e : es) {
                e_words.push_back(e.first);
                e_words.push_back(e.second);
            }
            n_edge += (int32_t)es.size();
        }
    }
    // Gap states: a run of consecutive ids q, q + 1, ... each passing any
    // byte to the next and sharing one other edge E, the last with E alone
    // (a bounded .{0,m} gap before E).  Marked from the highest id down, so
    // that the remaining length of the next state is known.
    {
        auto is_any = [](uint32_t t) { return ((t >> 8) & 3u) == 1u; };
        std::vector<int32_t> rem(n, -1);
        for (int32_t i = n - 1; i >= 0; --i) {
            NfaRec &r = recs[i];
            if (!live[i] || !en[i].empty() || !(r.info & kRecInline)) continue;
            if (r.n_edges == 1) {
                if (!is_any(r.e0_test)) rem[i] = 0;  // may end a gap
                continue;
            }
            if (r.n_edges != 2 || i + 1 >= n || S[i + 1] != S[i] + 1 || rem[i + 1] < 0) continue;
            const uint32_t next = (uint32_t)S[i + 1];
            int ai = -1;
            if (is_any(r.e1_test) && r.e1_tgt == next) ai = 1;
            else if (is_any(r.e0_test) && r.e0_tgt == next) ai = 0;
            if (ai < 0) continue;
            const uint32_t et = ai == 1 ? r.e0_test : r.e1_test, eg = ai == 1 ? r.e0_tgt : r.e1_tgt;
            const NfaRec &nr = recs[i + 1];  // its e0 is its E (ends and marked gap states)
            if (is_any(et) || nr.e0_test != et || nr.e0_tgt != eg) continue;
            r.e0_test = et;
            r.e0_tgt = eg;
            r.e1_test = 1u << 8;
            r.e1_tgt = next;
            r.info |= kRecGap;
            r.edge_off = rem[i + 1] + 1;
            rem[i] = rem[i + 1] + 1;
        }
        // Gap states whose E leads into a simple chain: from E's target on,
        // every state passes exactly one edge to a plain state (its epsilon
        // closure is itself) and is not final, up to a last state with no
        // edge, which is final, and every state after the first has only
        // its predecessor's edge coming in.  The attempts E starts at
        // different bytes then never share a state, chains after different
        // first states never meet, and each attempt reports only at its
        // chain's end.
        // Such a record (never final itself) keeps the chain's first edge
        // test in lab_off.
        for (int32_t i = 0; i < n; ++i) {
            NfaRec &r = recs[i];
            if (!(r.info & kRecGap) || (r.e0_tgt & kTgtList)) continue;
            uint32_t t0 = 0;
            bool ok = false;
            int32_t q = (int32_t)(r.e0_tgt & kStateMask);
            for (int32_t len = 0; len <= n; ++len) {
                if (h->comp_of[q] != ci) break;
                const int32_t j = loc(q);
                const NfaRec &u = recs[j];
                if (!live[j] || !(u.info & kRecInline) || (u.info & kRecGap)) break;
                const bool fin = !en[j].empty();
                if (u.n_edges == 0) {
                    ok = fin;
                    break;
                }
                if (fin || u.n_edges != 1 || (u.e0_tgt & kTgtList)) break;
                if (len > 0 && rev[j].size() != 1) break;  // another way in: chains could merge
                if (len == 0) t0 = u.e0_test;
                q = (int32_t)(u.e0_tgt & kStateMask);
            }
            if (!ok) continue;
            r.info |= kRecGapFin;
            r.lab_off = (int32_t)t0;
        }
    }
    // regions: new ones at the ends; old ones must hold the new tables
    if (place) {
        c.list_at = list_at;
        c.list_cap = n_lists + 1;
        c.cl_at = (int32_t)h->cl.host.size();
        c.cl_cap = (int32_t)l_words.size();
        c.edge_at = edge_at;
        c.edge_cap = n_edge;
        c.lab_at = lab_at;
        c.lab_cap = n_lab;
        h->n_lists += c.list_cap;
        h->cl_off.host.resize((size_t)h->n_lists + 1);
        h->cl.host.resize(h->cl.host.size() + l_words.size());
        h->edges.host.resize(h->edges.host.size() + 2 * (size_t)n_edge);
        h->lab.host.resize(h->lab.host.size() + (size_t)n_lab);
    } else if (n_lists + 1 > c.list_cap || (int32_t)l_words.size() > c.cl_cap || n_edge > c.edge_cap ||
               n_lab > c.lab_cap) {
        return fail(PFSM_EINVAL, "component %d outgrew its regions", ci);
    }
    for (int32_t i = 0; i < n; ++i) h->rec.host[S[i]] = recs[i];
    h->rec.dirty(S.front(), S.back() + 1);
    for (int32_t j = 0; j <= n_lists; ++j) h->cl_off.host[c.list_at + j] = c.cl_at + l_off[j];
    for (int32_t j = n_lists + 1; j < c.list_cap; ++j) h->cl_off.host[c.list_at + j] = c.cl_at + c.cl_cap;
    h->cl_off.host[(size_t)h->n_lists] = (int32_t)h->cl.host.size();
    h->cl_off.dirty(c.list_at, c.list_at + c.list_cap);
    h->cl_off.dirty(h->n_lists, h->n_lists + 1);
    std::fill(h->cl.host.begin() + c.cl_at, h->cl.host.begin() + c.cl_at + c.cl_cap, 0u);
    std::copy(l_words.begin(), l_words.end(), h->cl.host.begin() + c.cl_at);
    h->cl.dirty(c.cl_at, c.cl_at + c.cl_cap);
    std::fill(h->edges.host.begin() + 2 * (size_t)c.edge_at, h->edges.host.begin() + 2 * (size_t)(c.edge_at + c.edge_cap),
              0u);
    std::copy(e_words.begin(), e_words.end(), h->edges.host.begin() + 2 * (size_t)c.edge_at);
    h->edges.dirty(2 * (size_t)c.edge_at, 2 * (size_t)(c.edge_at + c.edge_cap));
    std::fill(h->lab.host.begin() + c.lab_at, h->lab.host.begin() + c.lab_at + c.lab_cap, 0);
    std::copy(labs.begin(), labs.end(), h->lab.host.begin() + c.lab_at);
    h->lab.dirty(c.lab_at, c.lab_at + c.lab_cap);

    // Start contribution.  Seeds: the states of this component in the
    // epsilon closure of the part's q0, and the byte edges of a hub q0 that
    // enter the component.
    Contrib &z = c.start;
    z = Contrib();
    std::vector<int32_t> seeds, zc;
    std::vector<std::pair<int32_t, int32_t>> hub_edges;
    if (p.hub) {
        for (auto &e : h->out[p.q0]) {
            if (h->comp_of[e.second] != ci) continue;
            if (e.first < 0) seeds.push_back(e.second);
            else hub_edges.push_back(e);
        }
    } else {
        seeds.push_back(p.q0);
    }
    closure(seeds, zc, false);
    // targets of a state set per byte
    std::vector<std::vector<int32_t>> by(256);
    auto bucket = [&](int32_t cls, int32_t d) {
        if (!h->cls_ok[cls]) return;
        if (h->cls_single[cls] >= 0) {
            by[h->cls_single[cls]].push_back(d);
            return;
        }
        for (int b = 0; b < 256; ++b)
            if (class_has(h->class_bits, cls, b)) by[b].push_back(d);
    };
    auto step_all = [&](const std::vector<int32_t> &src) {
        for (auto &v : by) v.clear();
        for (int32_t q : src)
            for (auto &e : h->out[q])
                if (e.first >= 0) bucket(e.first, e.second);
    };
    auto labels_of = [&](const std::vector<int32_t> &set, std::vector<int32_t> &outl) {
        outl.clear();
        for (int32_t q : set) {
            const auto &v = en[loc(q)];
            outl.insert(outl.end(), v.begin(), v.end());
        }
        std::sort(outl.begin(), outl.end());
        outl.erase(std::unique(outl.begin(), outl.end()), outl.end());
    };
    step_all(zc);
    for (auto &e : hub_edges) bucket(e.first, e.second);
    std::vector<std::vector<int32_t>> s1(256);
    std::vector<int32_t> lt;
    z.f1_off.push_back(0);
    z.e1_off.push_back(0);
    for (int b = 0; b < 256; ++b) {
        if (by[b].empty()) continue;
        closure(by[b], s1[b], true);
        if (s1[b].empty()) continue;
        z.f1_b.push_back(b);
        for (int32_t q : s1[b]) z.f1.push_back(word(q));
        z.f1_off.push_back((int32_t)z.f1.size());
        labels_of(s1[b], lt);
        z.e1.insert(z.e1.end(), lt.begin(), lt.end());
        z.e1_off.push_back((int32_t)z.e1.size());
    }
    z.pr_st_off.push_back(0);
    z.pr_lab_off.push_back(0);
    std::vector<int32_t> s2;
    for (int32_t b1 : z.f1_b) {
        step_all(s1[b1]);
        for (int b2 = 0; b2 < 256; ++b2) {
            if (by[b2].empty()) continue;
            closure(by[b2], s2, true);
            if (s2.empty()) continue;
            z.pr.push_back(b1 * 256 + b2);
            for (int32_t q : s2) z.pr_st.push_back(word(q));
            z.pr_st_off.push_back((int32_t)z.pr_st.size());
            labels_of(s2, lt);
            z.pr_lab.insert(z.pr_lab.end(), lt.begin(), lt.end());
            z.pr_lab_off.push_back((int32_t)z.pr_lab.size());
        }
    }
    return PFSM_OK;
}

auto by_state = [](uint32_t a, uint32_t b) { return (a & kStateMask) < (b & kStateMask); };

// Components whose parts are still in the union and that add to the start
// tables, in index order.
std::vector<int32_t> active_comps(const NfaHost *h) {
    std::vector<int32_t> act;
    for (int32_t ci = 0; ci < (int32_t)h->comps.size(); ++ci) {
        const Comp &c = h->comps[ci];
        if (!h->parts[c.part].cut && !c.start.f1_b.empty()) act.push_back(ci);
    }
    return act;
}

// Reassemble the first-symbol tables (256 lists) from the contributions of
// the active components: states concatenated in component order, then
// sorted; labels merged.
void assemble_first(NfaHost *h) {
    const std::vector<int32_t> act = active_comps(h);
    std::vector<int32_t> nst(257, 0), nlab(257, 0);
    for (int32_t ci : act) {
        const Contrib &z = h->comps[ci].start;
        for (size_t k = 0; k < z.f1_b.size(); ++k) {
            nst[z.f1_b[k] + 1] += z.f1_off[k + 1] - z.f1_off[k];
            nlab[z.f1_b[k] + 1] += z.e1_off[k + 1] - z.e1_off[k];
        }
    }
    for (int b = 0; b < 256; ++b) {
        nst[b + 1] += nst[b];
        nlab[b + 1] += nlab[b];
    }
    std::vector<uint32_t> f1(nst[256]);
    std::vector<int32_t> e1raw(nlab[256]);
    {
        std::vector<int32_t> cs(nst.begin(), nst.end() - 1), cl(nlab.begin(), nlab.end() - 1);
        for (int32_t ci : act) {
            const Contrib &z = h->comps[ci].start;
            for (size_t k = 0; k < z.f1_b.size(); ++k) {
                const int b = z.f1_b[k];
                for (int32_t j = z.f1_off[k]; j < z.f1_off[k + 1]; ++j) f1[cs[b]++] = z.f1[j];
                for (int32_t j = z.e1_off[k]; j < z.e1_off[k + 1]; ++j) e1raw[cl[b]++] = z.e1[j];
            }
        }
    }
    h->f1_off.host.assign(257, 0);
    h->e1_off.host.assign(257, 0);
    h->e1.host.clear();
    for (int b = 0; b < 256; ++b) {
        if (!std::is_sorted(f1.begin() + nst[b], f1.begin() + nst[b + 1], by_state))
            std::sort(f1.begin() + nst[b], f1.begin() + nst[b + 1], by_state);
        h->f1_off.host[b + 1] = nst[b + 1];
        std::sort(e1raw.begin() + nlab[b], e1raw.begin() + nlab[b + 1]);
        const auto end = std::unique(e1raw.begin() + nlab[b], e1raw.begin() + nlab[b + 1]);
        h->e1.host.insert(h->e1.host.end(), e1raw.begin() + nlab[b], end);
        h->e1_off.host[b + 1] = (int32_t)h->e1.host.size();
    }
    h->f1.host = std::move(f1);
    h->f1_off.all_dirty();
    h->f1.all_dirty();
    h->e1_off.all_dirty();
    h->e1.all_dirty();
}

// Byte-pair cache.  Pair p owns regions of the state and label arrays
// (p_rng[p] gives where its lists start and end); the components whose
// contributions list p are kept per pair, so an edit rebuilds only the
// pairs its components touch.  A list that outgrows its region moves to the
// end of its array; the space left behind is reclaimed by the next full
// layout.

// Entry k of z.pr for pair p, or -1.
int pair_entry(const Contrib &z, int p) {
    const auto it = std::lower_bound(z.pr.begin(), z.pr.end(), p);
    return it != z.pr.end() && *it == p ? (int)(it - z.pr.begin()) : -1;
}

// Region capacity for a list of n entries.
int32_t region_cap(int32_t n) { return n > 0 ? n + n / 4 + 1 : 0; }

// Rebuild pair p from the components that reach it.
void rebuild_pair(NfaHost *h, int p) {
    std::vector<uint32_t> &st = h->a_st;
    std::vector<int32_t> &lb = h->a_lb;
    st.clear();
    lb.clear();
    const std::vector<int32_t> &reach = h->pair_reach[p];
    for (int32_t ci : reach) {
        const Contrib &z = h->comps[ci].start;
        const int k = pair_entry(z, p);
        st.insert(st.end(), z.pr_st.begin() + z.pr_st_off[k], z.pr_st.begin() + z.pr_st_off[k + 1]);
        lb.insert(lb.end(), z.pr_lab.begin() + z.pr_lab_off[k], z.pr_lab.begin() + z.pr_lab_off[k + 1]);
    }
    if (reach.size() > 1) {
        if (!std::is_sorted(st.begin(), st.end(), by_state)) std::sort(st.begin(), st.end(), by_state);
        std::sort(lb.begin(), lb.end());
        lb.erase(std::unique(lb.begin(), lb.end()), lb.end());
    }
    PairRange &r = h->p_rng.host[p];
    const int32_t n = (int32_t)st.size(), ln = (int32_t)lb.size();
    h->pair_words += (int64_t)(n - (r.st_hi - r.st_lo)) + (int64_t)(ln - (r.lab_hi - r.lab_lo));
    if (n > h->st_cap[p]) {
        h->pair_garbage += h->st_cap[p];
        h->st_cap[p] = region_cap(n);
        r.st_lo = (int32_t)h->p_st.host.size();
        h->p_st.host.resize(h->p_st.host.size() + h->st_cap[p]);
    }
    if (ln > h->lab_cap[p]) {
        h->pair_garbage += h->lab_cap[p];
        h->lab_cap[p] = region_cap(ln);
        r.lab_lo = (int32_t)h->p_lab.host.size();
        h->p_lab.host.resize(h->p_lab.host.size() + h->lab_cap[p]);
    }
    r.st_hi = r.st_lo + n;
    r.lab_hi = r.lab_lo + ln;
    std::copy(st.begin(), st.end(), h->p_st.host.begin() + r.st_lo);
    std::copy(lb.begin(), lb.end(), h->p_lab.host.begin() + r.lab_lo);
    h->p_st.dirty(r.st_lo, r.st_hi);
    h->p_lab.dirty(r.lab_lo, r.lab_hi);
    h->p_rng.dirty(p, p + 1);
    if (n > 0) h->p_bits.host[p >> 5] |= 1u << (p & 31);
    else h->p_bits.host[p >> 5] &= ~(1u << (p & 31));
    h->p_bits.dirty(p >> 5, (p >> 5) + 1);
}

// Lay out every pair afresh (load, the cache turned on, or too much space
// left behind by moved lists).
void layout_pairs(NfaHost *h) {
    h->pair_reach.assign(65536, std::vector<int32_t>());
    h->st_cap.assign(65536, 0);
    h->lab_cap.assign(65536, 0);
    h->p_rng.host.assign(65536, PairRange{0, 0, 0, 0});
    h->p_bits.host.assign(2048, 0);
    h->p_st.host.clear();
    h->p_lab.host.clear();
    h->pair_words = 0;
    h->pair_garbage = 0;
    if (h->knobs.pair_cache) {
        for (int32_t ci : active_comps(h))
            for (int p : h->comps[ci].start.pr) h->pair_reach[p].push_back(ci);
        for (int p = 0; p < 65536; ++p)
            if (!h->pair_reach[p].empty()) rebuild_pair(h, p);
    }
    h->p_rng.all_dirty();
    h->p_bits.all_dirty();
    h->p_st.all_dirty();
    h->p_lab.all_dirty();
}

// Component ci's pair contributions changed from `old_pr` to its current
// ones (none when its part is cut): update the pairs either set names.
void update_pairs(NfaHost *h, int32_t ci, const std::vector<int32_t> &old_pr) {
    if (!h->knobs.pair_cache) return;
    const Comp &c = h->comps[ci];
    static const std::vector<int32_t> none;
    const std::vector<int32_t> &now = h->parts[c.part].cut ? none : c.start.pr;
    for (int p : old_pr) {
        auto &v = h->pair_reach[p];
        const auto it = std::lower_bound(v.begin(), v.end(), ci);
        if (it != v.end() && *it == ci) v.erase(it);
    }
    for (int p : now) {
        auto &v = h->pair_reach[p];
        v.insert(std::lower_bound(v.begin(), v.end(), ci), ci);
    }
    std::vector<int32_t> touched;
    std::set_union(old_pr.begin(), old_pr.end(), now.begin(), now.end(), std::back_inserter(touched));
    for (int p : touched) rebuild_pair(h, p);
}

// After the pair lists changed: reclaim space when much of it was left
// behind, and decide whether the cache is used.
void settle_pairs(NfaHost *h) {
    if (h->pair_garbage > (1 << 16) && 2 * h->pair_garbage > (int64_t)(h->p_st.host.size() + h->p_lab.host.size()))
        layout_pairs(h);
    h->pair_on = h->knobs.pair_cache != 0 && h->pair_words <= kPairBudget;
}

// Copy every dirty range to the device.  An array that outgrew its buffer
// gets a new one with room for half as much again (the old one is kept
// until the handle is freed, for scans or graphs that still refer to it)
// and the layout epoch advances.  Arrays written in place are written only
// after every scan already issued has finished (snapshot semantics).
template <typename T>
int grow_packed(NfaHost *h, Packed<T> &a, bool *moved) {
    const size_t need = std::max<size_t>(a.host.size(), 1);
    if (a.dev && need <= a.cap) return PFSM_OK;
    const size_t cap = need + need / 2 + 1024;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, cap * sizeof(T)));
    if (a.dev) h->retired.push_back(a.dev);
    a.dev = p;
    a.cap = cap;
    a.all_dirty();
    *moved = true;
    return PFSM_OK;
}

template <typename T>
int copy_packed(Packed<T> &a, hipStream_t s) {
    const size_t hi = std::min(a.hi, a.host.size());
    if (a.lo < hi)
        HIP_TRY(hipMemcpyAsync(a.ptr() + a.lo, a.host.data() + a.lo, (hi - a.lo) * sizeof(T), hipMemcpyHostToDevice, s));
    a.lo = SIZE_MAX;
    a.hi = 0;
    return PFSM_OK;
}

int commit(NfaHost *h, hipStream_t s, bool loaded, bool move_all = false) {
    bool moved = false;
    int rc;
    // When one array moves, all do: launches captured before (graphs) keep
    // a whole, unchanged set of old buffers.
    auto outgrown = [](const auto &a) { return !a.dev || std::max<size_t>(a.host.size(), 1) > a.cap; };
    if (loaded && (move_all || outgrown(h->rec) || outgrown(h->edges) || outgrown(h->cl) || outgrown(h->f1) ||
                   outgrown(h->p_bits) || outgrown(h->p_st) || outgrown(h->cls) || outgrown(h->cl_off) ||
                   outgrown(h->lab) || outgrown(h->f1_off) || outgrown(h->e1_off) || outgrown(h->e1) ||
                   outgrown(h->p_rng) || outgrown(h->p_lab))) {
        auto drop = [h](auto &a) {
            if (a.dev) h->retired.push_back(a.dev);
            a.dev = nullptr;
            a.cap = 0;
        };
        drop(h->rec), drop(h->edges), drop(h->cl), drop(h->f1), drop(h->p_bits), drop(h->p_st), drop(h->cls);
        drop(h->cl_off), drop(h->lab), drop(h->f1_off), drop(h->e1_off), drop(h->e1), drop(h->p_rng), drop(h->p_lab);
    }
    if ((rc = grow_packed(h, h->rec, &moved)) || (rc = grow_packed(h, h->edges, &moved)) ||
        (rc = grow_packed(h, h->cl, &moved)) || (rc = grow_packed(h, h->f1, &moved)) ||
        (rc = grow_packed(h, h->p_bits, &moved)) || (rc = grow_packed(h, h->p_st, &moved)) ||
        (rc = grow_packed(h, h->cls, &moved)) || (rc = grow_packed(h, h->cl_off, &moved)) ||
        (rc = grow_packed(h, h->lab, &moved)) || (rc = grow_packed(h, h->f1_off, &moved)) ||
        (rc = grow_packed(h, h->e1_off, &moved)) || (rc = grow_packed(h, h->e1, &moved)) ||
        (rc = grow_packed(h, h->p_rng, &moved)) || (rc = grow_packed(h, h->p_lab, &moved)))
        return rc;
    if (moved && loaded) ++h->layout_epoch;
    // scans issued before the edit read the arrays written below
    if (loaded) HIP_TRY(hipDeviceSynchronize());
    if ((rc = copy_packed(h->rec, s)) || (rc = copy_packed(h->edges, s)) || (rc = copy_packed(h->cl, s)) ||
        (rc = copy_packed(h->f1, s)) || (rc = copy_packed(h->p_bits, s)) || (rc = copy_packed(h->p_st, s)) ||
        (rc = copy_packed(h->cls, s)) || (rc = copy_packed(h->cl_off, s)) || (rc = copy_packed(h->lab, s)) ||
        (rc = copy_packed(h->f1_off, s)) || (rc = copy_packed(h->e1_off, s)) || (rc = copy_packed(h->e1, s)) ||
        (rc = copy_packed(h->p_rng, s)) || (rc = copy_packed(h->p_lab, s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return PFSM_OK;
}

// Tables of the components of part pi (just appended): placed at the ends.
int place_part(NfaHost *h, int32_t pi) {
    const Part &p = h->parts[pi];
    h->rec.host.resize((size_t)h->N);
    if (p.hub) {  // a hub q0 is never entered: an empty record
        std::memset(&h->rec.host[p.q0], 0, sizeof(NfaRec));
        h->rec.dirty(p.q0, p.q0 + 1);
    }
    if (h->cl_off.host.empty()) h->cl_off.host.assign(1, 0);
    const size_t cls0 = h->cls.host.size();
    h->cls.host = h->class_bits;
    h->cls.dirty(cls0, h->cls.host.size());
    for (int32_t ci : p.comps) {
        const int rc = compute_comp(h, ci, true);
        if (rc) return rc;
    }
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
    if ((rc = place_part(h.get(), 0))) return rc;
    assemble_first(h.get());
    layout_pairs(h.get());
    settle_pairs(h.get());
    if ((rc = commit(h.get(), s, false))) return rc;
    if ((rc = grid_size(h.get()))) return rc;
    *out = std::move(h);
    return PFSM_OK;
}

int nfa_add_pattern(NfaHost *h, const pfsm_nfa_desc *p, hipStream_t s) {
    int rc = validate(p);
    if (rc) return rc;
    for (int32_t i = 0; i < p->final_off[p->n_states]; ++i) {
        const auto it = h->enabled.find(p->final_labels[i]);
        if (it != h->enabled.end() && it->second > 0)
            return fail(PFSM_EEXIST, "label %d is already present", p->final_labels[i]);
    }
    if ((rc = append_part(h, p, true))) return rc;
    if ((rc = place_part(h, (int32_t)h->parts.size() - 1))) return rc;
    assemble_first(h);
    for (int32_t ci : h->parts.back().comps) update_pairs(h, ci, {});
    const int32_t pair_was = h->pair_on;
    settle_pairs(h);
    return commit(h, s, true, h->pair_on != pair_was);
}

int nfa_remove_pattern(NfaHost *h, int32_t label, hipStream_t s) {
    bool found = false;
    std::vector<int32_t> redo;
    for (Part &p : h->parts) {
        if (p.cut || std::binary_search(p.disabled.begin(), p.disabled.end(), label)) continue;
        // any state of the part, a hub q0 included, may carry the label
        bool carries = false;
        for (int32_t q = p.first; q < p.first + p.n && !carries; ++q)
            carries = std::binary_search(h->labels[q].begin(), h->labels[q].end(), label);
        if (!carries) continue;
        std::vector<int32_t> carrying;
        for (int32_t ci : p.comps)
            for (int32_t q : h->comps[ci].states)
                if (std::binary_search(h->labels[q].begin(), h->labels[q].end(), label)) {
                    carrying.push_back(ci);
                    break;
                }
        found = true;
        if (p.added) {
            p.cut = true;
            for (int32_t l : p.labs)
                if (!std::binary_search(p.disabled.begin(), p.disabled.end(), l)) --h->enabled[l];
            for (int32_t ci : p.comps) update_pairs(h, ci, h->comps[ci].start.pr);
        } else {
            p.disabled.insert(std::upper_bound(p.disabled.begin(), p.disabled.end(), label), label);
            --h->enabled[label];
            redo.insert(redo.end(), carrying.begin(), carrying.end());
        }
    }
    if (!found) return fail(PFSM_ENOENT, "no pattern carries label %d", label);
    for (int32_t ci : redo) {
        const std::vector<int32_t> old_pr = h->comps[ci].start.pr;
        const int rc = compute_comp(h, ci, false);
        if (rc) return rc;
        update_pairs(h, ci, old_pr);
    }
    assemble_first(h);
    const int32_t pair_was = h->pair_on;
    settle_pairs(h);
    return commit(h, s, true, h->pair_on != pair_was);
}

int nfa_grid_blocks(NfaHost *h) { return h->n_blocks; }

Knobs *nfa_knobs(NfaHost *h) { return &h->knobs; }

int nfa_occupancy(NfaHost *h) { return h->occ; }

uint64_t nfa_layout_epoch(NfaHost *h) { return h->layout_epoch; }

int nfa_apply_knobs(NfaHost *h, bool tables, hipStream_t s) {
    h->n_blocks = grid_blocks(h->occ, h->cus, h->knobs.wpc);
    if (!tables) return PFSM_OK;
    const int32_t pair_was = h->pair_on;
    layout_pairs(h);
    settle_pairs(h);
    return commit(h, s, true, h->pair_on != pair_was);
}

WorkspacePool *nfa_pool(NfaHost *h) { return &h->pool; }

namespace {

// The workspace of stream s with replay scratch for the state capacity of
// the packed arrays (the scratch stride the kernels are given).  Scratch
// outgrown by the union is kept until the workspace goes, for graphs that
// still refer to it.
int nfa_workspace(NfaHost *h, hipStream_t s, Workspace **out) {
    Workspace *w;
    int rc = h->pool.get(s, h->n_blocks, &w);
    if (rc) return rc;
    const int64_t states = (int64_t)h->rec.cap;
    const int64_t words_front = (int64_t)h->n_blocks * 2 * states;
    const int64_t words_bits = (int64_t)h->n_blocks * ((states + 31) / 32);
    if (w->big_states < states) {
        HIP_TRY(hipStreamSynchronize(s));
        if (w->big_front) w->retired.push_back(w->big_front);
        if (w->big_bits) w->retired.push_back(w->big_bits);
        w->big_front = w->big_bits = nullptr;
        w->big_states = 0;
        HIP_TRY(hipMalloc(&w->big_front, sizeof(uint32_t) * words_front));
        HIP_TRY(hipMalloc(&w->big_bits, sizeof(uint32_t) * words_bits));
        HIP_TRY(hipMemset(w->big_bits, 0, sizeof(uint32_t) * words_bits));
        HIP_TRY(hipDeviceSynchronize());
        w->big_states = states;
    }
    *out = w;
    return PFSM_OK;
}

// The scan's view of the current tables.
void nfa_table_args(NfaHost *h, NfaArgs &a) {
    a.n_states = (int32_t)h->rec.cap;
    a.rec = h->rec.ptr();
    a.edges = h->edges.ptr();
    a.class_bits = h->cls.ptr();
    a.cl_off = h->cl_off.ptr();
    a.cl = h->cl.ptr();
    a.lab = h->lab.ptr();
    a.f1_off = h->f1_off.ptr();
    a.f1 = h->f1.ptr();
    a.e1_off = h->e1_off.ptr();
    a.e1 = h->e1.ptr();
    a.pair_on = h->pair_on;
    a.p_bits = h->p_bits.ptr();
    a.p_rng = h->p_rng.ptr();
    a.p_st = h->p_st.ptr();
    a.p_lab = h->p_lab.ptr();
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
    // A plain scan places its segments' matches after the scan (dfa_defer.h).
    DfaDefer d;
    std::memset(&d, 0, sizeof d);
    if (!plan && !carry && !d_base && a.n_segs >= kDeferMinSegs) {
        const int64_t rows = std::min<int64_t>((int64_t)a.n_segs * kNfaMatchCap, kDeferRowsMax);
        if ((rc = grow_defer(w, a.n_segs, rows))) return rc;
        d.stage = w->defer_rows;
        d.stage_cap = std::min<int64_t>(w->c_defer_rows, cap);
        d.cursor = w->defer_cursor;
        d.seg_at = w->defer_seg;
        d.seg_cnt = w->defer_seg + w->c_defer_seg;
        d.seg_base = w->defer_seg + 2 * w->c_defer_seg;
    }
    void *args[] = {&a, &d};
    HIP_TRY(hipLaunchKernel(nfa_kernel_fn(carry != nullptr), dim3(grid), dim3(kNfaThreads), args, 0, s));
    if (d.stage) HIP_TRY(launch_dfa_place(d, a.n_segs, d_total, out, cap, s));
    w->last_grid = grid;
    h->pool.mark(w);
    return PFSM_OK;
}

int nfa_scan_async(NfaHost *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap, int64_t *d_total,
                   hipStream_t s) {
    return nfa_launch(h, x, n, nullptr, 0, out, cap, d_total, s);
}

}  // namespace pfsmk
