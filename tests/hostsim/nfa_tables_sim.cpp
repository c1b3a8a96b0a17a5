// Host build of the NFA table builder (the library's nfa_host.cpp) with a
// stand-in HIP runtime.  It loads an NFA, applies edits, and after each step
// scans an input using only the packed tables, read the way the scan kernel
// reads them: first-symbol lists, the byte-pair cache when it is on, then
// state records, inline or listed edges and closure lists.  It also checks
// that every index it follows stays inside its array.
//
// Input (text): a descriptor, the input bytes, then operations:
//   a <descriptor>   add a pattern        r <label>   remove a label
//   k <0|1>          pair cache off/on
// A descriptor is "n q0 n_classes", then row_ptr, edge_class, edge_dst,
// class_bits, final_off, final_labels, one array per line.
// Output: for the load and each operation, "== <rc>", then one line
// "start end label" per match, sorted.
#include "nfa_host.cpp"

#include <cstdio>
#include <set>
#include <string>
#include <tuple>

#include "dfa_defer.h"

namespace pfsmk {
std::string &last_error() {
    static std::string s;
    return s;
}
int device_cus(int *o) {
    *o = 4;
    return 0;
}
const void *nfa_kernel_fn(bool) {
    static int k;
    return &k;
}
hipError_t launch_nfa_resume(const NfaResumeArgs &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_dfa_place(const DfaDefer &, int, int64_t *, MatchOut *, int64_t, hipStream_t) { return hipSuccess; }
}  // namespace pfsmk

using namespace pfsmk;

namespace {

[[noreturn]] void die(const char *what) {
    printf("OUT OF BOUNDS: %s\n", what);
    exit(3);
}

struct Desc {
    int32_t n = 0, q0 = 0, nc = 0;
    std::vector<int32_t> row, ecls, edst, foff, flab;
    std::vector<uint32_t> bits;
    pfsm_nfa_desc view() {
        pfsm_nfa_desc x;
        memset(&x, 0, sizeof x);
        x.n_states = n;
        x.q0 = q0;
        x.n_classes = nc;
        x.row_ptr = row.data();
        x.edge_class = ecls.data();
        x.edge_dst = edst.data();
        x.class_bits = bits.data();
        x.final_off = foff.data();
        x.final_labels = flab.data();
        return x;
    }
};

template <typename T>
void read_n(FILE *f, std::vector<T> &v, size_t n) {
    v.resize(n);
    for (auto &x : v) {
        long long t;
        if (fscanf(f, "%lld", &t) != 1) die("truncated input");
        x = (T)t;
    }
}

bool read_desc(FILE *f, Desc &d) {
    if (fscanf(f, "%d %d %d", &d.n, &d.q0, &d.nc) != 3) return false;
    read_n(f, d.row, (size_t)d.n + 1);
    read_n(f, d.ecls, (size_t)d.row[d.n]);
    read_n(f, d.edst, (size_t)d.row[d.n]);
    read_n(f, d.bits, (size_t)d.nc * 8);
    read_n(f, d.foff, (size_t)d.n + 1);
    read_n(f, d.flab, (size_t)d.foff[d.n]);
    return true;
}

// The tables as the kernel sees them (device copies), with their lengths.
struct Tables {
    const NfaHost *h;
    template <typename T>
    static const T &at(const Packed<T> &a, int64_t i, const char *what) {
        if (i < 0 || (size_t)i >= a.host.size()) die(what);
        return a.ptr()[i];
    }
    bool edge_matches(uint32_t test, int c) const {
        const uint32_t kind = (test >> 8) & 3u;
        if (kind == 0) return (int)(test & 255u) == c;
        if (kind == 1) return true;
        const int64_t k = test >> 10;
        return (at(h->cls, k * 8 + (c >> 5), "class bits") >> (c & 31)) & 1u;
    }
    void add_target(uint32_t w, std::set<int32_t> &out) const {
        if (w & kTgtList) {
            const int64_t li = w & ~kTgtList;
            if (li + 1 > h->n_lists) die("closure list index");
            const int32_t lo = at(h->cl_off, li, "cl_off"), hi = at(h->cl_off, li + 1, "cl_off");
            for (int32_t j = lo; j < hi; ++j) add_word(at(h->cl, j, "closure words"), out);
        } else {
            add_word(w, out);
        }
    }
    void add_word(uint32_t w, std::set<int32_t> &out) const {
        const int32_t q = (int32_t)(w & kStateMask);
        if (q >= h->N) die("state id");
        out.insert(q);
    }
    std::set<int32_t> step(const std::set<int32_t> &S, int c) const {
        std::set<int32_t> T;
        for (int32_t q : S) {
            const NfaRec &r = at(h->rec, q, "records");
            if (r.info & kRecInline) {
                if (r.n_edges > 0 && edge_matches(r.e0_test, c)) add_target(r.e0_tgt, T);
                if (r.n_edges > 1 && edge_matches(r.e1_test, c)) add_target(r.e1_tgt, T);
            } else {
                for (int e = 0; e < r.n_edges; ++e)
                    if (edge_matches(at(h->edges, 2 * (int64_t)(r.edge_off + e), "edges"), c))
                        add_target(at(h->edges, 2 * (int64_t)(r.edge_off + e) + 1, "edges"), T);
            }
        }
        return T;
    }
    void report(const std::set<int32_t> &S, int32_t s, int32_t e, std::set<std::tuple<int, int, int>> &M) const {
        for (int32_t q : S) {
            const NfaRec &r = at(h->rec, q, "records");
            for (uint32_t j = 0; j < (r.info >> 8); ++j) M.insert({s, e, at(h->lab, r.lab_off + (int64_t)j, "labels")});
        }
    }
};

// Records marked kRecGapFin (a gap whose walks the scan finishes in one
// pass) must head a simple chain: from E's target on, every state passes one
// edge to a plain state and is not final, up to a final state without
// edges; lab_off holds the chain's first edge test; and no state after the
// first has another way in.  Returns how many such records there are.
int check_gap_chains(const NfaHost *h) {
    const int64_t ns = (int64_t)h->rec.host.size();
    auto rec = [&](uint32_t w) -> const NfaRec & { return Tables::at(h->rec, (int64_t)(w & kStateMask), "gap chain state"); };
    std::vector<int32_t> indeg(ns, 0);
    auto add_tgt = [&](uint32_t w) {
        if (w & kTgtList) {
            const int64_t l = (int64_t)(w & ~kTgtList);
            const int32_t lo = Tables::at(h->cl_off, l, "closure offsets"), hi = Tables::at(h->cl_off, l + 1, "closure offsets");
            for (int32_t j = lo; j < hi; ++j) ++indeg[Tables::at(h->cl, j, "closure lists") & kStateMask];
        } else {
            ++indeg[(int64_t)(w & kStateMask) < ns ? w & kStateMask : 0];
        }
    };
    for (int64_t q = 0; q < ns; ++q) {
        const NfaRec &r = Tables::at(h->rec, q, "records");
        if (!(r.info & kRecLive)) continue;
        if (r.info & kRecInline) {
            if (r.n_edges > 0) add_tgt(r.e0_tgt);
            if (r.n_edges > 1) add_tgt(r.e1_tgt);
        } else {
            for (int32_t e = 0; e < r.n_edges; ++e) add_tgt(Tables::at(h->edges, 2 * (int64_t)(r.edge_off + e) + 1, "edges"));
        }
    }
    int count = 0;
    for (int64_t q = 0; q < ns; ++q) {
        const NfaRec &r = Tables::at(h->rec, q, "records");
        if (!(r.info & kRecGapFin)) continue;
        ++count;
        if (!(r.info & kRecGap) || (r.e0_tgt & kTgtList)) die("gap chain: head is not a plain gap state");
        uint32_t w = r.e0_tgt;
        for (int64_t len = 0;; ++len) {
            const NfaRec &u = rec(w);
            const bool fin = (w & kTgtFinal) != 0;
            if (fin != ((u.info & kRecFinal) != 0)) die("gap chain: final flag of a target word");
            if (len > 0 && indeg[w & kStateMask] != 1) die("gap chain: a later state has another way in");
            if (fin) {
                if (!(u.info & kRecInline) || u.n_edges != 0) die("gap chain: final state with edges");
                break;
            }
            if (!(u.info & kRecInline) || u.n_edges != 1 || (u.info & kRecGap) || (u.e0_tgt & kTgtList))
                die("gap chain: not a simple chain state");
            if (len == 0 && (uint32_t)r.lab_off != u.e0_test) die("gap chain: first edge test");
            if (len > ns) die("gap chain: cycle");
            w = u.e0_tgt;
        }
    }
    return count;
}

void scan(const NfaHost *h, const std::vector<uint8_t> &x, FILE *o) {
    fprintf(stderr, "gap chains %d\n", check_gap_chains(h));
    Tables t{h};
    std::set<std::tuple<int, int, int>> M;
    const int32_t n = (int32_t)x.size();
    for (int32_t i = 0; i < n; ++i) {
        const int c1 = x[i];
        std::set<int32_t> S;
        const int32_t lo = Tables::at(h->f1_off, c1, "f1_off"), hi = Tables::at(h->f1_off, c1 + 1, "f1_off");
        for (int32_t j = lo; j < hi; ++j) t.add_word(Tables::at(h->f1, j, "f1"), S);
        for (int32_t j = Tables::at(h->e1_off, c1, "e1_off"); j < Tables::at(h->e1_off, c1 + 1, "e1_off"); ++j)
            M.insert({i, i, Tables::at(h->e1, j, "e1")});
        if (S.empty() || i + 1 >= n) continue;
        const int c2 = x[i + 1];
        if (h->pair_on) {
            const int p = c1 * 256 + c2;
            std::set<int32_t> S2;
            if ((Tables::at(h->p_bits, p >> 5, "pair bits") >> (p & 31)) & 1u) {
                const PairRange &r = Tables::at(h->p_rng, p, "pair ranges");
                for (int32_t j = r.st_lo; j < r.st_hi; ++j) t.add_word(Tables::at(h->p_st, j, "pair states"), S2);
                for (int32_t j = r.lab_lo; j < r.lab_hi; ++j) M.insert({i, i + 1, Tables::at(h->p_lab, j, "pair labels")});
            }
            S = S2;
        } else {
            S = t.step(S, c2);
            t.report(S, i, i + 1, M);
        }
        for (int32_t e = i + 2; e < n && !S.empty(); ++e) {
            S = t.step(S, x[e]);
            t.report(S, i, e, M);
        }
    }
    for (auto &m : M) fprintf(o, "%d %d %d\n", std::get<0>(m), std::get<1>(m), std::get<2>(m));
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "r");
    FILE *o = fopen(argv[2], "w");
    if (!f || !o) return 2;
    Desc d;
    if (!read_desc(f, d)) return 2;
    int32_t nx = 0;
    if (fscanf(f, "%d", &nx) != 1) return 2;
    std::vector<uint8_t> x;
    read_n(f, x, (size_t)nx);
    NfaPtr h;
    pfsm_nfa_desc dv = d.view();
    int rc = nfa_load(&dv, nullptr, &h);
    fprintf(o, "== %d\n", rc);
    if (rc) return 0;
    scan(h.get(), x, o);
    char op[8];
    while (fscanf(f, "%7s", op) == 1) {
        if (op[0] == 'a') {
            Desc p;
            if (!read_desc(f, p)) return 2;
            pfsm_nfa_desc pv = p.view();
            rc = nfa_add_pattern(h.get(), &pv, nullptr);
        } else if (op[0] == 'r') {
            int l = 0;
            if (fscanf(f, "%d", &l) != 1) return 2;
            rc = nfa_remove_pattern(h.get(), l, nullptr);
        } else if (op[0] == 'k') {
            int v = 0;
            if (fscanf(f, "%d", &v) != 1) return 2;
            nfa_knobs(h.get())->pair_cache = v;
            rc = nfa_apply_knobs(h.get(), true, nullptr);
        } else {
            return 2;
        }
        fprintf(o, "== %d\n", rc);
        scan(h.get(), x, o);
    }
    fclose(o);
    return 0;
}
