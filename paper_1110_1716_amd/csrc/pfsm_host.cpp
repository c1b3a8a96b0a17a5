// Host side of libpfsm: the C ABI declared in include/pfsm.h, DFA descriptor
// validation, the read-only caches derived from a DFA, device upload and the
// launch of the DFA scan.  The NFA half lives in nfa_host.cpp.
#include "pfsm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batch.h"
#include "dfa_defer.h"
#include "host_common.h"
#include "pfsm_dev.h"
#include "pfsm_nfa.h"
#include "stream.h"

using namespace pfsmk;

namespace pfsmk {

std::string &last_error() {
    thread_local std::string s;
    return s;
}

int device_cus(int *out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(out, hipDeviceAttributeMultiprocessorCount, dev));
    return PFSM_OK;
}

}  // namespace pfsmk

struct pfsm {
    int kind = 0;  // 0 = DFA, 1 = NFA
    // ---- DFA: host copy (used to rebuild caches when a label is removed)
    int32_t n_states = 0, n_symbols = 0, q0 = 0;
    bool identity = true;
    bool dev_identity = true;                  // the device table is indexed by byte
    int32_t dev_symbols = 0;                   // columns of the device table
    std::vector<int16_t> b2s;                  // [256]
    std::vector<int32_t> delta;                // [n_states * n_symbols]
    std::vector<std::vector<int32_t>> labels;  // per state: sorted unique labels
    std::vector<int32_t> disabled;             // removed labels (sorted)
    // ---- DFA: device tables and the kernel's launch shape
    DevBuf d_tbl, d_res, d_b2s, d_first, d_first_slot, d_flags, d_lab_off, d_lab;
    bool tbl16 = true;
    int enc = kCold16;
    int32_t res_bytes = 0, n_hot = 0;
    int32_t off_flags = 0, off_laboff = 0, off_lab = 0, off_tab = 0, off_q = 0, off_m = 0, off_list = 0,
            lds_bytes = 0;
    int n_blocks = 0;
    int occ = 0, cus = 0;  // workgroups per compute unit that fit; compute units
    Knobs knobs;
    // tag-merged scan (at most kMergedStates states): byte-indexed table
    DevBuf d_mtab;
    bool merged_ok = false;
    int m_occ = 0;
    const void *kernel = nullptr;
    // ---- NFA
    NfaPtr nfa;
    // ---- scan workspaces, one per stream
    WorkspacePool pool;
    // ---- successful edits (streams opened before an edit refuse to go on)
    uint64_t edits = 0;
    // ---- DFA: device buffers replaced by a new layout (freed with the
    // handle, since captured graphs may still refer to them) and the count
    // of such replacements
    std::vector<void *> retired;
    uint64_t layout_epoch = 0;
    bool laid_out = false;

    ~pfsm() {
        for (void *p : retired) (void)hipFree(p);
    }
};

namespace {

int check_labels(int32_t n_states, const int32_t *off, const int32_t *lab) {
    if (!off) return fail(PFSM_EINVAL, "final_off is NULL");
    if (off[0] != 0) return fail(PFSM_EINVAL, "final_off[0] must be 0");
    for (int32_t q = 0; q < n_states; ++q)
        if (off[q + 1] < off[q]) return fail(PFSM_EINVAL, "final_off decreases at state %d", q);
    const int32_t nnz = off[n_states];
    if (nnz > 0 && !lab) return fail(PFSM_EINVAL, "final_labels is NULL");
    for (int32_t i = 0; i < nnz; ++i)
        if (lab[i] < 0) return fail(PFSM_EINVAL, "label %d is negative", lab[i]);
    return PFSM_OK;
}

std::vector<std::vector<int32_t>> label_sets(int32_t n_states, const int32_t *off, const int32_t *lab) {
    std::vector<std::vector<int32_t>> out(n_states);
    for (int32_t q = 0; q < n_states; ++q) {
        auto &v = out[q];
        v.assign(lab + off[q], lab + off[q + 1]);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    return out;
}

bool has_label(const std::vector<int32_t> &sorted, int32_t l) {
    return std::binary_search(sorted.begin(), sorted.end(), l);
}

int align16(int v) { return (v + 15) & ~15; }

// Rebuild and upload every cache that depends on the enabled label sets:
// live flags (reverse search from states with an enabled label over
// transitions some byte can take), the q0 row per byte, the LDS copies of the
// rows of q0's successors, label CSR; then the LDS layout and grid size.
// With `in_place` (after a label is removed) the layout stays as it is and
// the caches that change are rewritten inside their buffers: the label area
// only shrinks, and neither the table nor its cached rows depend on labels.
int dfa_upload_caches(pfsm_t *h, hipStream_t s, bool in_place = false) {
    const int32_t N = h->n_states, S = h->n_symbols;
    std::vector<std::vector<int32_t>> en(N);
    for (int32_t q = 0; q < N; ++q)
        for (int32_t l : h->labels[q])
            if (!has_label(h->disabled, l)) en[q].push_back(l);

    std::vector<uint8_t> sym_used(S, 0);
    for (int b = 0; b < 256; ++b)
        if (h->b2s[b] >= 0) sym_used[h->b2s[b]] = 1;
    std::vector<int32_t> roff(N + 1, 0);
    for (int64_t i = 0; i < (int64_t)N * S; ++i)
        if (h->delta[i] >= 0 && sym_used[i % S]) roff[h->delta[i] + 1]++;
    for (int32_t q = 0; q < N; ++q) roff[q + 1] += roff[q];
    std::vector<int32_t> radj(roff[N]), fillp(roff.begin(), roff.end() - 1);
    for (int64_t i = 0; i < (int64_t)N * S; ++i)
        if (h->delta[i] >= 0 && sym_used[i % S]) radj[fillp[h->delta[i]]++] = (int32_t)(i / S);
    std::vector<uint8_t> flags(N, 0);
    std::vector<int32_t> queue;
    queue.reserve(N);
    for (int32_t q = 0; q < N; ++q)
        if (!en[q].empty()) {
            flags[q] = kLive | kFinal;
            queue.push_back(q);
        }
    for (size_t i = 0; i < queue.size(); ++i)
        for (int32_t k = roff[queue[i]]; k < roff[queue[i] + 1]; ++k)
            if (!(flags[radj[k]] & kLive)) {
                flags[radj[k]] |= kLive;
                queue.push_back(radj[k]);
            }
    std::vector<int32_t> first(256, -1);
    for (int b = 0; b < 256; ++b) {
        const int sym = h->b2s[b];
        if (sym < 0) continue;
        const int32_t t = h->delta[(int64_t)h->q0 * S + sym];
        if (t >= 0 && (flags[t] & kLive)) first[b] = t;
    }
    std::vector<int32_t> off(N + 1, 0), lab;
    for (int32_t q = 0; q < N; ++q) {
        lab.insert(lab.end(), en[q].begin(), en[q].end());
        off[q + 1] = (int32_t)lab.size();
    }

    if (in_place) {
        const bool resident = h->enc == kEnc8 || h->enc == kEnc8D || h->enc == kEnc16;
        if ((int64_t)lab.size() * 4 > (int64_t)h->d_lab.bytes ||
            (resident && (int64_t)lab.size() * 4 > h->off_tab - h->off_lab))
            return fail(PFSM_EINVAL, "label area outgrown");
        int rc;
        if ((rc = h->d_first.write(first.data(), 256, s))) return rc;
        if ((rc = h->d_flags.write(flags.data(), N, s))) return rc;
        if ((rc = h->d_lab_off.write(off.data(), N + 1, s))) return rc;
        if (!lab.empty() && (rc = h->d_lab.write(lab.data(), lab.size(), s))) return rc;
        std::vector<uint8_t> head;
        if (resident) {
            head.assign((size_t)(h->off_tab - h->off_flags), 0);
            std::memcpy(head.data(), flags.data(), (size_t)N);
            std::memcpy(head.data() + (h->off_laboff - h->off_flags), off.data(), sizeof(int32_t) * (size_t)(N + 1));
            if (!lab.empty())
                std::memcpy(head.data() + (h->off_lab - h->off_flags), lab.data(), sizeof(int32_t) * lab.size());
            if ((rc = h->d_res.write(head.data(), head.size(), s))) return rc;
        }
        std::vector<uint8_t> mt;
        if (h->merged_ok) {
            mt.resize((size_t)N * 256);
            for (int32_t q = 0; q < N; ++q)
                for (int b = 0; b < 256; ++b) {
                    const int sy = h->b2s[b];
                    const int32_t v = sy < 0 ? -1 : h->delta[(int64_t)q * S + sy];
                    const bool ok = v >= 0 && (flags[v] & kLive);
                    mt[(size_t)q * 256 + b] = ok ? (uint8_t)(v | ((flags[v] & kFinal) ? 128 : 0)) : 255;
                }
            if ((rc = h->d_mtab.write(mt.data(), mt.size(), s))) return rc;
        }
        HIP_TRY(hipStreamSynchronize(s));
        return PFSM_OK;
    }
    // A new layout: buffers a captured graph may still name are kept.
    if (h->laid_out) {
        DevBuf *old[] = {&h->d_first, &h->d_first_slot, &h->d_res, &h->d_flags, &h->d_lab_off, &h->d_lab, &h->d_mtab};
        for (DevBuf *b : old)
            if (b->p) h->retired.push_back(b->detach());
        ++h->layout_epoch;
    }

    // An automaton over a byte map whose byte-indexed 8-bit table fits LDS
    // is expanded to bytes, so the kernel indexes the table by the byte.
    const int64_t ns_b = (int64_t)N * 256;
    const int64_t expanded_bytes = N <= 255 ? ns_b : ns_b + ns_b / 8;
    const int64_t budget = h->knobs.table_budget >= 0 ? h->knobs.table_budget : kDfaTableBudget;
    const bool expand = !h->identity && N <= 256 && expanded_bytes <= budget;
    std::vector<int32_t> dexp;
    const int32_t *dl = h->delta.data();
    int32_t SD = S;
    if (expand) {
        dexp.resize(ns_b);
        for (int32_t q = 0; q < N; ++q)
            for (int b = 0; b < 256; ++b) {
                const int sy = h->b2s[b];
                dexp[(int64_t)q * 256 + b] = sy < 0 ? -1 : h->delta[(int64_t)q * S + sy];
            }
        dl = dexp.data();
        SD = 256;
    }

    // Transition table image for LDS.  A resident encoding keeps the whole
    // table, the flags and the label CSR in LDS; when none fits, the table is
    // read through L2 and the rows of q0's live successors are copied.
    const int64_t ns = (int64_t)N * SD;
    std::vector<uint8_t> res;
    std::vector<int16_t> first_slot(256, -1);
    int n_hot = 0;
    int enc = -1;
    auto lds_total = [&](int64_t tab_bytes, bool resident, int64_t flag_bytes) {
        int64_t off = align16(kDfaLdsFixed);
        if (resident) {
            off = align16(off + flag_bytes);
            off = align16(off + (N + 1) * 4);
            off = align16(off + (int64_t)lab.size() * 4);
        }
        off = align16(off + (tab_bytes + 15) / 16 * 16 + 16);
        off += (kDfaThreads / 64) * kDfaQueue * 16;
        off += kDfaMatchCap * 12;
        return off + kDfaWaves * kDfaList * 4;
    };
    const int64_t bytes8 = ns, bytes8d = ((ns + 3) & ~3ll) + (ns + 31) / 32 * 4, bytes16 = ns * 2;
    if (N <= 255 && bytes8 <= budget && lds_total(bytes8, true, kDfaFlags8) <= kDfaLdsLimit) {
        enc = kEnc8;
        res.resize(ns);
        for (int64_t i = 0; i < ns; ++i) res[i] = dl[i] < 0 ? 255 : (uint8_t)dl[i];
    } else if (N == 256 && bytes8d <= budget && lds_total(bytes8d, true, N) <= kDfaLdsLimit) {
        enc = kEnc8D;
        const int64_t dead_off = (ns + 3) & ~3ll;
        res.assign(bytes8d, 0);
        uint32_t *dead = reinterpret_cast<uint32_t *>(res.data() + dead_off);
        for (int64_t i = 0; i < ns; ++i) {
            if (dl[i] < 0) dead[i >> 5] |= 1u << (i & 31);
            else res[i] = (uint8_t)dl[i];
        }
    } else if (N <= 32767 && bytes16 <= budget && lds_total(bytes16, true, N) <= kDfaLdsLimit) {
        enc = kEnc16;
        res.resize(bytes16);
        int16_t *t = reinterpret_cast<int16_t *>(res.data());
        for (int64_t i = 0; i < ns; ++i) t[i] = (int16_t)dl[i];
    } else {
        SD = S;  // the cold encodings read the table as loaded
        enc = h->tbl16 ? kCold16 : kCold32;
        const int elem = h->tbl16 ? 2 : 4;
        const int max_hot = (int)std::min<int64_t>(32767, kDfaHotBudget / ((int64_t)S * elem));
        std::vector<std::pair<int, int32_t>> freq;  // (-bytes leading there, state)
        std::vector<int32_t> tg;
        for (int b = 0; b < 256; ++b)
            if (first[b] >= 0) tg.push_back(first[b]);
        std::sort(tg.begin(), tg.end());
        for (size_t i = 0; i < tg.size();) {
            size_t j = i;
            while (j < tg.size() && tg[j] == tg[i]) ++j;
            freq.push_back({-(int)(j - i), tg[i]});
            i = j;
        }
        std::sort(freq.begin(), freq.end());
        std::vector<int32_t> hot_states;
        for (auto &f : freq)
            if ((int)hot_states.size() < max_hot) hot_states.push_back(f.second);
        for (int b = 0; b < 256; ++b)
            for (size_t k = 0; k < hot_states.size(); ++k)
                if (first[b] == hot_states[k]) first_slot[b] = (int16_t)k;
        n_hot = (int)hot_states.size();
        res.resize((size_t)n_hot * S * elem);
        for (int k = 0; k < n_hot; ++k)
            for (int sy = 0; sy < S; ++sy) {
                const int32_t v = h->delta[(int64_t)hot_states[k] * S + sy];
                if (elem == 2) reinterpret_cast<int16_t *>(res.data())[(int64_t)k * S + sy] = (int16_t)v;
                else reinterpret_cast<int32_t *>(res.data())[(int64_t)k * S + sy] = v;
            }
    }
    res.resize((res.size() + 15) / 16 * 16 + 16, 0);  // whole 16-byte copies
    const bool resident = enc == kEnc8 || enc == kEnc8D || enc == kEnc16;
    h->off_flags = align16(kDfaLdsFixed);
    const int flag_bytes = enc == kEnc8 ? kDfaFlags8 : N;
    h->off_laboff = align16(h->off_flags + (resident ? flag_bytes : 0));
    h->off_lab = align16(h->off_laboff + (resident ? (N + 1) * 4 : 0));
    h->off_tab = align16(h->off_lab + (resident ? (int)lab.size() * 4 : 0));
    h->off_q = align16(h->off_tab + (int)res.size());
    h->off_m = h->off_q + (kDfaThreads / 64) * kDfaQueue * 16;
    h->off_list = h->off_m + kDfaMatchCap * 12;
    h->lds_bytes = h->off_list + kDfaWaves * kDfaList * 4;
    if (h->lds_bytes > kDfaLdsLimit) return fail(PFSM_EINVAL, "DFA scan LDS layout does not fit");

    // The LDS image from off_flags to the end of the table: flags, label CSR
    // (resident encodings) and the table or cached rows, in LDS layout, so
    // that the kernel copies it with one run of loads.
    std::vector<uint8_t> img((size_t)(h->off_tab - h->off_flags) + res.size(), 0);
    if (resident) {
        std::memcpy(img.data(), flags.data(), (size_t)N);
        std::memcpy(img.data() + (h->off_laboff - h->off_flags), off.data(), sizeof(int32_t) * (size_t)(N + 1));
        if (!lab.empty())
            std::memcpy(img.data() + (h->off_lab - h->off_flags), lab.data(), sizeof(int32_t) * lab.size());
    }
    std::memcpy(img.data() + (h->off_tab - h->off_flags), res.data(), res.size());

    int rc;
    if ((rc = h->d_first.upload(first.data(), 256, s))) return rc;
    if ((rc = h->d_first_slot.upload(first_slot.data(), 256, s))) return rc;
    if ((rc = h->d_res.upload(img.data(), img.size(), s))) return rc;
    if ((rc = h->d_flags.upload(flags.data(), N, s))) return rc;
    if ((rc = h->d_lab_off.upload(off.data(), N + 1, s))) return rc;
    if ((rc = h->d_lab.upload(lab.data(), lab.size(), s))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    h->enc = enc;
    h->n_hot = n_hot;
    h->res_bytes = (int32_t)img.size();
    h->laid_out = true;

    h->dev_identity = h->identity || (expand && SD == 256);
    h->dev_symbols = SD;
    h->kernel = dfa_kernel_fn(enc, h->dev_identity);
    if (!h->kernel) return fail(PFSM_EINVAL, "no DFA kernel for encoding %d", enc);
    HIP_TRY(hipFuncSetAttribute(h->kernel, hipFuncAttributeMaxDynamicSharedMemorySize, h->lds_bytes));
    int occ = 0, cus = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, h->kernel, kDfaThreads, h->lds_bytes));
    if ((rc = device_cus(&cus))) return rc;
    if (occ < 1) return fail(PFSM_EINVAL, "DFA scan kernel does not fit on a compute unit");
    h->occ = occ;
    h->cus = cus;
    h->n_blocks = grid_blocks(occ, cus, h->knobs.wpc);

    // The tag-merged scan's table by byte: the live target, with bit 7 set
    // when it is final; 255 = no live target.
    h->merged_ok = false;
    if (N <= kMergedStates) {
        std::vector<uint8_t> mt((size_t)N * 256);
        for (int32_t q = 0; q < N; ++q)
            for (int b = 0; b < 256; ++b) {
                const int sy = h->b2s[b];
                const int32_t v = sy < 0 ? -1 : h->delta[(int64_t)q * S + sy];
                const bool ok = v >= 0 && (flags[v] & kLive);
                mt[(size_t)q * 256 + b] = ok ? (uint8_t)(v | ((flags[v] & kFinal) ? 128 : 0)) : 255;
            }
        if ((rc = h->d_mtab.upload(mt.data(), mt.size(), s))) return rc;
        HIP_TRY(hipStreamSynchronize(s));
        const void *mk = dfa_merged_fn();
        HIP_TRY(hipFuncSetAttribute(mk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)merged_lds(N)));
        int mocc = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&mocc, mk, kMergedThreads, merged_lds(N)));
        h->m_occ = mocc;
        h->merged_ok = mocc > 0;
    }
    return PFSM_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char *pfsm_strerror(int code) {
    switch (code) {
    case PFSM_OK: return "success";
    case PFSM_EINVAL: return "invalid argument or descriptor";
    case PFSM_ENOMEM: return "out of memory";
    case PFSM_EOVERFLOW: return "more matches than the output capacity";
    case PFSM_EHIP: return "HIP runtime error";
    case PFSM_ENOENT: return "no pattern carries the label";
    case PFSM_EEXIST: return "label already present";
    case PFSM_ENOSYS: return "operation not supported for this handle";
    default: return "unknown error";
    }
}

const char *pfsm_last_error(void) { return last_error().c_str(); }

int pfsm_load_dfa(pfsm_t **out, const pfsm_dfa_desc *d, void *hip_stream) {
    if (!out || !d) return fail(PFSM_EINVAL, "NULL argument");
    *out = nullptr;
    const int32_t N = d->n_states, S = d->n_symbols;
    if (N < 1 || S < 1) return fail(PFSM_EINVAL, "n_states and n_symbols must be >= 1");
    if ((int64_t)N * S >= (1ll << 31)) return fail(PFSM_EINVAL, "n_states * n_symbols must be < 2^31");
    if (d->q0 < 0 || d->q0 >= N) return fail(PFSM_EINVAL, "q0 out of range");
    if (!d->byte_to_symbol && S != 256)
        return fail(PFSM_EINVAL, "byte_to_symbol may be NULL only when n_symbols == 256");
    if (!d->delta) return fail(PFSM_EINVAL, "delta is NULL");
    for (int64_t i = 0; i < (int64_t)N * S; ++i)
        if (d->delta[i] < -1 || d->delta[i] >= N)
            return fail(PFSM_EINVAL, "delta[%lld] = %d out of range", (long long)i, d->delta[i]);
    if (d->byte_to_symbol)
        for (int b = 0; b < 256; ++b)
            if (d->byte_to_symbol[b] < -1 || d->byte_to_symbol[b] >= S)
                return fail(PFSM_EINVAL, "byte_to_symbol[%d] out of range", b);
    int rc = check_labels(N, d->final_off, d->final_labels);
    if (rc) return rc;

    std::unique_ptr<pfsm_t> h(new (std::nothrow) pfsm_t);
    if (!h) return fail(PFSM_ENOMEM, "handle");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    h->kind = 0;
    h->n_states = N;
    h->n_symbols = S;
    h->q0 = d->q0;
    h->identity = d->byte_to_symbol == nullptr;
    h->b2s.resize(256);
    for (int b = 0; b < 256; ++b) h->b2s[b] = d->byte_to_symbol ? d->byte_to_symbol[b] : (int16_t)b;
    h->delta.assign(d->delta, d->delta + (int64_t)N * S);
    h->labels = label_sets(N, d->final_off, d->final_labels);
    h->tbl16 = N <= 32767;
    if (h->tbl16) {
        std::vector<int16_t> t16(h->delta.begin(), h->delta.end());
        if ((rc = h->d_tbl.upload(t16.data(), t16.size(), s))) return rc;
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        if ((rc = h->d_tbl.upload(h->delta.data(), h->delta.size(), s))) return rc;
    }
    if ((rc = h->d_b2s.upload(h->b2s.data(), 256, s))) return rc;
    if ((rc = dfa_upload_caches(h.get(), s))) return rc;
    *out = h.release();
    return PFSM_OK;
}

int pfsm_load_nfa(pfsm_t **out, const pfsm_nfa_desc *d, void *hip_stream) {
    if (!out || !d) return fail(PFSM_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_ptr<pfsm_t> h(new (std::nothrow) pfsm_t);
    if (!h) return fail(PFSM_ENOMEM, "handle");
    h->kind = 1;
    int rc = nfa_load(d, static_cast<hipStream_t>(hip_stream), &h->nfa);
    if (rc) return rc;
    *out = h.release();
    return PFSM_OK;
}

int pfsm_add_pattern(pfsm_t *h, const pfsm_nfa_desc *pattern, void *hip_stream) {
    if (!h || !pattern) return fail(PFSM_EINVAL, "NULL argument");
    if (h->kind == 0)
        return fail(PFSM_ENOSYS, "a DFA handle is one monolithic table; load the union as an NFA");
    const int rc = nfa_add_pattern(h->nfa.get(), pattern, static_cast<hipStream_t>(hip_stream));
    if (rc == PFSM_OK) ++h->edits;
    return rc;
}

int pfsm_remove_pattern(pfsm_t *h, int32_t label, void *hip_stream) {
    if (!h) return fail(PFSM_EINVAL, "NULL handle");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (h->kind == 1) {
        const int rc = nfa_remove_pattern(h->nfa.get(), label, s);
        if (rc == PFSM_OK) ++h->edits;
        return rc;
    }
    if (has_label(h->disabled, label)) return fail(PFSM_ENOENT, "label %d already removed", label);
    bool found = false;
    for (auto &v : h->labels)
        if (has_label(v, label)) {
            found = true;
            break;
        }
    if (!found) return fail(PFSM_ENOENT, "no final state carries label %d", label);
    h->disabled.insert(std::upper_bound(h->disabled.begin(), h->disabled.end(), label), label);
    // Scans already issued read the current caches: wait for the device,
    // then rewrite them in place.
    HIP_TRY(hipDeviceSynchronize());
    ++h->edits;
    return dfa_upload_caches(h, s, true);
}

// The fields of a DFA scan launch that come from the handle and the call:
// input, tables, output and the LDS layout.  The caller sets the scratch
// fields (ctl, lb, bstats, spill) and the segment plan.
static void dfa_common_args(const pfsm_t *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap,
                            int64_t *d_total, DfaArgs &a) {
    std::memset(&a, 0, sizeof a);
    a.x = x;
    a.n = n;
    a.tbl = h->d_tbl.p;
    a.res = h->d_res.p;
    a.res_bytes = h->res_bytes;
    a.n_states = h->n_states;
    a.n_symbols = h->dev_symbols;
    a.b2s = h->d_b2s.as<int16_t>();
    a.first = h->d_first.as<int32_t>();
    a.first_slot = h->d_first_slot.as<int16_t>();
    a.n_hot = h->n_hot;
    a.flags = h->d_flags.as<uint8_t>();
    a.lab_off = h->d_lab_off.as<int32_t>();
    a.lab = h->d_lab.as<int32_t>();
    a.out = out;
    a.cap = cap;
    a.total = d_total;
    a.off_flags = h->off_flags;
    a.off_laboff = h->off_laboff;
    a.off_lab = h->off_lab;
    a.off_tab = h->off_tab;
    a.off_q = h->off_q;
    a.off_m = h->off_m;
    a.off_list = h->off_list;
    a.lds_bytes = h->lds_bytes;
}

// One launch of the DFA scan kernel: a single stream (plan == nullptr) or the
// segments of a batch plan.
static int dfa_launch(pfsm_t *h, const uint8_t *x, int64_t n, const SegPlan *plan, int64_t seg, MatchOut *out,
                      int64_t cap, int64_t *d_total, hipStream_t s, const int64_t *d_base = nullptr,
                      const CarryOut *carry = nullptr) {
    Workspace *w;
    int rc = h->pool.get(s, h->n_blocks, &w);
    if (rc) return rc;
    if (!w->spill) HIP_TRY(hipMalloc(&w->spill, (size_t)h->n_blocks * kDfaSpill * 16));
    DfaArgs a;
    dfa_common_args(h, x, n, out, cap, d_total, a);
    a.ctl = w->ctl;
    a.bstats = w->bstats;
    a.spill = w->spill;
    int grid = h->n_blocks;
    if (plan) {
        a.plan = *plan;
        a.seg = seg;
    } else {
        int rounds;
        plan_segments(n, h->n_blocks, h->knobs.segment > 0 ? h->knobs.segment : kDfaSegMax,
                      dfa_seg_floor(n, h->res_bytes), &a.seg,
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
        const int64_t rows = std::min<int64_t>((int64_t)a.n_segs * kDfaMatchCap, kDeferRowsMax);
        if ((rc = grow_defer(w, a.n_segs, rows))) return rc;
        d.stage = w->defer_rows;
        d.stage_cap = std::min<int64_t>(w->c_defer_rows, cap);
        d.cursor = w->defer_cursor;
        d.seg_at = w->defer_seg;
        d.seg_cnt = w->defer_seg + w->c_defer_seg;
        d.seg_base = w->defer_seg + 2 * w->c_defer_seg;
    }
    void *args[] = {&a, &d};
    HIP_TRY(hipLaunchKernel(h->kernel, dim3(grid), dim3(kDfaThreads), args, h->lds_bytes, s));
    if (d.stage) HIP_TRY(launch_dfa_place(d, a.n_segs, d_total, out, cap, s));
    w->last_grid = grid;
    h->pool.mark(w);
    return PFSM_OK;
}

// One launch of the tag-merged scan (a single stream).
static int merged_launch(pfsm_t *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap, int64_t *d_total,
                         hipStream_t s) {
    const int blocks = grid_blocks(h->m_occ, h->cus, h->knobs.wpc);
    Workspace *w;
    int rc = h->pool.get(s, blocks, &w);
    if (rc) return rc;
    const int64_t n_segs = (n + kMergedSeg - 1) / kMergedSeg;
    auto grow_ll = [&](long long **p, int64_t *c, int64_t need) -> int {
        if (need <= *c) return PFSM_OK;
        HIP_TRY(hipStreamSynchronize(s));
        if (*p) HIP_TRY(hipFree(*p));
        *p = nullptr;
        *c = 0;
        HIP_TRY(hipMalloc(p, sizeof(long long) * (size_t)need));
        *c = need;
        return PFSM_OK;
    };
    if ((rc = grow_ll(&w->m_tag, &w->c_m_tag, n)) || (rc = grow_ll(&w->m_seg, &w->c_m_seg, 2 * n_segs + 1)))
        return rc;
    MergedArgs a;
    std::memset(&a, 0, sizeof a);
    a.x = x;
    a.n = n;
    a.tab = h->d_mtab.as<uint8_t>();
    a.lab_off = h->d_lab_off.as<int32_t>();
    a.lab = h->d_lab.as<int32_t>();
    a.n_states = h->n_states;
    a.q0 = h->q0;
    a.out = out;
    a.cap = cap;
    a.total = d_total;
    a.ctl = w->ctl;
    a.lb = w->lb;
    a.lb_cap = w->lb_cap;
    a.n_segs = (int32_t)n_segs;
    a.bstats = w->bstats;
    a.tag_cnt = w->m_tag;
    a.narrow_max = h->knobs.merged_lim > 0 ? h->knobs.merged_lim : INT32_MAX;
    a.seg_cnt = w->m_seg;
    a.seg_base = w->m_seg + n_segs;
    const int waves = kMergedThreads / 64;
    const int grid = (int)std::min<int64_t>((n_segs + waves - 1) / waves, blocks);
    HIP_TRY(launch_dfa_merged(a, grid, s));
    w->last_grid = grid;
    h->pool.mark(w);
    return PFSM_OK;
}

int pfsm_scan_async(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
                    int64_t *d_n_matches, void *hip_stream) {
    if (!h) return fail(PFSM_EINVAL, "NULL handle");
    if (n < 0 || n > kMaxStream) return fail(PFSM_EINVAL, "n must be in [0, 2^31 - 16]");
    if (cap < 0) return fail(PFSM_EINVAL, "cap must be >= 0");
    if (!d_n_matches) return fail(PFSM_EINVAL, "d_n_matches is NULL");
    if (n > 0 && !d_input) return fail(PFSM_EINVAL, "d_input is NULL");
    if (cap > 0 && !d_out) return fail(PFSM_EINVAL, "d_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (n == 0) {
        HIP_TRY(launch_write_zero(d_n_matches, s));
        return PFSM_OK;
    }
    if (h->kind == 1)
        return nfa_scan_async(h->nfa.get(), d_input, n, reinterpret_cast<MatchOut *>(d_out), cap, d_n_matches, s);
    if (h->knobs.merged && h->merged_ok)
        return merged_launch(h, d_input, n, reinterpret_cast<MatchOut *>(d_out), cap, d_n_matches, s);
    return dfa_launch(h, d_input, n, nullptr, 0, reinterpret_cast<MatchOut *>(d_out), cap, d_n_matches, s);
}

int pfsm_scan(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
              int64_t *n_matches, void *hip_stream) {
    if (!h || !n_matches) return fail(PFSM_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Workspace *w;
    const int nb = h->kind == 1 ? nfa_grid_blocks(h->nfa.get()) : h->n_blocks;
    int rc = (h->kind == 1 ? nfa_pool(h->nfa.get()) : &h->pool)->get(s, nb, &w);
    if (rc) return rc;
    rc = pfsm_scan_async(h, d_input, n, d_out, cap, w->h_total_dev, hip_stream);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    *n_matches = *reinterpret_cast<volatile int64_t *>(w->h_total);
    if (*n_matches > cap)
        return fail(PFSM_EOVERFLOW, "%lld matches, capacity %lld", (long long)*n_matches, (long long)cap);
    return PFSM_OK;
}

}  // extern "C"

// ---------------------------------------------------- scan without allocation

namespace {

// Scratch of pfsm_scan_noalloc, one copy per GPU in the module's own global
// memory: the scan's control block, its look-back words, the per-workgroup
// counters and the walks a workgroup parks out of LDS.  Sized for at most
// kNaBlocks workgroups and kNaSegs segments (about 32.3 MiB).
constexpr int kNaBlocks = 512;
constexpr int kNaSegs = kMaxSegs;
constexpr int kNaLbWords = kNaSegs + kNaBlocks;
constexpr size_t kNaOffLb = 256;  // after the ScanCtl
constexpr size_t kNaOffStats = kNaOffLb + (size_t)kNaLbWords * sizeof(unsigned long long);
constexpr size_t kNaOffSpill = (kNaOffStats + (size_t)kNaBlocks * 4 * sizeof(long long) + 255) / 256 * 256;
constexpr size_t kNaBytes = kNaOffSpill + (size_t)kNaBlocks * kDfaSpill * 16;
static_assert(sizeof(ScanCtl) <= kNaOffLb, "control block overlaps the look-back words");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Zero the control block and the look-back words (the counters and the
// parked walks are written before they are read).
__global__ void noalloc_clear_kernel(unsigned long long *p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Per device: the device address of `scratch` (hipGetSymbolAddress) and
// whether its control words have been cleared.
constexpr int kNaMaxDevices = 64;
struct NaDevice {
    unsigned char *ptr = nullptr;
    bool cleared = false;
};
std::mutex g_na_mu;
NaDevice g_na[kNaMaxDevices];

// Set-up on the current device, once: look up the scratch address and clear
// its control words on `s`, ahead of the first scan.
int noalloc_scratch(hipStream_t s, unsigned char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(PFSM_EINVAL, "device %d beyond the %d supported", dev, kNaMaxDevices);
    std::lock_guard<std::mutex> lk(g_na_mu);
    NaDevice &d = g_na[dev];
    if (!d.ptr) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        d.ptr = static_cast<unsigned char *>(p);
    }
    if (!d.cleared) {
        const int64_t words = (int64_t)(kNaOffStats / sizeof(unsigned long long));
        hipLaunchKernelGGL(noalloc_clear_kernel, dim3(64), dim3(256), 0, s,
                           reinterpret_cast<unsigned long long *>(d.ptr), words);
        HIP_TRY(hipGetLastError());
        d.cleared = true;
    }
    *out = d.ptr;
    return PFSM_OK;
}

}  // namespace

extern "C" {

int pfsm_scan_noalloc(pfsm_t *h, const uint8_t *d_input, int64_t n, pfsm_match_t *d_out, int64_t cap,
                      int64_t *d_n_matches, void *hip_stream) {
    if (!h) return fail(PFSM_EINVAL, "NULL handle");
    if (h->kind != 0) return fail(PFSM_ENOSYS, "the scan without allocation takes DFA handles");
    if (n < 0 || n > kMaxStream) return fail(PFSM_EINVAL, "n must be in [0, 2^31 - 16]");
    if (cap < 0) return fail(PFSM_EINVAL, "cap must be >= 0");
    if (!d_n_matches) return fail(PFSM_EINVAL, "d_n_matches is NULL");
    if (n > 0 && !d_input) return fail(PFSM_EINVAL, "d_input is NULL");
    if (cap > 0 && !d_out) return fail(PFSM_EINVAL, "d_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int blocks = std::min(h->n_blocks, kNaBlocks);
    int64_t seg = 0;
    int rounds = 0;
    if (n > 0)
        plan_segments(n, blocks, h->knobs.segment > 0 ? h->knobs.segment : kDfaSegMax, dfa_seg_floor(n, h->res_bytes),
                      &seg, &rounds);
    const int64_t n_segs = n > 0 ? (n + seg - 1) / seg : 0;
    if (n_segs > kNaSegs)
        return fail(PFSM_EINVAL, "%lld segments of %lld bytes exceed the %d the scratch holds (raise the segment size)",
                    (long long)n_segs, (long long)seg, kNaSegs);
    unsigned char *base = nullptr;
    int rc = noalloc_scratch(s, &base);
    if (rc) return rc;
    if (n == 0) {
        HIP_TRY(launch_write_zero(d_n_matches, s));
        return PFSM_OK;
    }
    DfaArgs a;
    dfa_common_args(h, d_input, n, reinterpret_cast<MatchOut *>(d_out), cap, d_n_matches, a);
    a.ctl = reinterpret_cast<ScanCtl *>(base);
    a.lb = reinterpret_cast<unsigned long long *>(base + kNaOffLb);
    a.lb_cap = kNaLbWords;
    a.bstats = reinterpret_cast<long long *>(base + kNaOffStats);
    a.spill = base + kNaOffSpill;
    a.seg = seg;
    a.n_segs = (int32_t)n_segs;
    // Matches go straight to their places: no staging rows.
    DfaDefer d;
    std::memset(&d, 0, sizeof d);
    const int grid = (int)std::min<int64_t>(n_segs, blocks);
    void *args[] = {&a, &d};
    HIP_TRY(hipLaunchKernel(h->kernel, dim3(grid), dim3(kDfaThreads), args, h->lds_bytes, s));
    return PFSM_OK;
}

int pfsm_set_option(pfsm_t *h, int32_t option, int64_t value, void *hip_stream) {
    if (!h) return fail(PFSM_EINVAL, "NULL handle");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Knobs *k = h->kind == 1 ? nfa_knobs(h->nfa.get()) : &h->knobs;
    switch (option) {
    case PFSM_OPT_SEGMENT:
        if (value != 0 && (value < 256 || value > 65536 || value % 16))
            return fail(PFSM_EINVAL, "segment must be 0 or a multiple of 16 in [256, 65536]");
        k->segment = value;
        return PFSM_OK;
    case PFSM_OPT_WORKGROUPS_PER_CU:
        if (value < 0 || value > 64) return fail(PFSM_EINVAL, "workgroups per CU must be in [0, 64]");
        k->wpc = (int32_t)value;
        if (h->kind == 1) return nfa_apply_knobs(h->nfa.get(), false, s);
        h->n_blocks = grid_blocks(h->occ, h->cus, k->wpc);
        return PFSM_OK;
    case PFSM_OPT_TABLE_BUDGET:
        if (h->kind == 1) return fail(PFSM_ENOSYS, "the table budget applies to DFA handles");
        if (value < -1 || value > kDfaLdsLimit) return fail(PFSM_EINVAL, "table budget must be in [-1, %d]", kDfaLdsLimit);
        if (value == k->table_budget) return PFSM_OK;
        k->table_budget = value;
        HIP_TRY(hipDeviceSynchronize());  // scans in flight read the current caches
        return dfa_upload_caches(h, s);
    case PFSM_OPT_MERGED_WALKS:
        if (value != 0 && value != 1) return fail(PFSM_EINVAL, "merged walks must be 0 or 1");
        if (value == 1 && (h->kind == 1 || !h->merged_ok))
            return fail(PFSM_ENOSYS, "tag-merged stepping needs a DFA with at most %d states", kMergedStates);
        k->merged = (int32_t)value;
        return PFSM_OK;
    case PFSM_OPT_MERGED_COUNT_LIMIT:
        if (value < 0 || value > INT32_MAX) return fail(PFSM_EINVAL, "merged count limit must be in [0, 2^31 - 1]");
        k->merged_lim = (int32_t)value;
        return PFSM_OK;
    case PFSM_OPT_PAIR_CACHE:
        if (h->kind == 0) return fail(PFSM_ENOSYS, "the pair cache applies to NFA handles");
        if (value != 0 && value != 1) return fail(PFSM_EINVAL, "pair cache must be 0 or 1");
        if (value == k->pair_cache) return PFSM_OK;
        k->pair_cache = (int32_t)value;
        return nfa_apply_knobs(h->nfa.get(), true, s);
    default:
        return fail(PFSM_EINVAL, "unknown option %d", option);
    }
}

int pfsm_get_option(const pfsm_t *h, int32_t option, int64_t *value) {
    if (!h || !value) return fail(PFSM_EINVAL, "NULL argument");
    const Knobs *k = h->kind == 1 ? nfa_knobs(h->nfa.get()) : &h->knobs;
    switch (option) {
    case PFSM_OPT_SEGMENT: *value = k->segment; return PFSM_OK;
    case PFSM_OPT_WORKGROUPS_PER_CU: *value = k->wpc; return PFSM_OK;
    case PFSM_OPT_TABLE_BUDGET:
        if (h->kind == 1) return fail(PFSM_ENOSYS, "the table budget applies to DFA handles");
        *value = k->table_budget;
        return PFSM_OK;
    case PFSM_OPT_PAIR_CACHE:
        if (h->kind == 0) return fail(PFSM_ENOSYS, "the pair cache applies to NFA handles");
        *value = k->pair_cache;
        return PFSM_OK;
    case PFSM_OPT_MAX_WORKGROUPS_PER_CU:
        *value = h->kind == 1 ? nfa_occupancy(h->nfa.get()) : (k->merged && h->merged_ok ? h->m_occ : h->occ);
        return PFSM_OK;
    case PFSM_OPT_MERGED_WALKS: *value = k->merged; return PFSM_OK;
    case PFSM_OPT_MERGED_COUNT_LIMIT: *value = k->merged_lim; return PFSM_OK;
    case PFSM_OPT_LAYOUT_EPOCH:
        *value = (int64_t)(h->kind == 1 ? nfa_layout_epoch(h->nfa.get()) : h->layout_epoch);
        return PFSM_OK;
    case PFSM_OPT_RESIDENT_TABLE:
        if (h->kind == 1) return fail(PFSM_ENOSYS, "the table encoding applies to DFA handles");
        *value = (h->enc == kEnc8 || h->enc == kEnc8D || h->enc == kEnc16) ? 1 : 0;
        return PFSM_OK;
    default:
        return fail(PFSM_EINVAL, "unknown option %d", option);
    }
}

}  // extern "C"

namespace {

// Device buffers of batched scans on one stream, kept until
// pfsm_release_cached.  The destructor makes no HIP call: it may run from
// static destruction at exit, after the runtime has gone.
struct BatchWs {
    int32_t *seg_first = nullptr, *seg_stream = nullptr, *n_segs = nullptr, *seg_base = nullptr;
    int64_t *bases = nullptr, *seg = nullptr, *stream_lo = nullptr, *stream_hi = nullptr;
    MatchOut *stage = nullptr;
    BatchInfo *info = nullptr, *h_info = nullptr;  // h_info: pinned
    int64_t c_first = 0, c_seg = 0, c_nsegs = 0, c_base = 0, c_bases = 0, c_lo = 0, c_hi = 0, c_stage = 0, c_segsz = 0;
    // Frees every buffer (the device must be idle).
    void release() {
        void *dev[] = {seg_first, seg_stream, n_segs, seg_base, bases, seg, stream_lo, stream_hi, stage, info};
        for (void *p : dev)
            if (p) (void)hipFree(p);
        if (h_info) (void)hipHostFree(h_info);
    }
};

std::mutex g_batch_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<BatchWs>> g_batch;

// Replace *p by a buffer of at least `need` elements when it holds fewer
// (the stream is synchronised first; contents are not kept).
template <typename T>
int grow(T **p, int64_t *cap, int64_t need, hipStream_t s) {
    if (need <= *cap) return PFSM_OK;
    HIP_TRY(hipStreamSynchronize(s));
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    HIP_TRY(hipMalloc(p, sizeof(T) * (size_t)need));
    *cap = need;
    return PFSM_OK;
}

int batch_ws(hipStream_t s, BatchWs **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto &slot = g_batch[{dev, s}];
    if (!slot) {
        auto w = std::make_unique<BatchWs>();
        HIP_TRY(hipMalloc(&w->info, sizeof(BatchInfo)));
        HIP_TRY(hipHostMalloc(&w->h_info, sizeof(BatchInfo), hipHostMallocDefault));
        slot = std::move(w);
    }
    *out = slot.get();
    return PFSM_OK;
}

}  // namespace

extern "C" {

static int batch_check(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data, const int64_t *d_stream_off,
                       const int32_t *d_stream_automaton, int32_t n_streams, pfsm_match_t *d_out, int64_t cap,
                       int64_t *d_match_off) {
    if (!hs || !d_match_off) return fail(PFSM_EINVAL, "NULL argument");
    if (n_automata < 1 || n_automata > kMaxBatchAutomata)
        return fail(PFSM_EINVAL, "n_automata must be in [1, %d]", kMaxBatchAutomata);
    for (int a = 0; a < n_automata; ++a)
        if (!hs[a]) return fail(PFSM_EINVAL, "handle %d is NULL", a);
    if (n_streams < 0) return fail(PFSM_EINVAL, "n_streams must be >= 0");
    if (n_streams > 0 && (!d_stream_off || !d_stream_automaton || !d_data))
        return fail(PFSM_EINVAL, "stream arrays are NULL");
    if (cap < 0) return fail(PFSM_EINVAL, "cap must be >= 0");
    if (cap > 0 && !d_out) return fail(PFSM_EINVAL, "d_out is NULL");
    return PFSM_OK;
}

// Everything of a batch on the device: plan, one scan launch per automaton,
// offsets and gather.  With `may_grow` the buffers are first grown to what
// the arguments need (allocations and synchronisation); without it a buffer
// that is too small is an error, so the work can be captured in a graph.
static int batch_enqueue(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data, const int64_t *d_stream_off,
                         const int32_t *d_stream_automaton, int32_t n_streams, pfsm_match_t *d_out, int64_t cap,
                         int64_t *d_match_off, hipStream_t s, bool may_grow, BatchWs **bw_out,
                         std::vector<Workspace *> &ws, int32_t *seg_cap_out, int *lb_cap_out) {
    BatchWs *bw;
    int rc = batch_ws(s, &bw);
    if (rc) return rc;
    const int64_t ns = std::max(n_streams, 1);
    const int64_t need[9] = {ns, ns, ns, n_automata, n_automata, n_automata + 1, std::max<int64_t>(cap, 1), 4 * ns + 4096,
                             n_automata};
    const int64_t have[9] = {bw->c_first, bw->c_lo, bw->c_hi, bw->c_nsegs, bw->c_base, bw->c_bases, bw->c_stage, bw->c_seg,
                             bw->c_segsz};
    if (!may_grow) {
        for (int k = 0; k < 9; ++k)
            if (have[k] < need[k])
                return fail(PFSM_ENOMEM, "batch buffers are smaller than this batch needs: run pfsm_scan_batch "
                                         "with the same sizes once first");
    } else {
        if ((rc = grow(&bw->seg_first, &bw->c_first, need[0], s))) return rc;
        if ((rc = grow(&bw->stream_lo, &bw->c_lo, need[1], s))) return rc;
        if ((rc = grow(&bw->stream_hi, &bw->c_hi, need[2], s))) return rc;
        if ((rc = grow(&bw->n_segs, &bw->c_nsegs, need[3], s))) return rc;
        if ((rc = grow(&bw->seg_base, &bw->c_base, need[4], s))) return rc;
        if ((rc = grow(&bw->bases, &bw->c_bases, need[5], s))) return rc;
        if ((rc = grow(&bw->stage, &bw->c_stage, need[6], s))) return rc;
        if ((rc = grow(&bw->seg_stream, &bw->c_seg, need[7], s))) return rc;
        if ((rc = grow(&bw->seg, &bw->c_segsz, need[8], s))) return rc;
    }
    ws.assign(n_automata, nullptr);
    for (int a = 0; a < n_automata; ++a) {
        pfsm_t *h = hs[a];
        const int nb = h->kind == 1 ? nfa_grid_blocks(h->nfa.get()) : h->n_blocks;
        if ((rc = (h->kind == 1 ? nfa_pool(h->nfa.get()) : &h->pool)->get(s, nb, &ws[a]))) return rc;
    }
    int lb_cap = 1 << 30;
    for (Workspace *w : ws) lb_cap = std::min(lb_cap, w->lb_cap);
    BatchPlanArgs p{};
    p.stream_off = d_stream_off;
    p.stream_aut = d_stream_automaton;
    p.n_streams = n_streams;
    p.n_aut = n_automata;
    p.seg_min = kBatchSegMin;
    p.seg_max = kBatchSegMax;
    p.max_stream = kMaxStream;
    p.seg = bw->seg;
    for (int a = 0; a < n_automata; ++a) {
        p.blocks[a] = hs[a]->kind == 1 ? nfa_grid_blocks(hs[a]->nfa.get()) : hs[a]->n_blocks;
        p.seg_fix[a] = (int32_t)(hs[a]->kind == 1 ? nfa_knobs(hs[a]->nfa.get())->segment : hs[a]->knobs.segment);
    }
    p.seg_first = bw->seg_first;
    p.seg_stream = bw->seg_stream;
    p.n_segs = bw->n_segs;
    p.seg_base = bw->seg_base;
    p.bases = bw->bases;
    p.stream_lo = bw->stream_lo;
    p.stream_hi = bw->stream_hi;
    p.info = bw->info;
    p.seg_cap = (int32_t)std::min<int64_t>(bw->c_seg, 1 << 30);
    p.lb_cap = lb_cap;
    HIP_TRY(launch_batch_plan(p, s));
    // One launch per automaton, each after the previous one's matches.
    for (int a = 0; a < n_automata; ++a) {
        SegPlan sp{};
        sp.stream_off = d_stream_off;
        sp.seg_stream = bw->seg_stream;
        sp.seg_first = bw->seg_first;
        sp.n_segs_dev = bw->n_segs + a;
        sp.seg_base_dev = bw->seg_base + a;
        sp.base_dev = bw->bases + a;
        sp.seg_dev = bw->seg + a;
        sp.stream_lo = bw->stream_lo;
        sp.stream_hi = bw->stream_hi;
        pfsm_t *h = hs[a];
        rc = h->kind == 1 ? nfa_launch(h->nfa.get(), d_data, 0, &sp, kBatchSegMax, bw->stage, bw->c_stage,
                                       bw->bases + a + 1, s)
                          : dfa_launch(h, d_data, 0, &sp, kBatchSegMax, bw->stage, bw->c_stage, bw->bases + a + 1, s);
        if (rc) return rc;
    }
    BatchGatherArgs g{};
    g.n_streams = n_streams;
    g.stream_lo = bw->stream_lo;
    g.stream_hi = bw->stream_hi;
    g.match_off = d_match_off;
    g.stage = bw->stage;
    g.stage_cap = bw->c_stage;
    g.out = reinterpret_cast<MatchOut *>(d_out);
    g.cap = cap;
    g.info = bw->info;
    HIP_TRY(launch_batch_gather(g, s));
    *bw_out = bw;
    *seg_cap_out = p.seg_cap;
    *lb_cap_out = lb_cap;
    return PFSM_OK;
}

}  // extern "C"

namespace pfsmk {

int batch_run(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data, const int64_t *d_stream_off,
              const int32_t *d_stream_automaton, int32_t n_streams, MatchOut *d_out, int64_t cap,
              int64_t *d_match_off, hipStream_t s, BatchRun *run) {
    int rc = batch_check(hs, n_automata, d_data, d_stream_off, d_stream_automaton, n_streams,
                         reinterpret_cast<pfsm_match_t *>(d_out), cap, d_match_off);
    if (rc) return rc;
    BatchWs *bw;
    rc = batch_enqueue(hs, n_automata, d_data, d_stream_off, d_stream_automaton, n_streams,
                       reinterpret_cast<pfsm_match_t *>(d_out), cap, d_match_off, s, true, &bw, run->ws,
                       &run->seg_cap, &run->lb_cap);
    if (rc) return rc;
    run->bw = bw;
    run->info = bw->info;
    run->stream_lo = bw->stream_lo;
    run->stream_hi = bw->stream_hi;
    run->stage_cap = bw->c_stage;
    return PFSM_OK;
}

int batch_fit(BatchRun *run, const BatchInfo &info, hipStream_t s, bool *again) {
    *again = false;
    if (info.err) return fail(PFSM_EINVAL, "invalid stream table");
    BatchWs *bw = static_cast<BatchWs *>(run->bw);
    int rc;
    if (info.total_segs > run->seg_cap) {
        if ((rc = grow(&bw->seg_stream, &bw->c_seg, (int64_t)info.total_segs + 4096, s))) return rc;
        *again = true;
    }
    if (info.max_segs > run->lb_cap) {
        for (Workspace *w : run->ws)
            if ((rc = grow_lb(w, info.max_segs + 1024))) return rc;
        *again = true;
    }
    return PFSM_OK;
}

}  // namespace pfsmk

extern "C" {

int pfsm_scan_batch(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data, const int64_t *d_stream_off,
                    const int32_t *d_stream_automaton, int32_t n_streams, pfsm_match_t *d_out, int64_t cap,
                    int64_t *d_match_off, int64_t *n_matches, void *hip_stream) {
    if (!n_matches) return fail(PFSM_EINVAL, "NULL argument");
    int rc = batch_check(hs, n_automata, d_data, d_stream_off, d_stream_automaton, n_streams, d_out, cap, d_match_off);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    for (int attempt = 0;; ++attempt) {
        BatchWs *bw;
        std::vector<Workspace *> ws;
        int32_t seg_cap;
        int lb_cap;
        if ((rc = batch_enqueue(hs, n_automata, d_data, d_stream_off, d_stream_automaton, n_streams, d_out, cap,
                                d_match_off, s, true, &bw, ws, &seg_cap, &lb_cap)))
            return rc;
        HIP_TRY(hipMemcpyAsync(bw->h_info, bw->info, sizeof(BatchInfo), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const BatchInfo info = *bw->h_info;
        if (info.err == 1) return fail(PFSM_EINVAL, "a stream names an automaton outside [0, %d)", n_automata);
        if (info.err)
            return fail(PFSM_EINVAL, "stream offsets must not decrease and streams must be at most 2^31 - 16 bytes");
        const bool more_segs = info.total_segs > seg_cap, more_lb = info.max_segs > lb_cap;
        if (!more_segs && !more_lb) {
            *n_matches = info.total;
            if (info.total > cap)
                return fail(PFSM_EOVERFLOW, "%lld matches, capacity %lld", (long long)info.total, (long long)cap);
            return PFSM_OK;
        }
        if (attempt > 0) return fail(PFSM_EHIP, "batch plan did not fit after growing its buffers");
        if (more_segs && (rc = grow(&bw->seg_stream, &bw->c_seg, (int64_t)info.total_segs + 4096, s))) return rc;
        if (more_lb)
            for (Workspace *w : ws)
                if ((rc = grow_lb(w, info.max_segs + 1024))) return rc;
    }
}

int pfsm_scan_batch_async(pfsm_t *const *hs, int32_t n_automata, const uint8_t *d_data, const int64_t *d_stream_off,
                          const int32_t *d_stream_automaton, int32_t n_streams, pfsm_match_t *d_out, int64_t cap,
                          int64_t *d_match_off, void *hip_stream) {
    int rc = batch_check(hs, n_automata, d_data, d_stream_off, d_stream_automaton, n_streams, d_out, cap, d_match_off);
    if (rc) return rc;
    BatchWs *bw;
    std::vector<Workspace *> ws;
    int32_t seg_cap;
    int lb_cap;
    return batch_enqueue(hs, n_automata, d_data, d_stream_off, d_stream_automaton, n_streams, d_out, cap, d_match_off,
                         static_cast<hipStream_t>(hip_stream), false, &bw, ws, &seg_cap, &lb_cap);
}

int pfsm_last_stats(pfsm_t *h, pfsm_stats *out, void *hip_stream) {
    if (!h || !out) return fail(PFSM_EINVAL, "NULL argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Workspace *w = (h->kind == 1 ? nfa_pool(h->nfa.get()) : &h->pool)->find(s);
    if (!w) return fail(PFSM_ENOENT, "no scan on this stream yet");
    long long v[4];
    int rc = workspace_stats(w, v);
    if (rc) return rc;
    out->transitions = v[0];
    out->activations = v[1];
    out->long_walks = v[2];
    out->matches = v[3];
    return PFSM_OK;
}

void pfsm_free(pfsm_t *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

void pfsm_release_cached(void) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (g_batch.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : g_batch) kv.second->release();
    g_batch.clear();
}

}  // extern "C"

// ---------------------------------------------------------------- streams

namespace pfsmk {

uint64_t handle_edits(const pfsm_t *h) { return h->edits; }

int piece_scan(pfsm_t *h, const uint8_t *x, int64_t n, MatchOut *out, int64_t cap, int64_t *d_total,
               const int64_t *d_base, const CarryOut *carry, hipStream_t s) {
    if (h->kind == 1) return nfa_launch(h->nfa.get(), x, n, nullptr, 0, out, cap, d_total, s, d_base, carry);
    return dfa_launch(h, x, n, nullptr, 0, out, cap, d_total, s, d_base, carry);
}

int piece_resume(pfsm_t *h, const uint8_t *x, int64_t n, int32_t base, const CarrySet &in, int64_t *cnt,
                 const int64_t *off, MatchOut *out, int64_t cap, const CarryOut &carry, int write, hipStream_t s) {
    if (h->kind == 1) return nfa_resume(h->nfa.get(), x, n, base, in, cnt, off, out, cap, carry, write, s);
    DfaResumeArgs r;
    std::memset(&r, 0, sizeof r);
    r.x = x;
    r.n = n;
    r.base = base;
    // the table as loaded (symbol columns through the byte map), not the
    // byte-indexed resident image
    r.tbl16 = h->tbl16 ? 1 : 0;
    r.n_symbols = h->n_symbols;
    r.identity = h->identity ? 1 : 0;
    r.tbl = h->d_tbl.p;
    r.b2s = h->d_b2s.as<int16_t>();
    r.flags = h->d_flags.as<uint8_t>();
    r.lab_off = h->d_lab_off.as<int32_t>();
    r.lab = h->d_lab.as<int32_t>();
    r.in = in;
    r.cnt = cnt;
    r.off = off;
    r.out = out;
    r.cap = cap;
    r.carry = carry;
    r.write = write;
    HIP_TRY(launch_dfa_resume(r, s));
    return PFSM_OK;
}

}  // namespace pfsmk
