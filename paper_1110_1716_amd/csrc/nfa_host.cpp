// NFA host side (placeholder until the NFA kernels land).
#include "pfsm_nfa.h"

namespace pfsmk {

struct NfaHost {
    WorkspacePool pool;
};
void NfaDeleter::operator()(NfaHost *p) const { delete p; }

int nfa_load(const pfsm_nfa_desc *, hipStream_t, NfaPtr *) {
    return fail(PFSM_ENOSYS, "NFA scans are not available yet");
}
int nfa_add_pattern(NfaHost *, const pfsm_nfa_desc *, hipStream_t) {
    return fail(PFSM_ENOSYS, "NFA scans are not available yet");
}
int nfa_remove_pattern(NfaHost *, int32_t, hipStream_t) {
    return fail(PFSM_ENOSYS, "NFA scans are not available yet");
}
int nfa_scan_async(NfaHost *, const uint8_t *, int64_t, MatchOut *, int64_t, int64_t *, hipStream_t) {
    return fail(PFSM_ENOSYS, "NFA scans are not available yet");
}
int nfa_grid_blocks(NfaHost *) { return 1; }
WorkspacePool *nfa_pool(NfaHost *h) { return &h->pool; }

}  // namespace pfsmk
