// NFA host side (placeholder until the NFA kernels land).
#include "pfsm_nfa.h"

namespace pfsmk {

struct NfaHost {};
void NfaDeleter::operator()(NfaHost *p) const { delete p; }

int nfa_load(const pfsm_nfa_desc *, hipStream_t, NfaPtr *, std::string *err) {
    *err = "NFA scans are not available yet";
    return PFSM_ENOSYS;
}
int nfa_add_pattern(NfaHost *, const pfsm_nfa_desc *, hipStream_t, std::string *err) {
    *err = "NFA scans are not available yet";
    return PFSM_ENOSYS;
}
int nfa_remove_pattern(NfaHost *, int32_t, hipStream_t, std::string *err) {
    *err = "NFA scans are not available yet";
    return PFSM_ENOSYS;
}
int nfa_scan_async(NfaHost *, const uint8_t *, int64_t, MatchOut *, int64_t, int64_t *, hipStream_t,
                   std::string *err) {
    *err = "NFA scans are not available yet";
    return PFSM_ENOSYS;
}
int nfa_last_stats(NfaHost *, hipStream_t, long long *, std::string *err) {
    *err = "NFA scans are not available yet";
    return PFSM_ENOSYS;
}

}  // namespace pfsmk
