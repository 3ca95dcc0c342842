// Checked builds: index checks at the accesses whose indices come from data
// (flows, disparities, chain geometry) rather than from the launch grid alone.
// With -DSF_CHECKED (build(checked=True) -> libsf_checked.so) a failed check
// sets its site's bit in a device word of the kernel's source file; the access
// then proceeds exactly as in the normal build, which is in range whenever the
// check holds.  Nothing traps, so a checked run always completes and reports.
// Normal builds compile the checks away.  sf_debug_check collects the words.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sf {

enum CheckSite : int {
    CHK_COMBINE_TAP = 0,   // bilinear taps of D1 at x + F(x)
    CHK_TEMPORAL = 1,      // chained pixel of the temporal check
    CHK_WTA_LR = 2,        // d*_R(x - d*_L) of the LR check
    CHK_FLOW_SAMPLE = 3,   // census samples of a flow candidate
    CHK_DENSIFY = 4,       // source pixel of the densification
    CHK_SGM_COST = 5,      // cost bytes of a chain step inside its chain
    CHK_SGM_SLAB = 6,      // slab bytes of a chain step inside its chain
    CHK_SELFTEST = 31,     // sf_debug_selftest
};

// Per source file: its check word and a host reader (bits of the current
// device; clear = reset them to 0).  Returns 0 on success.
#ifdef SF_CHECKED
#define SF_CHECK_TU(name)                                                                   \
    static __device__ uint32_t sf_check_word;                                               \
    namespace sf {                                                                          \
    int check_read_##name(uint32_t *bits, bool clear)                                       \
    {                                                                                       \
        void *p = nullptr;                                                                  \
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(sf_check_word)) != hipSuccess || !p) return 1; \
        uint32_t v = 0;                                                                     \
        if (hipMemcpy(&v, p, 4, hipMemcpyDeviceToHost) != hipSuccess) return 1;            \
        *bits |= v;                                                                         \
        if (clear) {                                                                        \
            const uint32_t z = 0;                                                           \
            if (hipMemcpy(p, &z, 4, hipMemcpyHostToDevice) != hipSuccess) return 1;        \
        }                                                                                   \
        return 0;                                                                           \
    }                                                                                       \
    }
#define SF_BOUNDS(cond, site)                                              \
    do {                                                                   \
        if (!(cond)) atomicOr(&sf_check_word, 1u << (unsigned)(site));    \
    } while (0)
#else
#define SF_CHECK_TU(name)                                                        \
    namespace sf {                                                               \
    int check_read_##name(uint32_t *, bool) { return 0; }                        \
    }
#define SF_BOUNDS(cond, site) \
    do {                      \
    } while (0)
#endif

int check_read_combine(uint32_t *bits, bool clear);
int check_read_wta(uint32_t *bits, bool clear);
int check_read_flow(uint32_t *bits, bool clear);
int check_read_densify(uint32_t *bits, bool clear);
int check_read_sgm(uint32_t *bits, bool clear);
int check_read_abi(uint32_t *bits, bool clear);

}  // namespace sf
