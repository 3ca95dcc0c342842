// Status and error reporting of the C ABI, and an opt-in per-kernel timer
// (HIP events recorded on the launch stream around each timed launch).
#include <cstring>
#include <string>
#include <vector>

#include "sf_internal.hpp"

namespace sf {

static thread_local char g_err[512] = {0};

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// --- kernel timer ---------------------------------------------------------
struct ProfRec {
    std::string name;
    hipEvent_t start, stop;
};
static bool g_prof_on = false;
static std::string g_prof_only;  // record only launches of this name (empty = all)
static std::vector<hipEvent_t> g_prof_pool;
static size_t g_prof_next = 0;
static std::vector<ProfRec> g_prof_recs;

ProfScope::ProfScope(const char *name, hipStream_t st) : st_(st), idx_(-1)
{
    if (!g_prof_on || g_prof_next + 2 > g_prof_pool.size()) return;
    if (!g_prof_only.empty() && g_prof_only != name) return;
    ProfRec r{name, g_prof_pool[g_prof_next], g_prof_pool[g_prof_next + 1]};
    g_prof_next += 2;
    if (hipEventRecord(r.start, st) != hipSuccess) return;  // the timer is optional: this launch goes untimed
    idx_ = (int)g_prof_recs.size();
    g_prof_recs.push_back(r);
}

ProfScope::~ProfScope()
{
    // A failed stop record shows up as an error of sf_prof_query for this launch.
    if (idx_ >= 0) (void)hipEventRecord(g_prof_recs[idx_].stop, st_);
}

}  // namespace sf

extern "C" int sf_prof_enable(int max_launches)
{
    using namespace sf;
    clear_error();
    SF_REQUIRE(max_launches > 0 && max_launches <= (1 << 20), SF_EINVAL,
               "sf_prof_enable: max_launches out of range");
    for (hipEvent_t e : g_prof_pool) (void)hipEventDestroy(e);
    g_prof_pool.assign((size_t)2 * max_launches, nullptr);
    for (auto &e : g_prof_pool)
        // Timing-only events: no system-scope fence when one is recorded between
        // two launches of a timed region (sf_prof_query only reads timestamps).
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
            return fail(SF_EHIP, "sf_prof_enable: hipEventCreateWithFlags");
    g_prof_next = 0;
    g_prof_recs.clear();
    g_prof_on = true;
    return SF_OK;
}

extern "C" int sf_prof_only(const char *kernel)
{
    sf::clear_error();
    sf::g_prof_only = kernel ? kernel : "";
    return SF_OK;
}

extern "C" int sf_prof_disable(void)
{
    sf::g_prof_on = false;
    return SF_OK;
}

extern "C" int sf_prof_query(const char *kernel, double *total_ms, int *launches)
{
    using namespace sf;
    clear_error();
    SF_REQUIRE(kernel && total_ms && launches, SF_EINVAL, "sf_prof_query: NULL pointer");
    double tot = 0.0;
    int n = 0;
    for (const ProfRec &r : g_prof_recs) {
        if (r.name != kernel) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return fail(SF_EHIP, "sf_prof_query: sync");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            return fail(SF_EHIP, "sf_prof_query: elapsed");
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return SF_OK;
}

extern "C" int sf_abi_version(void) { return SF_ABI_VERSION; }

extern "C" const char *sf_last_error(void) { return sf::g_err; }

// --- checked builds --------------------------------------------------------
#include "sf_check.hpp"

SF_CHECK_TU(abi)

namespace sf {

// Checks i < n for i = 0 .. n (one thread each) and touches no memory, so in a
// checked build the thread i = n records CHK_SELFTEST.
__global__ void check_selftest_kernel(int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    SF_BOUNDS(i < n, CHK_SELFTEST);
}

}  // namespace sf

using namespace sf;

extern "C" int sf_debug_checked(void)
{
#ifdef SF_CHECKED
    return 1;
#else
    return 0;
#endif
}

extern "C" int sf_debug_selftest(int n, void *stream)
{
    clear_error();
    SF_REQUIRE(n >= 0 && n < (1 << 24), SF_EINVAL, "sf_debug_selftest: n must be in [0, 2^24)");
    hipLaunchKernelGGL(check_selftest_kernel, dim3((n + 256) / 256), dim3(256), 0, as_stream(stream), n);
    return launch_status("check_selftest_kernel");
}

extern "C" int sf_debug_check(uint32_t *bits, int clear)
{
    clear_error();
    SF_REQUIRE(bits, SF_EINVAL, "sf_debug_check: NULL pointer");
    *bits = 0;
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_error("sf_debug_check: %s", hipGetErrorString(e));
        return SF_EHIP;
    }
    int (*const readers[])(uint32_t *, bool) = {check_read_combine, check_read_wta, check_read_flow,
                                                check_read_densify, check_read_sgm, check_read_abi};
    for (auto rd : readers)
        if (rd(bits, clear != 0)) {
            set_error("sf_debug_check: reading a check word failed");
            return SF_EHIP;
        }
    return SF_OK;
}
