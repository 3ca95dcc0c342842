// Status and error reporting of the C ABI.
#include <cstring>

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

}  // namespace sf

extern "C" int sf_abi_version(void) { return SF_ABI_VERSION; }

extern "C" const char *sf_last_error(void) { return sf::g_err; }
