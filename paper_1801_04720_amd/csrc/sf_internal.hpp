// Internal helpers shared by the HIP translation units of libsf (host-side
// status handling and a few device primitives for CDNA wave64 code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "sf.h"

namespace sf {

// Thread-local last-error message (defined in abi.hip).
void set_error(const char *fmt, ...);
void clear_error();

inline int fail(int code, const char *what)
{
    set_error("%s", what);
    return code;
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Records HIP events around the enclosed launch when sf_prof_enable() is on.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t st);
    ~ProfScope();

  private:
    hipStream_t st_;
    int idx_;
};

// Check the launch that was just enqueued.
inline int launch_status(const char *kernel)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", kernel, hipGetErrorString(e));
        return SF_EHIP;
    }
    return SF_OK;
}

#define SF_REQUIRE(cond, code, msg)            \
    do {                                       \
        if (!(cond)) return ::sf::fail(code, msg); \
    } while (0)

// ---------------------------------------------------------------------------
// Device primitives.

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 as_u16x2(uint32_t u) { return __builtin_bit_cast(u16x2, u); }

// DPP control codes (GFX9 / CDNA encoding).
enum : int {
    DPP_QUAD_XOR1 = 0xB1,      // quad_perm [1,0,3,2]
    DPP_QUAD_XOR2 = 0x4E,      // quad_perm [2,3,0,1]
    DPP_ROW_SHL1 = 0x101,      // lane i <- lane i+1 within a row of 16
    DPP_ROW_SHR1 = 0x111,      // lane i <- lane i-1 within a row of 16
    DPP_ROW_MIRROR = 0x140,    // lane i <- lane 15-i within a row
    DPP_ROW_HALF_MIRROR = 0x141  // lane i <- lane 7-i within each half row
};

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

// Lanes whose DPP source falls outside their row receive `fill`.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_fill(uint32_t fill, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, CTRL, 0xF, 0xF, false);
}

// Minimum over the 16 lanes of a row, left in every lane of the row.  The DPP
// "old" operand is the identity of the reduction, which lets the compiler fold
// each move into the min itself (v_min_u32_dpp).
__device__ __forceinline__ uint32_t row16_min(uint32_t m)
{
    m = min(m, dpp_fill<DPP_QUAD_XOR1>(0xFFFFFFFFu, m));
    m = min(m, dpp_fill<DPP_QUAD_XOR2>(0xFFFFFFFFu, m));
    m = min(m, dpp_fill<DPP_ROW_HALF_MIRROR>(0xFFFFFFFFu, m));
    m = min(m, dpp_fill<DPP_ROW_MIRROR>(0xFFFFFFFFu, m));
    return m;
}

__device__ __forceinline__ uint32_t row16_max(uint32_t m)
{
    m = max(m, dpp_fill<DPP_QUAD_XOR1>(0u, m));
    m = max(m, dpp_fill<DPP_QUAD_XOR2>(0u, m));
    m = max(m, dpp_fill<DPP_ROW_HALF_MIRROR>(0u, m));
    m = max(m, dpp_fill<DPP_ROW_MIRROR>(0u, m));
    return m;
}

}  // namespace sf
