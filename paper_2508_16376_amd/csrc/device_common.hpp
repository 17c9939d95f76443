// Device helpers shared by the kernels: operator evaluation, forcing, wave scans.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "design.hpp"

namespace riros {

__device__ __forceinline__ uint64_t width_mask(uint32_t w)
{
    return w >= 64 ? ~0ull : ((1ull << w) - 1ull);
}

__device__ __forceinline__ int dev_arity(uint32_t op)
{
    // CONST PI REG ADD SUB AND OR XOR NOT MUX SHL SHR EQ NE ULT SLICE CONCAT MUL
    // 0     0  1   2   2   2   2  2   1   3   1   1   2  2  2   1     2      2
    return op == RIROS_OP_MUX ? 3
         : (op == RIROS_OP_NOT || op == RIROS_OP_SHL || op == RIROS_OP_SHR || op == RIROS_OP_SLICE) ? 1
         : 2;
}

// Result of a combinational operator on masked operand values (the operator
// table of riros.h).  Shift amounts and the CONCAT low width live in the
// descriptor's b and c fields (pb, pc).
__device__ __forceinline__ uint64_t apply_opw(uint32_t op, uint32_t width, uint32_t pb, uint32_t pc, uint64_t x0,
                                              uint64_t x1, uint64_t x2)
{
    uint64_t r;
    switch (op) {
    case RIROS_OP_ADD: r = x0 + x1; break;
    case RIROS_OP_SUB: r = x0 - x1; break;
    case RIROS_OP_AND: r = x0 & x1; break;
    case RIROS_OP_OR: r = x0 | x1; break;
    case RIROS_OP_XOR: r = x0 ^ x1; break;
    case RIROS_OP_NOT: r = ~x0; break;
    case RIROS_OP_MUX: r = x0 != 0 ? x2 : x1; break;
    case RIROS_OP_SHL: r = pb >= 64 ? 0 : (x0 << pb); break;
    case RIROS_OP_SHR:
    case RIROS_OP_SLICE: r = pb >= 64 ? 0 : (x0 >> pb); break;
    case RIROS_OP_EQ: r = x0 == x1; break;
    case RIROS_OP_NE: r = x0 != x1; break;
    case RIROS_OP_ULT: r = x0 < x1; break;
    case RIROS_OP_CONCAT: r = (pc >= 64 ? 0 : (x0 << pc)) | x1; break;
    case RIROS_OP_MUL: r = x0 * x1; break;
    default: r = 0; break;
    }
    return r & width_mask(width);
}

__device__ __forceinline__ uint64_t apply_op(const Desc& d, uint64_t x0, uint64_t x1, uint64_t x2)
{
    return apply_opw(d.op, d.width, d.b, d.c, x0, x1, x2);
}

// Stuck-at forcing of one bit (Sec. IV-A: the faulty value replaces the
// computed one at the injected node).
// The fault's effect on its site's value in cycle t: a stuck-at fault
// (stuck 0 or 1) forces bit `bit` in every cycle; a bit flip (RIROS_FAULT_FLIP)
// inverts it in cycle t0 only.
__device__ __forceinline__ uint64_t apply_fault(uint64_t v, uint32_t bit, uint32_t stuck, uint32_t t, uint32_t t0)
{
    const uint64_t m = 1ull << bit;
    if (stuck == RIROS_FAULT_FLIP) return t == t0 ? (v ^ m) : v;
    return stuck ? (v | m) : (v & ~m);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Orders one wavefront's LDS accesses across its lanes (writes before the
// call are seen by reads after it) without a workgroup barrier, so that one
// wavefront of a larger workgroup can use it alone.  The workgroup-scope
// fences wait for the wave's outstanding LDS operations; the wave barrier
// keeps the compiler from moving memory operations across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint64_t make_u64(uint32_t lo, uint32_t hi)
{
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

}  // namespace riros
