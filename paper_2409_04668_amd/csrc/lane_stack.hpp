// Per-work-item LIFO of split daughters in HBM (history schedule, and the
// lead stage of the hybrid schedule).
#pragma once
#include "transport_device.hpp"

namespace mcdc {

// Daughter stack in HBM, SoA [field][depth][lane]: each field access of a
// wave is one contiguous 512-byte transaction.
MCDC_DEV void stack_push(const RunArgs &A, uint64_t lane, int cap, int depth, const Part &q) {
    const uint64_t L = A.n_lanes;
    const uint64_t o = (uint64_t)depth * L + lane;
    const uint64_t F = (uint64_t)cap * L;
    A.stk_d[0 * F + o] = q.x[0];
    A.stk_d[1 * F + o] = q.x[1];
    A.stk_d[2 * F + o] = q.x[2];
    A.stk_d[3 * F + o] = q.u[0];
    A.stk_d[4 * F + o] = q.u[1];
    A.stk_d[5 * F + o] = q.u[2];
    A.stk_d[6 * F + o] = q.t;
    A.stk_d[7 * F + o] = q.w;
    A.stk_i[0 * F + o] = q.g;
    A.stk_i[1 * F + o] = q.cell;
    A.stk_i[2 * F + o] = q.ci;
    A.stk_i[3 * F + o] = (int32_t)q.tag;
}

MCDC_DEV void stack_pop(const RunArgs &A, uint64_t lane, int cap, int depth, Part &q) {
    const uint64_t L = A.n_lanes;
    const uint64_t o = (uint64_t)depth * L + lane;
    const uint64_t F = (uint64_t)cap * L;
    q.x[0] = A.stk_d[0 * F + o];
    q.x[1] = A.stk_d[1 * F + o];
    q.x[2] = A.stk_d[2 * F + o];
    q.u[0] = A.stk_d[3 * F + o];
    q.u[1] = A.stk_d[4 * F + o];
    q.u[2] = A.stk_d[5 * F + o];
    q.t = A.stk_d[6 * F + o];
    q.w = A.stk_d[7 * F + o];
    q.g = A.stk_i[0 * F + o];
    q.cell = A.stk_i[1 * F + o];
    q.ci = A.stk_i[2 * F + o];
    q.tag = (uint32_t)A.stk_i[3 * F + o];
    q.k = 0;
    q.seq = 0;
    q.alive = true;
}

}  // namespace mcdc
