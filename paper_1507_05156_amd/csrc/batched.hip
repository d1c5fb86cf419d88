// fock_apply_batched: every cell of an FP32 plan in one call.
#include <hip/hip_runtime.h>

#include "../../include/fockmi.h"
#include "plan.hpp"

using namespace fockmi;

namespace fockmi {
extern thread_local std::string g_last_error;
}

extern "C" fock_status fock_apply_batched(fockmi_plan plan, const void* const* u_occ, const void* const* phi,
                                          const int* nphi, void* const* vphi, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(FOCK_ERR_ARG, "plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  fock_status s = p->check_ready(0);
  if (s != FOCK_OK) return s;
  if (!u_occ || !phi || !nphi || !vphi) return fail(FOCK_ERR_ARG, "NULL pointer array");
  for (int ci = 0; ci < (int)p->cells.size(); ++ci) {
    if (!u_occ[ci] || !phi[ci] || !vphi[ci]) return fail(FOCK_ERR_ARG, "cell %d: NULL device pointer", ci);
    if (nphi[ci] < 1) return fail(FOCK_ERR_ARG, "cell %d: nphi must be >= 1", ci);
  }
  for (int ci = 0; ci < (int)p->cells.size(); ++ci) {
    Cell& c = p->cells[ci];
    if ((s = p->general(c, (const c128*)phi[ci], nphi[ci], (const c128*)u_occ[ci], (const c128*)u_occ[ci], c.nb,
                        (c128*)vphi[ci], -1.0 / c.nk, false, (hipStream_t)stream)) != FOCK_OK)
      return s;
  }
  return FOCK_OK;
}
