// Entry points whose device code lives elsewhere are declared in fockmi.h; this file
// holds the ones not built yet, which report FOCK_ERR_STATE with a message.
#include "plan.hpp"
using namespace fockmi;
extern "C" {
fock_status taylor_step(fockmi_plan, int, void*, const double*, const double*, double, double, int, double*, void*) {
  return fail(FOCK_ERR_STATE, "taylor_step: not available in this build");
}
fock_status taylor_step_vjp(fockmi_plan, int, const void*, const double*, const double*, double, double, int,
                            const void*, void*, double*, void*) {
  return fail(FOCK_ERR_STATE, "taylor_step_vjp: not available in this build");
}
fock_status fock_orthonormalize(fockmi_plan, int, void*, void*) {
  return fail(FOCK_ERR_STATE, "fock_orthonormalize: not available in this build");
}
fock_status fock_apply_batched(fockmi_plan, const void* const*, const void* const*, const int*, void* const*, void*) {
  return fail(FOCK_ERR_STATE, "fock_apply_batched: not available in this build");
}
}
