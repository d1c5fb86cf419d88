// fock_apply_noalloc: the FP32-form application of the exchange operator for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).
//
// Every scratch buffer of the call (the complex64 shadows of the orbitals and
// targets, the Neumaier compensation field and, for 32^3 cells, the FP32 band
// sums) is carved out of one file-scope device array, `scratch`, of
// kNoAllocBytes. Each GPU holds its own copy of the array until the process
// ends; its device address is looked up once per device at plan creation
// (noalloc_setup) and kept per device. Host code never passes the array's name
// to a kernel: in host code that name is only a stand-in for the symbol.
//
// The call runs the grid form of the fused kernel (one workgroup per target),
// the form fock_apply uses for grid lengths up to 24, so that for those cells
// the two calls give the same bits. Every call on a GPU shares that GPU's
// array and leaves its contents behind; calls that overlap on one GPU race.
// The fused kernel writes every compensation and band-sum element before it
// reads it, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fockmi.h"
#include "plan.hpp"

using namespace fockmi;

namespace fockmi {

extern thread_local std::string g_last_error;

constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};
}  // namespace

// Looks up this device's copy of `scratch` (the device must be current). Called
// by fock_plan_create; idempotent per device.
fock_status noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return FOCK_OK;  // the allocation-free call reports it
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return FOCK_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch array address");
  }
  g_noalloc_ptr[device] = ptr;
  return FOCK_OK;
}

}  // namespace fockmi

extern "C" fock_status fock_apply_noalloc(fockmi_plan plan, int cell, const void* u_occ, const void* phi, int nphi,
                                          void* vphi, void* stream) {
  g_last_error.clear();
  if (!plan) return fail(FOCK_ERR_ARG, "plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  fock_status s = p->check_ready(cell);
  if (s != FOCK_OK) return s;
  if (p->prec != FOCK_FP32_COMP) return fail(FOCK_ERR_ARG, "fock_apply_noalloc needs a FOCK_FP32_COMP plan");
  Cell& c = p->cells[cell];
  if (c.f32plain) return fail(FOCK_ERR_SIZE, "fock_apply_noalloc needs a cubic grid");
  if (!u_occ || !phi || !vphi) return fail(FOCK_ERR_ARG, "NULL device pointer");
  if (!aligned16(u_occ) || !aligned16(phi) || !aligned16(vphi))
    return fail(FOCK_ERR_ARG, "device pointers must be 16-byte aligned");
  if (nphi < 1) return fail(FOCK_ERR_ARG, "nphi must be >= 1");
  const size_t bu = (size_t)c.nk * c.nb * c.nr * sizeof(c128);
  const size_t bp = (size_t)c.nk * nphi * c.nr * sizeof(c128);
  if (overlap(vphi, bp, u_occ, bu) || overlap(vphi, bp, phi, bp))
    return fail(FOCK_ERR_ARG, "vphi overlaps an input array");
  void* base = (p->device >= 0 && p->device < kNoAllocMaxDevices) ? g_noalloc_ptr[p->device] : nullptr;
  if (!base) return fail(FOCK_ERR_STATE, "the scratch array of device %d was not set up", p->device);

  // scratch layout (256-byte aligned pieces): source shadow [nsrc][nb][N_r],
  // target shadow [nk][nphi][N_r] unless phi is u_occ, compensation
  // [nk][nphi][N_r], FP32 band sums [nk * nphi][N_r] where the kernel keeps them
  // in global memory
  const PairSet ps = c.fwd();
  const int nitems = ps.ntk * nphi;
  const bool x_is_u = phi == u_occ && nphi == c.nb && !c.ds;
  const size_t blk = (size_t)c.nb * c.nr;  // elements of one source k-point
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t o_u = 0;
  const size_t o_x = o_u + up((size_t)ps.nsk * blk * sizeof(c64));
  const size_t o_c = o_x + (x_is_u ? 0 : up((size_t)nitems * c.nr * sizeof(c64)));
  const size_t o_a = o_c + up((size_t)nitems * c.nr * sizeof(c64));
  const size_t need = o_a + up(fused_acc_scratch_elems(c.geom.n1, nitems) * sizeof(c64));
  if (need > kNoAllocBytes)
    return fail(FOCK_ERR_SIZE, "fock_apply_noalloc: this cell needs %zu bytes of scratch, above the fixed %zu bytes",
                need, kNoAllocBytes);
  char* sp = (char*)base;
  c64* su = (c64*)(sp + o_u);
  c64* sx = x_is_u ? su : (c64*)(sp + o_x);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  // shadows: the source k-points' orbitals (gathered from S when down-sampled), then the targets
  const c128* U = (const c128*)u_occ;
  if (!c.ds) {
    if ((e = launch_to_c64(su, U, (long)ps.nsk * (long)blk, st)) != hipSuccess) return hip_fail(e, "complex64 shadow (u)");
  } else {
    for (int i = 0; i < ps.nsk; ++i)
      if ((e = launch_to_c64(su + (size_t)i * blk, U + (size_t)c.src[i] * blk, (long)blk, st)) != hipSuccess)
        return hip_fail(e, "complex64 shadow (u)");
  }
  if (!x_is_u && (e = launch_to_c64(sx, (const c128*)phi, (long)nitems * c.nr, st)) != hipSuccess)
    return hip_fail(e, "complex64 shadow (phi)");
  FusedArgs a{};
  a.X = sx;
  a.P = su;
  a.M = su;
  a.Kt = (const float*)c.Kt.ptr;
  a.qidx = ps.qidx;
  a.out = (c128*)vphi;
  a.comp = (c64*)(sp + o_c);
  a.accs = (c64*)(sp + o_a);
  a.nk = ps.nsk;
  a.nx = nphi;
  a.nb = c.nb;
  a.item0 = 0;
  a.nitems = nitems;
  a.scale = -1.0 / c.nsrc;
  a.accumulate = 0;
  a.xcd_map = 1;
  a.n = c.geom.n1;
  a.ksplit = 1;
  a.part_out = nullptr;
  if ((e = launch_fused_apply(c.geom.n1, a, st, 0, nullptr)) != hipSuccess) return hip_fail(e, "fused pair kernel");
  return FOCK_OK;
}
