// Allocation-free entry point: piso_solve_velocity (App. A.6: BiCGStab for the velocity
// predictor) whose BiCGStab workspace lives in one fixed device array per GPU instead of
// the context's buffers.
//
// The array `scratch` is a device global of this code object.  In host code its name is
// only a stand-in for the symbol: its device address on each GPU (every GPU holds its
// own copy) comes from hipGetSymbolAddress, taken once per device when the first context
// on that device is created, and only that address is used afterwards.
#include <mutex>

#include "piso_impl.h"

static __device__ __align__(256) unsigned char scratch[PISO_NOALLOC_SCRATCH_BYTES];

namespace piso {
namespace {

constexpr int kNoallocMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_addr[kNoallocMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

int noalloc_bind(piso_ctx* c) {
  if (c->device < 0 || c->device >= kNoallocMaxDevices)
    return fail(c, PISO_E_HIP, "device index beyond the allocation-free entry's table");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_addr[c->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, PISO_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_noalloc_addr[c->device] = ptr;
  }
  c->noalloc_scratch = g_noalloc_addr[c->device];
  return PISO_OK;
}

}  // namespace piso

using namespace piso;

extern "C" int piso_solve_velocity_noalloc(piso_ctx* c, void* stream, const piso_system* sys, void* u_star,
                                           const piso_solve_opts* o, piso_solve_info* info) {
  if (!c) return PISO_E_ARG;
  DevGuard guard(c->device);
  hipStream_t s = (hipStream_t)stream;
  if (!sys || !sys->A || !sys->C || !sys->b || !u_star || !o)
    return fail(c, PISO_E_ARG, "piso_solve_velocity_noalloc: null pointer");
  if (!(o->rtol > 0) || o->max_iter <= 0) return fail(c, PISO_E_ARG, "piso_solve_velocity_noalloc: bad options");
  if (c->prec == PISO_MIXED)
    return fail(c, PISO_E_ARG, "piso_solve_velocity_noalloc: not available for MIXED contexts");
  if (!c->noalloc_scratch) return fail(c, PISO_E_HIP, "piso_solve_velocity_noalloc: scratch address unknown");
  const size_t N = c->N, D = c->dim, e = c->esz;
  const size_t vec = align256(D * N * e), iab = align256(N * e), prow = (size_t)kRedGrid * sizeof(double);
  const size_t need = 10 * vec + 2 * iab + 18 * prow + align256(sizeof(BiState));
  if (need > (size_t)PISO_NOALLOC_SCRATCH_BYTES)
    return fail(c, PISO_E_ARG, "piso_solve_velocity_noalloc: the grid needs " + std::to_string(need) +
                                   " bytes of workspace, more than the fixed " +
                                   std::to_string((long long)PISO_NOALLOC_SCRATCH_BYTES));
  char* base = (char*)c->noalloc_scratch;
  BiWork w;
  void** vecs[10] = {&w.r, &w.rh, &w.p0, &w.p1, &w.v0, &w.v1, &w.s, &w.t, &w.ph, &w.sh};
  size_t off = 0;
  for (void** v : vecs) {
    *v = base + off;
    off += vec;
  }
  w.iA = base + off;
  off += iab;
  w.sinv = base + off;
  off += iab;
  w.part1 = (double*)(base + off);
  w.part2 = w.part1 + 3 * kRedGrid;
  w.part3 = w.part2 + 6 * kRedGrid;
  off += 18 * prow;
  w.st = (BiState*)(base + off);
  piso_solve_info tmp{};
  const int rc = c->esz == 8
                     ? velocity_solve_ws<double>(c, s, false, (const double*)sys->A, (const double*)sys->C,
                                                 (const double*)sys->b, (double*)u_star, o, &tmp, w)
                     : velocity_solve_ws<float>(c, s, false, (const float*)sys->A, (const float*)sys->C,
                                                (const float*)sys->b, (float*)u_star, o, &tmp, w);
  if (info) *info = tmp;
  return rc < 0 ? rc : tmp.status;
}
