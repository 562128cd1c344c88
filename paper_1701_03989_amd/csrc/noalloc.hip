// sscg_gram_noalloc: the Gram stage (sscg_gram) for callers that cannot
// allocate device memory during the call (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// sscg_gram keeps its per-group partial sums (one double per upper-triangle
// entry and 1024-row group) in the context's workspace, which grows with
// hipMalloc on demand.  This variant keeps them in the file-scope device
// array `scratch` below instead: SCRATCH_PARTS doubles (8 MiB) that every
// GPU the library runs on holds until the process ends.  Its device address
// is looked up once per device when the first context on that device is
// created (sscg_create) and kept in a per-device table; host code uses only
// that address, never the array's name (which on the host is a stand-in, not
// a device address).  The partials follow the stated order of the Gram
// matrix, so the same kernels give the same bits as sscg_gram; a Gram whose
// d(d+1)/2 entries x ceil(n / 1024) groups exceed the array is refused.
#include <mutex>

#include "ctx.h"

using namespace sscg_host;

namespace {

constexpr int64_t SCRATCH_PARTS = int64_t(1) << 20;  // doubles (8 MiB)
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) double scratch[SCRATCH_PARTS];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each device (NULL: not looked up)

}  // namespace

// Called by sscg_create with `device` current.
int sscg_host::scratch_setup(sscg_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
    return fail(ctx, SSCG_ERR_ARG, "device %d: the static scratch table has %d entries",
                ctx->device, MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[ctx->device]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ctx, SSCG_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[ctx->device] = p;
  }
  ctx->scratch = g_ptr[ctx->device];
  return SSCG_OK;
}

extern "C" int sscg_gram_noalloc(sscg_ctx* ctx, int n, int s, int first, const double* Y,
                                 int64_t ldy, int rcol, double* G) {
  if (!ctx) return SSCG_ERR_ARG;
  ctx->err.clear();
  int rc = set_device(ctx);
  if (rc) return rc;
  if (n < 1 || s < 1 || s > SSCG_S_LIMIT || !Y || !G || ldy < n)
    return fail(ctx, SSCG_ERR_ARG, "bad Gram arguments");
  if (!first && rcol < s + 1) return fail(ctx, SSCG_ERR_ARG, "rcol must be >= s+1");
  if (!ctx->scratch) return fail(ctx, SSCG_ERR_HIP, "static scratch not set up on this context");
  const int d = first ? s + 1 : 2 * s + 1;
  const int64_t pairs = (int64_t)d * (d + 1) / 2;
  const int ng = gram_ngroups(n);
  if (pairs * ng > SCRATCH_PARTS)
    return fail(ctx, SSCG_ERR_ARG,
                "Gram of %d columns x %d rows needs %lld partials; the static scratch holds %lld "
                "(use sscg_gram)", d, n, (long long)(pairs * ng), (long long)SCRATCH_PARTS);
  double* part = static_cast<double*>(ctx->scratch);
  double* Yw = const_cast<double*>(Y);
  BasisCols bc{Y, Y + (int64_t)rcol * ldy, Yw, ldy, rcol};
  const ColPtr cols = colptr_of(bc, s, first ? 1 : 0);
  // every partial slot [0, ng * pairs) is written by the first kernel before
  // the second reads it: nothing needs clearing between calls
  HIPCHK(launch_gram(cols, n, d, part, Gate{nullptr, nullptr}, ctx->stream));
  HIPCHK(launch_gram_finalize(part, ng, d, G, nullptr, ctx->stream));
  return SSCG_OK;
}
