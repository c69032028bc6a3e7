// Allocation-free form of the deflation projection X - W (W^H X) (the complex-FP32
// matrix-core path of dmlmc_apply with DMLMC_OP_DEFL_P), for callers that cannot allocate
// device memory.  Its K-chunk partial products and coefficients live in one file-scope
// device array of fixed size; each device holds its own copy, whose address is looked up
// once per context (dmlmc_create) and then passed to the kernels as an ordinary pointer.
#include "defl.h"
#include "noalloc.h"

namespace {
constexpr size_t kScratchBytes = size_t(16) << 20;  // 16 MiB per device
}

// Device-side storage.  In host code this name is only a handle for hipGetSymbolAddress;
// host code uses the address that call returns, never the name itself.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t noalloc_scratch_bytes() { return kScratchBytes; }

void* noalloc_scratch_address() {
  void* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw DmlmcError(DMLMC_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  return ptr;
}

void deflate_project_noalloc(dmlmc_ctx* ctx, const dmlmc_defl* D, const void* in, void* out, int nrhs) {
  REQUIRE(ctx->noalloc_scratch != nullptr, "context has no scratch address");
  const size_t need = sizeof(c128) * defl_project_scratch_entries(D, nrhs);
  if (need > kScratchBytes)
    throw DmlmcError(DMLMC_EINVAL, "invalid argument: the projection of " + std::to_string(nrhs) + " RHS with k = " +
                                       std::to_string(D->k) + " and n = " + std::to_string(D->n) + " needs " +
                                       std::to_string(need) + " bytes of scratch, more than the " +
                                       std::to_string(kScratchBytes) + " the allocation-free entry point has");
  defl_project_mfma_into(ctx->stream, D, (const c128*)in, (c128*)out, nrhs, (c128*)ctx->noalloc_scratch);
  HIPCHK(hipStreamSynchronize(ctx->stream));
}
