// The operator entry point that allocates nothing: mfq_dslash in FP64 with
// its packed input, output and intermediate fields in a fixed device array
// instead of the handle's workspaces, for callers that cannot call hipMalloc
// (code under stream capture, tight serving loops).
//
// The array is a file-scope __device__ variable.  Its host-side name is not a
// device address: each device holds its own copy, whose address is looked up
// once per device with hipGetSymbolAddress and used for every kernel
// argument.
#include <string.h>

#include <mutex>

#include "handle.h"

namespace mfq {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;  // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Look up (once) the current device's copy of the scratch array.
int noalloc_init_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(MFQ_ERR_STATE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return MFQ_OK;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return fail(MFQ_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
  g_scratch_ptr[dev] = p;
  return MFQ_OK;
}

static void* scratch_ptr_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

}  // namespace mfq

using namespace mfq;

extern "C" {

int mfq_dslash_noalloc(mfq_handle* h, int op, const double* in_dev, double* out_dev, int n_rhs, void* stream) {
  if (!h || !in_dev || !out_dev) return fail(MFQ_ERR_ARG, "NULL argument");
  if (n_rhs < 1) return fail(MFQ_ERR_ARG, "n_rhs must be >= 1");
  if (op < MFQ_OP_HOP_EO || op > MFQ_OP_SCHUR_NORMAL) return fail(MFQ_ERR_ARG, "unknown operator");
  const Geom& g = h->g;
  const size_t field_bytes = field_chunks<double>(g, n_rhs) * sizeof(d2);
  const int n_fields = (op == MFQ_OP_DDAGD || op >= MFQ_OP_SCHUR) ? 3 : 2;
  if ((size_t)n_fields * field_bytes > NOALLOC_SCRATCH_BYTES)
    return fail(MFQ_ERR_ARG, "mfq_dslash_noalloc: " + std::to_string(n_fields) + " packed fields of " +
                                 std::to_string(field_bytes) + " bytes exceed the 64 MiB workspace");
  void* base = scratch_ptr_current_device();
  if (!base) {
    // the handle was created on another device: look this one up now
    if (int rc = noalloc_init_current_device()) return rc;
    base = scratch_ptr_current_device();
  }
  hipStream_t st = (hipStream_t)stream;
  auto view = [&](int k) {
    Field<double> f;
    f.data = (d2*)((unsigned char*)base + (size_t)k * field_bytes);
    f.norm = nullptr;
    f.vh = g.vs;
    return f;
  };
  const Field<double> in = view(0), out = view(1), tmp = view(n_fields == 3 ? 2 : 1);
  // the both-parity launches use the FP64 shape the handle has already tuned
  // for this RHS count (no tuning, no file lookup here), else the default
  Shape sh2 = default_shape(n_rhs);
  for (auto& e : h->tuned)
    if (e.n == n_rhs && e.prec == 8) sh2 = e.sh;
  HIPCHK(launch_pack_spinor<double>(g, in_dev, in, n_rhs, 0, nullptr, st));
  if (int rc = apply_op_fp64(h, op, in, tmp, out, n_rhs, sh2, st)) return rc;
  HIPCHK(launch_unpack_spinor(g, out, out_dev, n_rhs, st));
  return MFQ_OK;
}

}  // extern "C"
