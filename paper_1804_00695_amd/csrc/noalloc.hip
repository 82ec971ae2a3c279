// noalloc.hip -- the numeric phase for callers that cannot allocate memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): spgemm_numeric with its workspace taken from a fixed array in
// device memory instead of a caller's buffer.
//
// The array lives in this file's code object; every GPU the library runs on
// holds its own copy at its own address until the process ends. Host code
// never uses the array's name as an address (on the host it names a stand-in,
// not device memory): the device address comes from hipGetSymbolAddress,
// called once per device with that device current, and only that address is
// handed to kernels and fills. Every call on one GPU shares that GPU's copy,
// so calls that overlap in time on one GPU race; the header words the kernels
// count with are cleared at the start of every call, and every per-row array
// is written before it is read.
#include <cstring>
#include <mutex>

#include "../../include/mlspgemm.h"
#include "common.h"
#include "internal.h"
#include "launch.h"

using namespace mls;

namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kNoAllocBytes];

std::mutex g_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array; resolved on the first
// call on each device, with that device current.
spgemm_status scratch_of_current_device(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return SPGEMM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p || ((uintptr_t)p & 255) != 0) return SPGEMM_ERR_HIP;
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return SPGEMM_OK;
}

}  // namespace

extern "C" spgemm_status spgemm_numeric_noalloc(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                                hipStream_t stream)
{
    // argument and size checks come before any HIP call
    if (!A || !B || !C) return SPGEMM_ERR_INVALID_ARG;
    if (A->nrows < 0 || B->nrows < 0 || B->ncols < 0) return SPGEMM_ERR_INVALID_ARG;
    if (C->nrows != A->nrows || C->ncols != B->ncols) return SPGEMM_ERR_DIM_MISMATCH;
    if (!C->row_ptr || (C->nnz > 0 && (!C->col_idx || !C->values))) return SPGEMM_ERR_INVALID_ARG;
    const Layout need = make_layout(1, A->nrows, B->nrows, 0, B->ncols, false);
    if (need.total_min > kNoAllocBytes) return SPGEMM_ERR_WORKSPACE_TOO_SMALL;
    char *ws = nullptr;
    spgemm_status st = scratch_of_current_device(&ws);
    if (st != SPGEMM_OK) return st;
    BatchHost bh;
    st = prepare_batch(1, A, B, C, true, false, ws, kNoAllocBytes, stream, bh, /*upload=*/false);
    if (st != SPGEMM_OK) return st;
    return run_numeric(bh, ws, stream);
}
