// placement.hip -- the numeric phase with operands left in pinned host memory
// and accessed in place by the kernels over the host link (Sec. 3.3, Table
// "gpudp": the A_Pin, B_Pin, C_Pin and HostPin placements, which the paper
// measures to decide what its chunking must move into fast memory).
//
// Nothing is copied: every array pointer is translated to the address the
// device uses for it (device memory as is, page-locked host memory through
// its device mapping) and the unchanged kernels of spgemm_numeric run on
// those addresses. Pageable or managed memory, and memory of another device,
// are refused before anything is queued.
#include <cstring>

#include "../../include/mlspgemm.h"
#include "internal.h"

using namespace mls;

namespace mls {

// Device-visible address of p: device memory of device `dev` is returned
// unchanged; page-locked host memory gives its device mapping and sets
// *on_host. Anything else is an invalid argument.
spgemm_status device_view(const void *p, int dev, const void **out, bool *on_host)
{
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // pageable memory: clear the error the query left
        return SPGEMM_ERR_INVALID_ARG;
    }
    if (a.isManaged) return SPGEMM_ERR_INVALID_ARG;
    if (a.type == hipMemoryTypeDevice) {
        if (a.device != dev) return SPGEMM_ERR_INVALID_ARG;
        *out = p;
        return SPGEMM_OK;
    }
    if (a.type == hipMemoryTypeHost && a.devicePointer) {
        *out = a.devicePointer;
        *on_host = true;
        return SPGEMM_OK;
    }
    return SPGEMM_ERR_INVALID_ARG;
}

}  // namespace mls

namespace {

template <typename T>
spgemm_status translate(T *&p, int dev, bool *on_host)
{
    if (!p) return SPGEMM_OK;
    const void *q = nullptr;
    spgemm_status st = device_view(p, dev, &q, on_host);
    if (st == SPGEMM_OK) p = (T *)q;
    return st;
}

spgemm_status translate_csr(spgemm_csr &M, int dev, bool *on_host)
{
    spgemm_status st = translate(M.row_ptr, dev, on_host);
    if (st == SPGEMM_OK && M.nnz > 0) st = translate(M.col_idx, dev, on_host);
    if (st == SPGEMM_OK && M.nnz > 0) st = translate(M.values, dev, on_host);
    return st;
}

}  // namespace

extern "C" spgemm_status spgemm_numeric_placed(const spgemm_csr *A, const spgemm_csr *B, spgemm_csr *C,
                                               uint32_t *placement_out, void *ws, size_t ws_bytes,
                                               hipStream_t stream)
{
    if (!A || !B || !C) return SPGEMM_ERR_INVALID_ARG;
    if (!A->row_ptr || !B->row_ptr || !C->row_ptr) return SPGEMM_ERR_INVALID_ARG;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    spgemm_csr a = *A, b = *B, c = *C;
    bool host[3] = {false, false, false};
    spgemm_status st = translate_csr(a, dev, &host[0]);
    if (st == SPGEMM_OK) st = translate_csr(b, dev, &host[1]);
    if (st == SPGEMM_OK) st = translate_csr(c, dev, &host[2]);
    if (st != SPGEMM_OK) return st;
    // the workspace takes the kernels' atomics: it must be this device's memory
    if (ws) {
        const void *q = nullptr;
        bool ws_host = false;
        st = device_view(ws, dev, &q, &ws_host);
        if (st != SPGEMM_OK || ws_host) return SPGEMM_ERR_INVALID_ARG;
    }
    if (placement_out) *placement_out = (host[0] ? 1u : 0u) | (host[1] ? 2u : 0u) | (host[2] ? 4u : 0u);
    return spgemm_batch_numeric(1, &a, &b, &c, ws, ws_bytes, stream);
}
