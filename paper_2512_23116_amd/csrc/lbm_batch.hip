// lbm_batch.hip — batched stepping of independent FP32/AA lattices.
//
// The device slot table lists, per slot, the lattice arguments, the first
// tile (256 cells) of the slot in the flattened tile space, how many of the
// graph's launches the slot takes part in, and the AA parity of its state
// before the first one.  Every launch walks the whole tile space with a fixed
// grid (grid-stride over tiles), so the launch configuration never depends on
// which lattices are active: one captured graph serves every mix.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "lbm_device.hpp"

namespace lbm {

struct SlotDesc {
    LatticeArgs L;
    uint32_t tile_begin;
    uint32_t nsteps;     // launches k < nsteps step this slot
    uint32_t parity0;    // AA parity before launch k = 0
    uint32_t pad;
};

struct BatchTable {
    uint32_t n_slots;
    uint32_t total_tiles;
    uint32_t pad[2];
    SlotDesc slot[1];    // n_slots entries follow
};

// The table is read through the constant address space (4) in device code: the
// kernel never writes it, and uniform reads from that space become scalar loads
// even after the kernel's own global stores (which would otherwise force vector
// loads of the 38 plane pointers and the slot constants per tile).  The host
// pass only checks the kernel body, which has no address spaces.
#if defined(__HIP_DEVICE_COMPILE__)
#define LBM_CONSTANT_SPACE __attribute__((address_space(4)))
#else
#define LBM_CONSTANT_SPACE
#endif
typedef const LBM_CONSTANT_SPACE BatchTable ConstTable;

__global__ __launch_bounds__(256) void k_batch_step(const BatchTable* tab_generic, int k) {
    ConstTable* tab = (ConstTable*)tab_generic;
    const uint32_t ns = tab->n_slots, total = tab->total_tiles;
    // Consecutive workgroups are dispatched round-robin over the 8 XCDs: give each
    // XCD one contiguous eighth of the tile space (its L2 then holds neighbouring
    // planes), walked by that XCD's workgroups in turn.  The grid is a multiple of 8.
    const uint32_t xcd = blockIdx.x & 7u, per = gridDim.x >> 3;
    const uint32_t t_end = (uint32_t)(((uint64_t)total * (xcd + 1u)) >> 3);
    uint32_t s = 0;   // tiles only increase along the loop, so the slot does too
    for (uint32_t t = (uint32_t)(((uint64_t)total * xcd) >> 3) + (blockIdx.x >> 3); t < t_end;
         t += per) {
        while (s + 1 < ns && tab->slot[s + 1].tile_begin <= t) ++s;
        if ((uint32_t)k >= tab->slot[s].nsteps) continue;
        const uint32_t cell = (t - tab->slot[s].tile_begin) * 256u + threadIdx.x;
        LatticeArgs L;
        __builtin_memcpy(&L, (const LBM_CONSTANT_SPACE char*)&tab->slot[s].L, sizeof L);
        if (cell >= L.ncell) continue;
        if (((tab->slot[s].parity0 + (uint32_t)k) & 1u) == 0u)
            step_cell<CdF32, PAT_AA_EVEN>(L, cell);
        else
            step_cell<CdF32, PAT_AA_ODD>(L, cell);
    }
}

}  // namespace lbm

using namespace lbm;

struct lbm_batch {
    int max_slots = 0;
    int G = 0;
    int grid = 0;
    hipStream_t stream = nullptr;
    BatchTable* d_table = nullptr;
    BatchTable* h_table = nullptr;     // pinned; reused once `copied` has completed
    hipEvent_t copied = nullptr;
    size_t table_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;
};

namespace {

lbm_status bfail(lbm_batch* b, lbm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    return st;
}

lbm_status bhip(lbm_batch* b, hipError_t e, const char* what) {
    return bfail(b, e == hipErrorOutOfMemory ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE, "%s: %s",
                 what, hipGetErrorString(e));
}

#define BCHK(b, call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return bhip(b, e_, #call); \
    } while (0)

lbm_status launch_batch(lbm_batch* b, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_step, dim3(b->grid), dim3(256), 0, s, (const BatchTable*)b->d_table, k);
    BCHK(b, hipGetLastError());
    return LBM_OK;
}

lbm_status capture(lbm_batch* b) {
    if (!b->cap_stream) BCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    BCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < b->G; ++k) {
        hipLaunchKernelGGL(k_batch_step, dim3(b->grid), dim3(256), 0, b->cap_stream,
                           (const BatchTable*)b->d_table, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(b->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return bhip(b, e, "batch launch during capture");
        }
    }
    BCHK(b, hipStreamEndCapture(b->cap_stream, &b->graph));
    const hipError_t e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {   // no half-made graph is kept: the next call captures anew
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        b->gexec = nullptr;
        return bhip(b, e, "hipGraphInstantiate");
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(int32_t max_slots, int32_t steps_per_graph, void* hip_stream,
                            lbm_batch** out) {
    if (!out) return LBM_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 1024) return LBM_ERR_INVALID_ARG;
    if (steps_per_graph != 0 &&
        (steps_per_graph < 2 || steps_per_graph > 1024 || (steps_per_graph & 1)))
        return LBM_ERR_INVALID_ARG;
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ERR_OUT_OF_MEMORY;
    b->max_slots = max_slots;
    b->G = steps_per_graph;
    b->stream = (hipStream_t)hip_stream;
    b->table_bytes = sizeof(BatchTable) + (size_t)max_slots * sizeof(SlotDesc);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_table, b->table_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_table, b->table_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
    if (e != hipSuccess) {
        lbm_batch_destroy(b);
        return e == hipErrorOutOfMemory ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE;
    }
    b->grid = std::max(1, cus) * 8;   // a multiple of 8 (the kernel splits it per XCD)
    memset(b->h_table, 0, b->table_bytes);
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, lbm_handle* const* hs, const int32_t* steps, int32_t n) {
    if (!b) return LBM_ERR_INVALID_ARG;
    if (n < 0 || n > b->max_slots) return bfail(b, LBM_ERR_INVALID_ARG, "n must be in 0..%d", b->max_slots);
    if (n > 0 && (!hs || !steps)) return bfail(b, LBM_ERR_INVALID_ARG, "hs or steps is NULL");
    int kmax = 0;
    uint64_t tiles = 0;
    for (int i = 0; i < n; ++i) {
        const lbm_handle* h = hs[i];
        if (!h) return bfail(b, LBM_ERR_INVALID_ARG, "handle %d is NULL", i);
        if (h->cfg.precision != LBM_FP32 || h->cfg.streaming != LBM_STREAM_AA)
            return bfail(b, LBM_ERR_INVALID_ARG, "handle %d is not FP32 with AA streaming", i);
        if (!h->initialized) return bfail(b, LBM_ERR_STATE, "handle %d is not initialised", i);
        if (h->stream != b->stream) return bfail(b, LBM_ERR_INVALID_ARG, "handle %d is on another stream", i);
        if (steps[i] < 0 || (b->G > 0 && steps[i] > b->G))
            return bfail(b, LBM_ERR_INVALID_ARG, "steps[%d] = %d out of range", i, steps[i]);
        for (int j = 0; j < i; ++j)
            if (hs[j] == h) return bfail(b, LBM_ERR_INVALID_ARG, "handle %d appears twice", i);
        kmax = std::max(kmax, (int)steps[i]);
        tiles += (h->args.ncell + 255u) / 256u;
    }
    if (tiles >= (1ull << 32)) return bfail(b, LBM_ERR_INVALID_ARG, "too many cells in one batch");
    if (kmax == 0) return LBM_OK;

    // the pinned table may still feed the previous call's copy
    BCHK(b, hipEventSynchronize(b->copied));
    BatchTable* t = b->h_table;
    t->n_slots = (uint32_t)n;
    uint32_t begin = 0;
    for (int i = 0; i < n; ++i) {
        const lbm_handle* h = hs[i];
        SlotDesc& S = t->slot[i];
        S.L = current_args(h);
        S.tile_begin = begin;
        S.nsteps = (uint32_t)steps[i];
        S.parity0 = (uint32_t)(h->steps & 1);
        S.pad = 0;
        begin += (h->args.ncell + 255u) / 256u;
    }
    t->total_tiles = begin;
    const size_t bytes = sizeof(BatchTable) + (size_t)n * sizeof(SlotDesc);
    BCHK(b, hipMemcpyAsync(b->d_table, t, bytes, hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipEventRecord(b->copied, b->stream));

    // the graph only when every one of its launches has work: a shorter call
    // launches exactly kmax kernels instead of replaying empty ones
    if (b->G > 0 && kmax == b->G) {
        if (!b->gexec) {
            lbm_status st = capture(b);
            if (st != LBM_OK) return st;
        }
        BCHK(b, hipGraphLaunch(b->gexec, b->stream));
    } else {
        for (int k = 0; k < kmax; ++k) {
            lbm_status st = launch_batch(b, k, b->stream);
            if (st != LBM_OK) return st;
        }
    }
    for (int i = 0; i < n; ++i) hs[i]->steps += steps[i];
    return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : ""; }

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->copied) (void)hipEventDestroy(b->copied);
    if (b->d_table) (void)hipFree(b->d_table);
    if (b->h_table) (void)hipHostFree(b->h_table);
    delete b;
}

}  // extern "C"
