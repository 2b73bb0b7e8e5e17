// static_sweep.hip -- sl_sweep_static: create + sweep + measure + copy_spins of
// one lattice in a single call that allocates nothing, for callers that cannot
// allocate (code under graph capture, tight serving loops, harnesses that
// forbid allocation).
//
// The lattice's working memory (two copies of both colour arrays, the record
// accumulators, the folded-record staging and the threshold table) lives in a
// file-scope device array, `scratch`, of kStaticScratchBytes.  Every GPU the
// library runs on holds its own copy of it until the process ends.  Host code
// never passes the array's name to a kernel (in host code it is only a
// stand-in for the symbol): the device address of each GPU's copy comes from
// hipGetSymbolAddress, once per device, and that pointer is what the kernels
// take.  Calls on one GPU share its copy, so calls that overlap on one GPU
// race; every call clears what must start at zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/spinlat.h"
#include "host_common.h"
#include "runtime_internal.h"
#include "spinlat_internal.h"

using namespace spinlat;
using namespace spinlat::host;
using namespace spinlat::rt;

namespace {

// 32 MiB holds the four colour arrays of 2^24 sites (2D 4096^2, 3D 256^3);
// the rest holds kStaticRing record slots, their folded copies and the table.
constexpr size_t kStaticScratchBytes = (32u << 20) + (1u << 20);
constexpr uint32_t kStaticRing = 256;  // records folded per chunk of sweeps
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

std::mutex g_mutex;
uint8_t* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

struct TableArg {
    unsigned long long v[kMaxLut];
};

__global__ void k_store_table(unsigned long long* dst, TableArg t, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = t.v[threadIdx.x];
}

// Device address of this device's `scratch`, looked up once per device.
sl_status scratch_of(uint8_t** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "sweep_static: current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(SL_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "sweep_static: scratch address");
        g_scratch[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch[dev];
    return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_sweep_static(const sl_params* params, uint64_t n, int8_t* spins_out, sl_record* records_out,
                          void* hip_stream)
{
    sl_status st = validate(params);
    if (st != SL_OK) return st;
    if (!spins_out || !records_out) return fail(SL_E_BUFFER, "spins_out and records_out are required");
    sl_params p = *params;
    p.record_capacity = kStaticRing;
    st = check_sweep_count(0, ~0ull, p.t0, sweep_limit(p.model), n);
    if (st != SL_OK) return st;
    const Layout lay = layout_of(&p);
    if (lay.total > kStaticScratchBytes)
        return fail(SL_E_UNSUPPORTED, "sweep_static holds at most %zu bytes of working memory; this "
                    "lattice of %llu sites needs %zu (use sl_create_lattice)", kStaticScratchBytes,
                    (unsigned long long)lay.nsites, lay.total);
    uint8_t* base = nullptr;
    st = scratch_of(&base);
    if (st != SL_OK) return st;

    // the handle lives on the stack: no host or device allocation
    sl_lattice h{};
    h.params = p;
    h.lay = lay;
    h.base = base;
    h.stream = static_cast<hipStream_t>(hip_stream);
    h.kind = kind_of(&p);
    h.next_t = p.t0;
    h.pending = 0;
    h.first_t = p.t0;
    h.cur = 0;
    h.table_n = build_table(&p, h.table);
    h.launch = is_sub_lattice(p.model) ? sl_launch{} : auto_launch(&h);
    h.stage = nullptr;

    TableArg tab{};
    for (size_t i = 0; i < h.table_n; ++i) tab.v[i] = h.table[i];
    hipLaunchKernelGGL(k_store_table, dim3(1), dim3(kMaxLut), 0, h.stream,
                       reinterpret_cast<unsigned long long*>(base + lay.off_lut), tab, (int)h.table_n);
    hipError_t e = hipGetLastError();
    // the ring keeps the last call's sums: clear it with a kernel (no memset node)
    if (e == hipSuccess) e = launch_fill_u64(slot_ptr(&h, 0), (uint64_t)kStaticRing * kSlotWords, h.stream);
    SweepArgs a = args_of(&h);
    if (e == hipSuccess) {
        if (p.init == SL_INIT_BUFFER) {
            e = launch_from_natural(a, p.init_spins, h.stream);
        } else {
            const uint64_t bern = thr_from_prob(p.c);
            e = launch_init(a, h.kind, p.init == SL_INIT_COLD ? 0 : 1, (uint32_t)bern, (uint32_t)(bern >> 32),
                            h.stream);
        }
    }
    if (e != hipSuccess) return hip_fail(e, "sweep_static: set-up");
    st = enqueue_observe(&h, 0);
    if (st != SL_OK) return st;
    h.pending = 1;

    // sweeps in chunks that fit the ring; each chunk's records are folded
    // straight into the caller's array (which clears the ring for the next)
    int64_t* out = reinterpret_cast<int64_t*>(records_out);
    const int ising = p.model == SL_ISING ? 1 : 0;
    uint64_t done = 0, written = 0;
    for (;;) {
        const uint64_t k = std::min<uint64_t>(n - done, kStaticRing - h.pending);
        if (k) {
            st = enqueue_sweeps(&h, k);
            if (st != SL_OK) return st;
            done += k;
        }
        e = launch_fold(slot_ptr(&h, 0), out + written * kRecordWords, h.pending, h.first_t, ising, h.stream);
        if (e != hipSuccess) return hip_fail(e, "sweep_static: fold");
        written += h.pending;
        h.first_t += h.pending;
        h.pending = 0;
        if (done == n) break;
    }
    e = launch_to_natural(args_of(&h), spins_out, h.stream);
    if (e != hipSuccess) return hip_fail(e, "sweep_static: copy out");
    return SL_OK;
}

}  // extern "C"
