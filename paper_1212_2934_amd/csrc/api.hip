// C ABI of libffbh: argument checking, workspace layout, and launch sequencing.
#include <mutex>
#include <new>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "ffbh_internal.h"

namespace ffbh {

// A named range on the host timeline around each entry point (rocprofv3 --marker-trace shows them beside
// the kernels the call enqueued).
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Traversal launch shapes selectable by tuning_id: waves per workgroup of the traversals, how many
// targets an adjoint wave owns (fewer than 64 gives small systems more walks in flight), whether each
// adjoint walk is split over the root's children (8 parts) or not (1), and whether the adjoint waves run in
// one persistent launch that orders its items by the previous launch's costs (1) or one wave per item in
// that order (2).
static const int kTuneWaves[] = {4, 1, 2, 8, 4, 4, 4, 4, 4, 2, 4, 1, 1, 2, 4};
static const int kTuneTpw[] = {64, 64, 64, 64, 32, 16, 64, 32, 16, 64, 64, 64, 64, 64, 64};
static const int kTuneParts[] = {1, 1, 1, 1, 1, 1, 8, 8, 8, 1, 1, 1, 1, 1, 1};
static const int kTuneSched[] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2, 2, 2};
static const int kNumTunings = (int)(sizeof(kTuneWaves) / sizeof(kTuneWaves[0]));
static_assert(sizeof(kTuneTpw) == sizeof(kTuneWaves) && sizeof(kTuneParts) == sizeof(kTuneWaves) &&
                  sizeof(kTuneSched) == sizeof(kTuneWaves),
              "one entry per tuning in every table");

Layout plan_layout(const bh_params &p)
{
    Layout L{};
    L.n = p.n;
    L.B = p.batch;
    L.ntot = L.n * L.B;
    L.max_nodes = 2 * L.ntot + L.B;
    const int tid = p.tuning_id < 0 || p.tuning_id >= kNumTunings ? 0 : p.tuning_id;
    L.adj_parts = kTuneParts[tid] > 1 ? kTuneParts[tid] : 0;
    L.expansion = p.expansion == 2 ? 2 : 1;
    // radix-sort tiles of 256 x sort_items keys: 16 items per thread once there are 2^20 keys, fewer
    // below so that a pass still spreads over about 256 workgroups
    const int64_t items = (L.ntot + 65535) / 65536;
    L.sort_items = (int)(items < 1 ? 1 : items > kSortItems ? kSortItems : items);
    L.tiles = (L.n + (int64_t)kSortThreads * L.sort_items - 1) / ((int64_t)kSortThreads * L.sort_items);
    L.hist_len = L.B * kRadixBins * L.tiles;
    L.bin_int = L.B * (L.n - 1);
    L.num_waves = L.B * ((L.n + kWave - 1) / kWave);
    // short-range grid: at most 32 entries per particle and level 7
    int lg = 0;
    while (((int64_t)2 << lg) <= 32 * L.n) ++lg;
    L.cell_lcap = lg / 3 < 7 ? lg / 3 : 7;
    L.cell_T = (int64_t)1 << (3 * L.cell_lcap);
    Workspace w{};
    carve(L, nullptr, w);
    return L;
}

// Carve the workspace; with base == nullptr only computes L.bytes (passed back through a const_cast).
void carve(const Layout &Lc, void *base, Workspace &w)
{
    Layout &L = const_cast<Layout &>(Lc);
    size_t off = 0;
    char *b = (char *)base;
    auto take = [&](size_t bytes) -> void * {
        off = align_up(off, 256);
        void *p = b ? (void *)(b + off) : nullptr;
        off += bytes ? bytes : 1;
        return p;
    };
    const size_t nt = (size_t)L.ntot, mn = (size_t)L.max_nodes, bi = (size_t)(L.bin_int > 0 ? L.bin_int : 1);
    w.status = (uint32_t *)take(64);
    w.bbox = (double *)take(8 * sizeof(double) * L.B);
    w.bbox_part = (double *)take(6 * sizeof(double) * kBboxBlocks * L.B);
    w.keys[0] = (uint64_t *)take(8 * nt);
    w.keys[1] = (uint64_t *)take(8 * nt);
    w.vals[0] = (uint32_t *)take(4 * nt);
    w.vals[1] = (uint32_t *)take(4 * nt);
    w.hist = (uint32_t *)take(4 * (size_t)L.hist_len);
    w.scan_tmp = (uint32_t *)take(4 * ((size_t)(L.hist_len > L.bin_int ? L.hist_len : L.bin_int) / 4096 + 64));
    w.perm = w.vals[0];
    w.codes = w.keys[0];
    // the target-order sort ping-pongs between (keys[1], vals[1]), free once the particles are sorted, and
    // these; its scan has its own partial sums because it may run beside the octree's scan
    const size_t no = uses_target_order(L) ? nt : 0;
    w.hkeys = (uint64_t *)take(8 * no);
    w.tgt_order = (uint32_t *)take(4 * no);
    w.hscan_tmp = (uint32_t *)take(no ? 4 * ((size_t)L.hist_len / 4096 + 64) : 0);
    w.spos = (double *)take(3 * 8 * nt);
    w.smom = (double *)take(3 * 8 * nt);
    // one 48-byte source record per particle, in the handle's precision (src64 or src32, never both)
    w.src64 = take(48 * nt);
    w.src32 = w.src64;
    w.bin_left = (int32_t *)take(4 * bi);
    w.bin_right = (int32_t *)take(4 * bi);
    w.bin_first = (int32_t *)take(4 * bi);
    w.bin_last = (int32_t *)take(4 * bi);
    w.bin_delta = (int32_t *)take(4 * bi);
    w.bin_parent = (int32_t *)take(4 * bi);
    w.leaf_parent = (int32_t *)take(4 * nt);
    w.bin_nchild = (int32_t *)take(4 * bi);
    w.bin_scan = (uint32_t *)take(4 * bi);
    w.bin_octid = (int32_t *)take(4 * bi);
    w.nodes = (NodeRec *)take(sizeof(NodeRec) * mn);
    w.node_level = (int32_t *)take(4 * mn);
    w.node_m64 = (double *)take(4 * 8 * mn);
    w.ones = (double *)take(8 * (size_t)L.B);
    w.lvl = (uint32_t *)take(4 * 128);
    w.lvl_nodes = (int32_t *)take(4 * mn);
    w.leaf_of = (int32_t *)take(4 * nt);
    w.e_part = (double *)take(8 * (size_t)(L.B * ((L.n + kMinTpw - 1) / kMinTpw)));  // waves of kMinTpw targets
    w.node_adj = (double *)take(8 * 8 * mn);
    w.g_gather = (double *)take(3 * 8 * nt);
    w.g_rm = (double *)take(8 * 8 * nt);
    w.hbar = (double *)take(3 * 8 * nt);
    w.Hs = (double *)take(3 * 8 * nt);
    w.H_scratch = (double *)take(3 * 8 * nt);
    w.md_force = (double *)take(3 * 8 * nt);
    w.md_grad_r = (double *)take(3 * 8 * nt);
    w.md_grad_m = (double *)take(3 * 8 * nt);
    w.cells = (uint2 *)take(8 * (size_t)L.B * (size_t)L.cell_T);
    w.part_buf = (double *)take(6 * 8 * nt * (size_t)L.adj_parts);  // split-walk partial sums (parts > 1)
    const size_t nwmax = (size_t)(L.B * ((L.n + kMinTpw - 1) / kMinTpw));  // wave items of any shape
    w.wave_cost = (uint32_t *)take(4 * nwmax);
    w.wave_order = (uint32_t *)take(4 * nwmax);
    w.sched_ctr = (uint32_t *)take(64);
    w.field_cost = (uint32_t *)take(4 * (size_t)L.num_waves);
    w.field_order = (uint32_t *)take(4 * (size_t)L.num_waves);
    w.field_ctr = (uint32_t *)take(64);
    const size_t qn = L.expansion == 2 ? mn : 0;  // first moments only for order-2 cells
    w.node_q64 = (double *)take(16 * 8 * qn);
    w.node_q32 = (float *)take(16 * 4 * qn);
    w.node_adjq = (double *)take(8 * 8 * qn);  // adjoints of the first moments
    L.bytes = align_up(off, 256);
}

static bool params_ok(const bh_params *p)
{
    if (!p) return false;
    if (p->n < 1 || p->batch < 1) return false;
    if (p->n * (int64_t)p->batch > ((int64_t)1 << 26)) return false;  // node ids below 2^28
    if (p->leaf_size < 1 || p->leaf_size > 64) return false;
    if (!(p->theta >= 0.0) || !__builtin_isfinite(p->theta)) return false;
    if (p->precision != BH_FP64 && p->precision != BH_FP32_MIXED) return false;
    if (p->tuning_id < -1 || p->tuning_id >= kNumTunings) return false;
    if (p->expansion < 0 || p->expansion > 2) return false;
    return true;
}

static bool dptr_ok(const void *p) { return p && ((uintptr_t)p % 8) == 0; }

// Clears the flags only: the count of calls in flight stays (other streams may have calls running).
__global__ void k_clear_status(uint32_t *status)
{
    if (threadIdx.x == 0) status[0] = 0u;
}

// First and last kernel of the entry points whose own kernels do not count the call in and out.
__global__ void k_enter(uint32_t *status)
{
    if (threadIdx.x == 0) call_enter(status);
}
__global__ void k_leave(uint32_t *status)
{
    if (threadIdx.x == 0) call_leave(status);
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *a, int64_t len, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) a[i] = v;
}

__global__ void k_init(uint32_t *status, double *ones, int64_t B)
{
    if (threadIdx.x < 16) status[threadIdx.x] = 0u;
    for (int64_t b = threadIdx.x; b < B; b += blockDim.x) ones[b] = 1.0;
}

__global__ __launch_bounds__(256) void k_export(const NodeRec *__restrict__ nodes,
                                                const int32_t *__restrict__ level, const uint32_t *__restrict__ nn,
                                                int32_t *first, int32_t *count, int32_t *lev, int32_t *nchild,
                                                int32_t *child, double *centroid)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= (int)*nn) return;
    if (first) first[i] = nodes[i].first;
    if (count) count[i] = nodes[i].count;
    if (lev) lev[i] = level[i];
    if (nchild) nchild[i] = nodes[i].nchild;
    if (child) child[i] = nodes[i].child;
    if (centroid) {
        centroid[3 * i] = nodes[i].cx;
        centroid[3 * i + 1] = nodes[i].cy;
        centroid[3 * i + 2] = nodes[i].cz;
    }
}

__global__ __launch_bounds__(256) void k_copy_u32(const uint32_t *__restrict__ a, int64_t len, int32_t *__restrict__ b)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) b[i] = (int32_t)a[i];
}

__global__ void k_copy_bbox(const double *__restrict__ bbox, int64_t B, double *__restrict__ out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    for (int k = 0; k < 5; ++k) out[5 * b + k] = bbox[8 * b + k];
}

__global__ void k_copy_flags(const uint32_t *__restrict__ status, uint32_t *__restrict__ out)
{
    if (threadIdx.x == 0) *out = status[0];
}

// Workspace of bh_field_noalloc: one fixed array per device, reserved when the library's code is loaded
// on that device.  In host code `scratch` names a host-side stand-in, never the device memory: host code
// reaches the array only through the address hipGetSymbolAddress returns for the current device
// (scratch_ptr below), which each device records once.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices];

// Device address of this device's array (looked up on the first call on the device); nullptr on failure.
static void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr ||
            ((uintptr_t)ptr % 256) != 0)
            return nullptr;
        g_scratch_dev[device] = ptr;
    }
    return g_scratch_dev[device];
}

}  // namespace ffbh

using namespace ffbh;

struct bh_handle {
    Handle h;
};

// The MD step's side stream and events (none of them carries timing).
constexpr size_t kHandleAlign = 16;  // alignment bh_init asks of the caller's memory

static hipError_t create_side(Handle &h)
{
    h.side = nullptr;
    h.fork_ev = h.sorted_ev = h.join_ev = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&h.side, hipStreamNonBlocking);
    hipEvent_t *evs[3] = {&h.fork_ev, &h.sorted_ev, &h.join_ev};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(evs[k], hipEventDisableTiming);
    return e;
}

static void destroy_side(Handle &h)
{
    hipEvent_t evs[3] = {h.fork_ev, h.sorted_ev, h.join_ev};
    for (hipEvent_t ev : evs)
        if (ev) (void)hipEventDestroy(ev);
    if (h.side) (void)hipStreamDestroy(h.side);
    h.side = nullptr;
    h.fork_ev = h.sorted_ev = h.join_ev = nullptr;
}

extern "C" {

bh_status bh_workspace_bytes(const bh_params *p, size_t *out_bytes)
{
    if (!params_ok(p) || !out_bytes) return BH_EINVAL;
    *out_bytes = plan_layout(*p).bytes;
    return BH_OK;
}

int32_t bh_num_tunings(void) { return kNumTunings; }

uint64_t bh_morton_code(uint32_t qx, uint32_t qy, uint32_t qz)
{
    return morton(qx & kQMax, qy & kQMax, qz & kQMax);
}

// What bh_create and bh_init share: the handle's fields (no side stream yet) and the launch shape.
static hipError_t setup_handle(Handle &h, const bh_params *p, const Layout &L, void *d_workspace)
{
    h.p = *p;
    h.L = L;
    carve(L, d_workspace, h.w);
    h.side = nullptr;
    h.fork_ev = h.sorted_ev = h.join_ev = nullptr;
    h.built = 0;
    const int tid = p->tuning_id < 0 ? 0 : p->tuning_id;
    h.waves_per_block = kTuneWaves[tid];
    h.adj_tpw = kTuneTpw[tid];
    h.adj_parts = kTuneParts[tid];
    h.adj_sched = kTuneSched[tid];
    h.adj_resident = 0;
    h.field_sched = 0;
    h.cnt_far = h.cnt_near = nullptr;
    for (int k = 0; k < 4; ++k) h.ev[k] = nullptr;
    hipError_t e = hipGetDevice(&h.device);
    if (e == hipSuccess && h.adj_sched) e = adjoint_resident_blocks(h, h.adj_resident);
    return e;
}

// The workspace words that must start at zero (status) or hold constants (ones, first-launch costs).
static hipError_t init_workspace(Handle &h, hipStream_t s)
{
    const Layout &L = h.L;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, h.w.status, h.w.ones, (int64_t)L.B);
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, s, h.w.wave_cost,
                       (int64_t)(L.B * ((L.n + kMinTpw - 1) / kMinTpw)), 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, s, h.w.field_cost, L.num_waves, 0u);
    return hipGetLastError();
}

bh_status bh_create(const bh_params *p, void *d_workspace, size_t workspace_bytes, bh_handle **out)
{
    if (!params_ok(p) || !out) return BH_EINVAL;
    Layout L = plan_layout(*p);
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 || workspace_bytes < L.bytes) return BH_EWORKSPACE;
    bh_handle *hh = new (std::nothrow) bh_handle();
    if (!hh) return BH_EDEVICE;
    Handle &h = hh->h;
    h.owned = 1;
    if (setup_handle(h, p, L, d_workspace) != hipSuccess) {
        delete hh;
        return BH_EDEVICE;
    }
    if (create_side(h) != hipSuccess) {
        destroy_side(h);
        delete hh;
        return BH_EDEVICE;
    }
    if (init_workspace(h, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        destroy_side(h);
        delete hh;
        return BH_EDEVICE;
    }
    *out = hh;
    return BH_OK;
}

bh_status bh_destroy(bh_handle *h)
{
    if (!h || !h->h.owned) return BH_EINVAL;
    // a step still running on the side stream must not lose its stream
    if (h->h.side) (void)hipStreamSynchronize(h->h.side);
    destroy_side(h->h);
    delete h;
    return BH_OK;
}

size_t bh_handle_bytes(void) { return sizeof(bh_handle); }

bh_status bh_init(void *mem, size_t mem_bytes, const bh_params *p, void *d_workspace, size_t workspace_bytes,
                  void *stream, bh_handle **out)
{
    if (!mem || mem_bytes < sizeof(bh_handle) || ((uintptr_t)mem % kHandleAlign) != 0) return BH_EINVAL;
    if (!params_ok(p) || !out) return BH_EINVAL;
    Layout L = plan_layout(*p);
    if (!d_workspace || ((uintptr_t)d_workspace % 256) != 0 || workspace_bytes < L.bytes) return BH_EWORKSPACE;
    static_assert(alignof(bh_handle) <= kHandleAlign, "handle alignment");
    bh_handle *hh = new (mem) bh_handle();
    Handle &h = hh->h;
    h.owned = 0;
    if (setup_handle(h, p, L, d_workspace) != hipSuccess || init_workspace(h, (hipStream_t)stream) != hipSuccess) {
        hh->~bh_handle();
        return BH_EDEVICE;
    }
    *out = hh;
    return BH_OK;
}

bh_status bh_fini(bh_handle *h)
{
    if (!h || h->h.owned) return BH_EINVAL;
    h->~bh_handle();
    return BH_OK;
}

bh_status bh_build(bh_handle *hh, const double *d_pos, void *stream)
{
    const Range range("bh_build");
    if (!hh || !dptr_ok(d_pos)) return BH_EINVAL;
    // large builds put the targets in Hilbert order on the handle's side stream, beside the octree
    Handle &h = hh->h;
    const hipStream_t side = h.L.ntot >= kForkMinParticles && uses_target_order(h.L) ? h.side : nullptr;
    const hipStream_t s = (hipStream_t)stream;
    // the forward walk's wave items are ordered from the costs of the previous walk, and the next bh_field
    // takes them in that order: beside the octree on the side stream, or after the build on the caller's
    // stream for a handle without one (the ordering costs less than the walk's tail it removes from 16384
    // particles up)
    SortedWork order_field;
    if (side) order_field = [&h](hipStream_t q) {
        launch_order_field(h, q);
        return hipGetLastError();
    };
    const bool order_here = !side && h.L.ntot >= kForkMinParticles;
    if (launch_build(h, d_pos, s, nullptr, side, true, true, order_field) != hipSuccess) return BH_EDEVICE;
    if (order_here) launch_order_field(h, s);
    h.field_sched = side || order_here ? 1 : 0;
    hipLaunchKernelGGL(k_leave, dim3(1), dim3(64), 0, s, h.w.status);
    if (hipGetLastError() != hipSuccess) return BH_EDEVICE;
    hh->h.built = 1;
    return BH_OK;
}

bh_status bh_field(bh_handle *hh, const double *d_mom, const double *d_hext, double *d_H, double *d_E,
                   void *stream)
{
    const Range range("bh_field");
    if (!hh || !dptr_ok(d_mom) || !dptr_ok(d_H)) return BH_EINVAL;
    if ((d_hext && !dptr_ok(d_hext)) || (d_E && !dptr_ok(d_E))) return BH_EINVAL;
    if (!hh->h.built) return BH_ESTATE;
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_enter, dim3(1), dim3(64), 0, s, hh->h.w.status);
    if (launch_field(hh->h, d_mom, d_hext, d_H, d_E, s) != hipSuccess) return BH_EDEVICE;
    hipLaunchKernelGGL(k_leave, dim3(1), dim3(64), 0, s, hh->h.w.status);
    return hipGetLastError() == hipSuccess ? BH_OK : BH_EDEVICE;
}

bh_status bh_field_backward(bh_handle *hh, const double *d_mom, const double *d_hext, const double *d_gH,
                            const double *d_gE, double *d_dpos, double *d_dmom, double *d_dhext, void *stream)
{
    const Range range("bh_field_backward");
    if (!hh || !dptr_ok(d_mom) || !dptr_ok(d_dpos) || !dptr_ok(d_dmom)) return BH_EINVAL;
    if ((d_hext && !dptr_ok(d_hext)) || (d_gH && !dptr_ok(d_gH)) || (d_gE && !dptr_ok(d_gE)) ||
        (d_dhext && !dptr_ok(d_dhext)))
        return BH_EINVAL;
    if (!hh->h.built) return BH_ESTATE;
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_enter, dim3(1), dim3(64), 0, s, hh->h.w.status);
    if (launch_backward(hh->h, d_mom, d_hext, d_gH, d_gE, d_dpos, d_dmom, d_dhext, s) != hipSuccess)
        return BH_EDEVICE;
    hipLaunchKernelGGL(k_leave, dim3(1), dim3(64), 0, s, hh->h.w.status);
    return hipGetLastError() == hipSuccess ? BH_OK : BH_EDEVICE;
}

static bh_status md_args_ok(bh_handle *hh, const md_state *s, const md_params *p);

bh_status md_step(bh_handle *hh, const md_state *s, const md_params *p, void *stream)
{
    const Range range("md_step");
    bh_status st = md_args_ok(hh, s, p);
    if (st != BH_OK) return st;
    if (launch_md(hh->h, s, p, (hipStream_t)stream) != hipSuccess) return BH_EDEVICE;
    hh->h.built = 1;
    return BH_OK;
}

static bh_status md_args_ok(bh_handle *hh, const md_state *s, const md_params *p)
{
    if (!hh || !s || !p) return BH_EINVAL;
    if (!dptr_ok(s->pos) || !dptr_ok(s->vel) || !dptr_ok(s->mom) || !dptr_ok(s->omega) || !dptr_ok(s->d_step))
        return BH_EINVAL;
    if (!(p->dt > 0.0) || !(p->mass > 0.0) || !(p->inertia > 0.0) || !(p->kT >= 0.0) || !(p->gamma_t >= 0.0) ||
        !(p->gamma_r >= 0.0) || !(p->wca_sigma >= 0.0) || !(p->wca_eps >= 0.0))
        return BH_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!(p->box_hi[a] > p->box_lo[a])) return BH_EINVAL;
    if (p->d_hext && !dptr_ok(p->d_hext)) return BH_EINVAL;
    if (p->sr_kind != 0 && p->sr_kind != 1) return BH_EINVAL;
    if (!(p->sr_cut >= 0.0) || !__builtin_isfinite(p->sr_cut)) return BH_EINVAL;
    return BH_OK;
}

bh_status bh_graph_capture_md(bh_handle *hh, const md_state *s, const md_params *p, void *stream, void **graph_exec)
{
    const Range range("bh_graph_capture_md");
    bh_status st = md_args_ok(hh, s, p);
    if (st != BH_OK) return st;
    if (!stream || !graph_exec) return BH_EINVAL;
    hipStream_t hs = (hipStream_t)stream;
    if (hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal) != hipSuccess) return BH_EDEVICE;
    hipError_t le = launch_md(hh->h, s, p, hs);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(hs, &g);
    if (le != hipSuccess || ce != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return BH_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return BH_EDEVICE;
    hh->h.built = 1;
    *graph_exec = (void *)ex;
    return BH_OK;
}

bh_status bh_graph_launch(void *graph_exec, void *stream)
{
    const Range range("bh_graph_launch");
    if (!graph_exec) return BH_EINVAL;
    return hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream) == hipSuccess ? BH_OK : BH_EDEVICE;
}

bh_status bh_graph_destroy(void *graph_exec)
{
    if (!graph_exec) return BH_EINVAL;
    return hipGraphExecDestroy((hipGraphExec_t)graph_exec) == hipSuccess ? BH_OK : BH_EDEVICE;
}

bh_status bh_allpairs(int64_t n, int32_t batch, int32_t precision, const double *d_pos, const double *d_mom,
                      const double *d_hext, double *d_H, double *d_dEdr, double *d_E, void *stream)
{
    const Range range("bh_allpairs");
    if (n < 1 || batch < 1 || batch > 65535) return BH_EINVAL;
    if (precision != BH_FP64 && precision != BH_FP32_MIXED) return BH_EINVAL;
    if (!dptr_ok(d_pos) || !dptr_ok(d_mom) || !dptr_ok(d_H)) return BH_EINVAL;
    if ((d_dEdr && !dptr_ok(d_dEdr)) || (d_E && !dptr_ok(d_E)) || (d_hext && !dptr_ok(d_hext))) return BH_EINVAL;
    if (launch_ap(n, batch, precision, d_pos, d_mom, d_hext, d_H, d_dEdr, d_E, (hipStream_t)stream) != hipSuccess)
        return BH_EDEVICE;
    return BH_OK;
}

bh_status bh_field_noalloc(const bh_params *p, const double *d_pos, const double *d_mom, const double *d_hext,
                           double *d_H, double *d_E, uint32_t *d_flags, void *stream)
{
    const Range range("bh_field_noalloc");
    if (!params_ok(p)) return BH_EINVAL;
    const Layout L = plan_layout(*p);
    if (L.bytes > kScratchBytes) return BH_EWORKSPACE;
    if (!dptr_ok(d_pos) || !dptr_ok(d_mom) || !dptr_ok(d_H)) return BH_EINVAL;
    if ((d_hext && !dptr_ok(d_hext)) || (d_E && !dptr_ok(d_E)) || (d_flags && ((uintptr_t)d_flags % 4) != 0))
        return BH_EINVAL;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return BH_EDEVICE;
    void *base = scratch_ptr(device);
    if (!base) return BH_EDEVICE;
    // a handle on the stack over the array: the traversal shape of tuning_id, no counters, no timing
    // events, no side stream (the build and the field use none of them)
    Handle h{};
    h.p = *p;
    h.L = L;
    carve(L, base, h.w);
    h.device = device;
    h.built = 1;
    const int tid = p->tuning_id < 0 ? 0 : p->tuning_id;
    h.waves_per_block = kTuneWaves[tid];
    h.adj_tpw = kTuneTpw[tid];
    h.adj_parts = kTuneParts[tid];
    h.adj_sched = 0;
    hipStream_t s = (hipStream_t)stream;
    // the array keeps the previous call's contents: the status word starts at zero (a kernel, not a
    // memset, so that the call can be captured in a graph)
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, h.w.status, h.w.ones, (int64_t)L.B);
    if (hipGetLastError() != hipSuccess) return BH_EDEVICE;
    if (launch_build(h, d_pos, s) != hipSuccess) return BH_EDEVICE;
    if (launch_field(h, d_mom, d_hext, d_H, d_E, s) != hipSuccess) return BH_EDEVICE;
    if (d_flags) hipLaunchKernelGGL(k_copy_flags, dim3(1), dim3(64), 0, s, h.w.status, d_flags);
    return hipGetLastError() == hipSuccess ? BH_OK : BH_EDEVICE;
}

bh_status bh_check_status(bh_handle *hh, void *stream, uint32_t *flags)
{
    if (!hh) return BH_EINVAL;
    uint32_t v = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&v, hh->h.w.status, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return BH_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return BH_EDEVICE;
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, hh->h.w.status);
    if (hipGetLastError() != hipSuccess) return BH_EDEVICE;
    if (flags) *flags = v;
    return v ? BH_EDEGENERATE : BH_OK;
}

bh_status bh_enable_counters(bh_handle *hh, int32_t *d_n_far, int32_t *d_n_near)
{
    if (!hh) return BH_EINVAL;
    if ((d_n_far == nullptr) != (d_n_near == nullptr)) return BH_EINVAL;
    hh->h.cnt_far = d_n_far;
    hh->h.cnt_near = d_n_near;
    return BH_OK;
}

bh_status bh_set_timing_events(bh_handle *hh, void *fwd_start, void *fwd_stop, void *adj_start, void *adj_stop)
{
    if (!hh) return BH_EINVAL;
    if ((fwd_start == nullptr) != (fwd_stop == nullptr) || (adj_start == nullptr) != (adj_stop == nullptr))
        return BH_EINVAL;
    hh->h.ev[0] = (hipEvent_t)fwd_start;
    hh->h.ev[1] = (hipEvent_t)fwd_stop;
    hh->h.ev[2] = (hipEvent_t)adj_start;
    hh->h.ev[3] = (hipEvent_t)adj_stop;
    return BH_OK;
}

bh_status bh_num_nodes(bh_handle *hh, void *stream, int64_t *out_nodes)
{
    if (!hh || !out_nodes) return BH_EINVAL;
    if (!hh->h.built) return BH_ESTATE;
    uint32_t v = 0;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&v, hh->h.w.status + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return BH_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return BH_EDEVICE;
    *out_nodes = v;
    return BH_OK;
}

bh_status bh_export_tree(bh_handle *hh, int32_t *d_perm, int32_t *d_first, int32_t *d_count, int32_t *d_level,
                         int32_t *d_nchild, int32_t *d_child_first, double *d_centroid, double *d_bbox,
                         void *stream)
{
    if (!hh) return BH_EINVAL;
    if (!hh->h.built) return BH_ESTATE;
    Handle &h = hh->h;
    hipStream_t s = (hipStream_t)stream;
    if (d_perm)
        hipLaunchKernelGGL(k_copy_u32, dim3(grid_for(h.L.ntot, 256)), dim3(256), 0, s, h.w.perm, h.L.ntot, d_perm);
    hipLaunchKernelGGL(k_export, dim3(grid_for(h.L.max_nodes, 256)), dim3(256), 0, s, h.w.nodes, h.w.node_level,
                       h.w.status + 2, d_first, d_count, d_level, d_nchild, d_child_first, d_centroid);
    if (d_bbox)
        hipLaunchKernelGGL(k_copy_bbox, dim3(grid_for(h.L.B, 64)), dim3(64), 0, s, h.w.bbox, h.L.B, d_bbox);
    return hipGetLastError() == hipSuccess ? BH_OK : BH_EDEVICE;
}

const char *bh_status_str(bh_status s)
{
    switch (s) {
    case BH_OK: return "ok";
    case BH_EINVAL: return "invalid argument";
    case BH_EWORKSPACE: return "workspace missing, misaligned or too small";
    case BH_EDEVICE: return "HIP runtime error";
    case BH_EDEGENERATE: return "device flagged degenerate input";
    case BH_ESTATE: return "no tree built";
    default: return "unknown status";
    }
}

}  // extern "C"
