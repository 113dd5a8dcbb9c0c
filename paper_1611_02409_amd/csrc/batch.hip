// C ABI of batches of independent domains (see include/esbgk.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batch_impl.hpp"

namespace esbgk {
const Ops *get_ops(int D, int Q, int storage);
const BatchOps *batch_ops_d2q37(int storage);
const BatchOps *batch_ops_d2q33(int storage);
const BatchOps *batch_ops_d3q39(int storage);

// Zero the launch's counters (a plain kernel, so the reset can live inside a
// captured graph).
static __global__ void k_batch_reset(uint32_t *ctr) {
    if (threadIdx.x < 3) ctr[threadIdx.x] = 0;
}

static const BatchOps *get_batch_ops(int D, int Q, int storage) {
    if (D == 2 && Q == 37) return batch_ops_d2q37(storage);
    if (D == 2 && Q == 33) return batch_ops_d2q33(storage);
    if (D == 3 && Q == 39) return batch_ops_d3q39(storage);
    return nullptr;
}
}  // namespace esbgk

using namespace esbgk;

struct esbgk_batch {
    int D = 0, Q = 0, storage = 0, n = 0;
    bool pull = false;   // two-copy pull layout (else A-A in place)
    std::vector<DomainSetup> su;
    std::vector<esbgk_domain_desc> desc;
    std::vector<uint64_t> f_off, g_off;
    std::vector<bool> inited;
    const Ops *ops = nullptr;
    const BatchOps *bops = nullptr;
    char *buf = nullptr;
    uint64_t bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t steps = 0;
    // launch shape
    int block = 256, policy = 0;
    uint32_t window = 1;
    double group_bytes = 1e30;   // one group: every step covers all domains
    // device tables
    DomDev *d_doms = nullptr;
    uint32_t *d_tile_dom = nullptr, *d_tile_cell = nullptr;
    GroupDev *d_groups = nullptr;
    uint32_t *d_ctr = nullptr;   // [barrier arrivals, status, tile tickets]
    uint32_t tiles = 0, ngroups = 0;
    int tables_block = -1;
    // captured graphs keyed by (mode, n, parity, block, policy, window)
    std::map<std::tuple<int, int64_t, int, int, int, uint32_t>, hipGraphExec_t> graphs;

    // storage of domain k's state after s steps (pull: copy s % 2)
    uint64_t copy_at(int k, int64_t s) const { return pull && (s & 1) ? su[k].copy_bytes : 0; }
    char *fb(int k) const { return buf + f_off[k] + copy_at(k, steps); }
    char *gb(int k) const { return su[k].npop == 2 ? buf + g_off[k] + copy_at(k, steps) : nullptr; }
    int lay() const { return pull ? LAY_PULL : (steps & 1) ? LAY_ODD : LAY_EVEN; }
};

namespace {

int bcheck(const esbgk_batch_t *b) {
    if (!b) {
        set_error("batch handle is NULL");
        return ESBGK_EINVAL;
    }
    return ESBGK_OK;
}

int bcheck_k(const esbgk_batch_t *b, int k) {
    if (int rc = bcheck(b)) return rc;
    if (k < 0 || k >= b->n) {
        set_error("domain index %d out of range [0, %d)", k, b->n);
        return ESBGK_EINVAL;
    }
    return ESBGK_OK;
}

void drop_graphs(esbgk_batch_t *b) {
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

// Tile and group tables for the current block size.
int build_tables(esbgk_batch_t *b) {
    if (b->tables_block == b->block) return ESBGK_OK;
    drop_graphs(b);
    std::vector<uint32_t> tdom, tcell;
    std::vector<DomDev> doms(b->n);
    std::vector<GroupDev> groups;
    double gbytes = 0;
    uint32_t gstart = 0;
    for (int k = 0; k < b->n; k++) {
        const DomainSetup &s = b->su[k];
        const uint32_t nt = (s.geom.ncell + b->block - 1) / b->block;
        DomDev &dd = doms[k];
        dd.f_off = b->f_off[k];
        dd.g_off = b->g_off[k];
        dd.copy_off = b->pull ? s.copy_bytes : 0;
        dd.pb = (uint32_t)s.plane_bytes;
        dd.sb = (uint32_t)(s.plane_bytes * b->Q);
        dd.ntiles = nt;
        dd.has_g = s.npop == 2;
        dd.geom = s.geom;
        dd.coll = s.coll;
        const double db = (double)s.bytes;
        // close the current group before a domain that would overflow it
        if (!tdom.empty() && (uint32_t)tdom.size() > gstart && gbytes + db > b->group_bytes) {
            groups.push_back({gstart, (uint32_t)tdom.size()});
            gstart = (uint32_t)tdom.size();
            gbytes = 0;
        }
        gbytes += db;
        for (uint32_t t = 0; t < nt; t++) {
            tdom.push_back((uint32_t)k);
            tcell.push_back(t * (uint32_t)b->block);
        }
    }
    groups.push_back({gstart, (uint32_t)tdom.size()});
    b->tiles = (uint32_t)tdom.size();
    b->ngroups = (uint32_t)groups.size();
    if (b->d_tile_dom) (void)hipFree(b->d_tile_dom);
    if (b->d_tile_cell) (void)hipFree(b->d_tile_cell);
    if (b->d_groups) (void)hipFree(b->d_groups);
    b->d_tile_dom = b->d_tile_cell = nullptr;
    b->d_groups = nullptr;
    ESBGK_HIP(hipMalloc(&b->d_tile_dom, sizeof(uint32_t) * b->tiles));
    ESBGK_HIP(hipMalloc(&b->d_tile_cell, sizeof(uint32_t) * b->tiles));
    ESBGK_HIP(hipMalloc(&b->d_groups, sizeof(GroupDev) * b->ngroups));
    ESBGK_HIP(hipMemcpyAsync(b->d_doms, doms.data(), sizeof(DomDev) * b->n, hipMemcpyHostToDevice, b->stream));
    ESBGK_HIP(hipMemcpyAsync(b->d_tile_dom, tdom.data(), sizeof(uint32_t) * b->tiles, hipMemcpyHostToDevice, b->stream));
    ESBGK_HIP(hipMemcpyAsync(b->d_tile_cell, tcell.data(), sizeof(uint32_t) * b->tiles, hipMemcpyHostToDevice,
                             b->stream));
    ESBGK_HIP(hipMemcpyAsync(b->d_groups, groups.data(), sizeof(GroupDev) * b->ngroups, hipMemcpyHostToDevice,
                             b->stream));
    ESBGK_HIP(hipStreamSynchronize(b->stream));
    b->tables_block = b->block;
    return ESBGK_OK;
}

int all_inited(const esbgk_batch_t *b) {
    for (int k = 0; k < b->n; k++)
        if (!b->inited[k]) {
            set_error("domain %d has no state yet: call esbgk_batch_init_fields first", k);
            return ESBGK_ESTATE;
        }
    return ESBGK_OK;
}

// Enqueue the work of n steps in the given mode onto b->stream (no graph).
void enqueue(esbgk_batch_t *b, int64_t n, int mode, uint32_t grid) {
    if (mode == 2) {
        Tile t;
        t.block = b->block;
        t.policy = b->policy;
        for (int64_t s = 0; s < n; s++) {
            const int64_t at = b->steps + s;
            const int lay = b->pull ? LAY_PULL : (at & 1) ? LAY_ODD : LAY_EVEN;
            for (int k = 0; k < b->n; k++) {
                const DomainSetup &su = b->su[k];
                char *rf = b->buf + b->f_off[k] + b->copy_at(k, at);
                char *wf = b->buf + b->f_off[k] + b->copy_at(k, at + 1);
                char *rg = su.npop == 2 ? b->buf + b->g_off[k] + b->copy_at(k, at) : nullptr;
                char *wg = su.npop == 2 ? b->buf + b->g_off[k] + b->copy_at(k, at + 1) : nullptr;
                b->ops->step(rf, rg, wf, wg, (uint32_t)su.plane_bytes, (uint32_t)(su.plane_bytes * b->Q), su.geom,
                             su.coll, lay, su.npop == 2, t, b->stream);
            }
        }
    } else if (mode == 1) {
        for (int64_t s = 0; s < n; s++)
            b->bops->step(b->buf, b->d_doms, b->d_tile_dom, b->d_tile_cell, b->tiles, b->block,
                          ((b->steps + s) & 1) != 0, b->policy, b->pull, b->stream);
    } else {
        k_batch_reset<<<1, 64, 0, b->stream>>>(b->d_ctr);
        BatchDev bd{};
        bd.doms = b->d_doms;
        bd.tile_dom = b->d_tile_dom;
        bd.tile_cell = b->d_tile_cell;
        bd.groups = b->d_groups;
        bd.ngroups = b->ngroups;
        bd.tiles = b->tiles;
        bd.nsteps = (uint32_t)n;
        bd.window = b->window;
        bd.parity0 = (uint32_t)(b->steps & 1);
        bd.arrive = b->d_ctr;
        bd.status = b->d_ctr + 1;
        bd.claim = b->d_ctr + 2;
        b->bops->persistent(b->buf, bd, grid, b->block, b->policy, b->pull, b->stream);
    }
}

int persistent_grid(esbgk_batch_t *b, uint32_t *grid) {
    int per_cu = 0;
    if (b->bops->occupancy(b->block, b->policy, b->pull, &per_cu) || per_cu < 1) {
        set_error("occupancy query failed for block %d", b->block);
        return ESBGK_EDEVICE;
    }
    int dev = 0, ncu = 0;
    ESBGK_HIP(hipGetDevice(&dev));
    ESBGK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    *grid = (uint32_t)(per_cu * ncu);
    return ESBGK_OK;
}

// A persistent launch needs all of its work-groups resident at once (they
// meet at grid-wide barriers), so two of them must never run at the same
// time: another batch's persistent kernel on another stream would hold the
// compute units one of them waits for.  Every mode-0 call therefore orders
// its launch after the previous one issued in this process on the same
// device: its stream waits on an event recorded behind that launch.  The
// events live until the process ends.
struct PersistentOrder {
    std::mutex m;
    std::map<int, hipEvent_t> last;   // device -> event after its last persistent launch
};

PersistentOrder &persistent_order() {
    static PersistentOrder o;
    return o;
}

}  // namespace

extern "C" {

int esbgk_batch_create(int D, int Q, int n, const esbgk_domain_desc *desc, int storage, esbgk_batch_t **out) {
    clear_error();
    if (!out || !desc || n < 1 || n > (1 << 20)) {
        set_error("need out, desc and 1 <= n <= 2^20");
        return ESBGK_EINVAL;
    }
    *out = nullptr;
    const int codec = storage_codec(storage);
    auto *b = new (std::nothrow) esbgk_batch();
    if (!b) {
        set_error("host allocation failed");
        return ESBGK_ENOMEM;
    }
    b->D = D;
    b->Q = Q;
    b->storage = storage;
    b->pull = (storage & ESBGK_PULL) != 0;
    b->n = n;
    b->su.resize(n);
    b->desc.assign(desc, desc + n);
    b->f_off.resize(n);
    b->g_off.resize(n);
    b->inited.assign(n, false);
    uint64_t off = 0;
    for (int k = 0; k < n; k++) {
        const double kappa = desc[k].kappa > 0 ? desc[k].kappa : 0.2;
        int rc = setup_domain(D, Q, desc[k].N_f, desc[k].Pr, desc[k].tau, kappa, desc[k].dims, storage, b->su[k]);
        if (rc) {
            char msg[1100];
            snprintf(msg, sizeof msg, "domain %d: %s", k, esbgk_last_error());
            set_error("%s", msg);
            delete b;
            return rc;
        }
        b->desc[k].kappa = kappa;
        b->f_off[k] = off;
        b->g_off[k] = b->su[k].npop == 2 ? off + b->su[k].g_off : 0;
        off += b->su[k].bytes;
    }
    b->bytes = off;
    b->ops = get_ops(D, Q, codec);
    b->bops = get_batch_ops(D, Q, codec);
    int rc = ESBGK_OK;
    do {
        hipError_t e = hipStreamCreate(&b->stream);
        if (e != hipSuccess) {
            set_error("hipStreamCreate failed: %s", hipGetErrorString(e));
            rc = ESBGK_EDEVICE;
            break;
        }
        b->own_stream = true;
        e = hipMalloc(&b->buf, b->bytes);
        if (e != hipSuccess) {
            set_error("hipMalloc of %llu bytes failed: %s", (unsigned long long)b->bytes, hipGetErrorString(e));
            rc = e == hipErrorOutOfMemory ? ESBGK_ENOMEM : ESBGK_EDEVICE;
            break;
        }
        if (hipMalloc(&b->d_doms, sizeof(DomDev) * n) != hipSuccess ||
            hipMalloc(&b->d_ctr, sizeof(uint32_t) * 3) != hipSuccess ||
            hipMemsetAsync(b->d_ctr, 0, sizeof(uint32_t) * 3, b->stream) != hipSuccess) {
            set_error("device allocation of batch tables failed");
            rc = ESBGK_ENOMEM;
            break;
        }
        rc = build_tables(b);
    } while (0);
    if (rc) {
        (void)hipGetLastError();
        esbgk_batch_destroy(b);
        return rc;
    }
    *out = b;
    return ESBGK_OK;
}

int esbgk_batch_set_stream(esbgk_batch_t *b, void *hip_stream) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (!hip_stream) {
        set_error("a batch needs a non-NULL stream (graphs are captured on it)");
        return ESBGK_EINVAL;
    }
    ESBGK_HIP(hipStreamSynchronize(b->stream));
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    b->own_stream = false;
    b->stream = (hipStream_t)hip_stream;
    return ESBGK_OK;
}

int esbgk_batch_init_fields(esbgk_batch_t *b, int k, const double *rho, const double *u, const double *T) {
    clear_error();
    if (int rc = bcheck_k(b, k)) return rc;
    if (b->steps != 0) {
        set_error("domains can be initialised only before the batch has stepped");
        return ESBGK_ESTATE;
    }
    const DomainSetup &s = b->su[k];
    const uint64_t n = s.geom.ncell;
    std::vector<float> host;
    if (int rc = host_buffer(host, (2 + b->D) * n)) return rc;
    if (int rc = fields_to_dev(rho, u, T, b->D, n, host.data())) return rc;
    void *tmp = nullptr;
    ESBGK_HIP(hipMalloc(&tmp, host.size() * sizeof(float)));
    hipError_t e = hipMemcpyAsync(tmp, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) {
        b->ops->init(b->fb(k), b->gb(k), (uint32_t)s.plane_bytes, (uint32_t)(s.plane_bytes * b->Q), s.geom, s.coll,
                     (const float *)tmp, b->pull ? LAY_PULL : LAY_EVEN, s.npop == 2, b->stream);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    (void)hipFree(tmp);
    if (e != hipSuccess) {
        set_error("batch init failed: %s", hipGetErrorString(e));
        return ESBGK_EDEVICE;
    }
    b->inited[k] = true;
    return ESBGK_OK;
}

int esbgk_batch_set_tile(esbgk_batch_t *b, int block, int policy, int window, double group_bytes) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (block == 0) block = 256;
    if (block < 64 || block > 512 || (block & 63) || policy < 0 || policy > 3 || window < 0 || window > 4096) {
        set_error("block must be a multiple of 64 in [64, 512], policy 0..3, window 0..4096");
        return ESBGK_EINVAL;
    }
    b->block = block;
    b->policy = policy == 2 ? 1 : policy == 3 ? 2 : 0;
    b->window = window == 0 ? 1 : (uint32_t)window;
    if (group_bytes > 0) b->group_bytes = group_bytes;
    b->tables_block = -1;   // group layout may have changed
    return build_tables(b);
}

int esbgk_batch_step(esbgk_batch_t *b, int64_t n, int mode) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (int rc = all_inited(b)) return rc;
    if (n < 0 || mode < 0 || mode > 2) {
        set_error("need n >= 0 and mode 0, 1 or 2");
        return ESBGK_EINVAL;
    }
    if (n == 0) return ESBGK_OK;
    if ((uint64_t)n * b->tiles >= (1ull << 32)) {
        set_error("n * tiles must stay below 2^32 per call (split the call)");
        return ESBGK_EINVAL;
    }
    if (int rc = build_tables(b)) return rc;
    if (mode == 2) {
        enqueue(b, n, 2, 0);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) {
            set_error("launch failed: %s", hipGetErrorString(e));
            return ESBGK_EDEVICE;
        }
        b->steps += n;
        return ESBGK_OK;
    }
    uint32_t grid = 0;
    if (mode == 0)
        if (int rc = persistent_grid(b, &grid)) return rc;
    const auto key = std::make_tuple(mode, n, (int)(b->steps & 1), b->block, b->policy, b->window);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipGraph_t g = nullptr;
        ESBGK_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        enqueue(b, n, mode, grid);
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            (void)hipGetLastError();
            return ESBGK_EDEVICE;
        }
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(e));
            return ESBGK_EDEVICE;
        }
        it = b->graphs.emplace(key, ge).first;
    }
    if (mode == 0) {
        int dev = 0;
        ESBGK_HIP(hipGetDevice(&dev));
        PersistentOrder &po = persistent_order();
        std::lock_guard<std::mutex> lock(po.m);
        hipEvent_t &ev = po.last[dev];
        if (!ev) ESBGK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ESBGK_HIP(hipStreamWaitEvent(b->stream, ev, 0));
        ESBGK_HIP(hipGraphLaunch(it->second, b->stream));
        ESBGK_HIP(hipEventRecord(ev, b->stream));
    } else {
        ESBGK_HIP(hipGraphLaunch(it->second, b->stream));
    }
    b->steps += n;
    return ESBGK_OK;
}

int esbgk_batch_step_timed(esbgk_batch_t *b, int64_t n, int mode, double *ms) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (!ms) {
        set_error("ms is NULL");
        return ESBGK_EINVAL;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        set_error("event creation failed");
        return ESBGK_EDEVICE;
    }
    (void)hipEventRecord(e0, b->stream);
    int rc = esbgk_batch_step(b, n, mode);
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float f = 0;
    (void)hipEventElapsedTime(&f, e0, e1);
    *ms = f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int esbgk_batch_sync(esbgk_batch_t *b) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    ESBGK_HIP(hipStreamSynchronize(b->stream));
    return ESBGK_OK;
}

int esbgk_batch_status(esbgk_batch_t *b, int *status) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (!status) {
        set_error("status is NULL");
        return ESBGK_EINVAL;
    }
    uint32_t s = 0;
    ESBGK_HIP(hipMemcpyAsync(&s, b->d_ctr + 1, sizeof s, hipMemcpyDeviceToHost, b->stream));
    ESBGK_HIP(hipStreamSynchronize(b->stream));
    *status = (int)s;
    return ESBGK_OK;
}

int esbgk_batch_info(const esbgk_batch_t *b, int64_t *cells, double *bytes_per_step) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    int64_t c = 0;
    double by = 0;
    for (int k = 0; k < b->n; k++) {
        c += b->su[k].geom.ncell;
        by += 2.0 * (double)b->su[k].geom.ncell * b->Q * b->su[k].npop * b->su[k].esize;
    }
    if (cells) *cells = c;
    if (bytes_per_step) *bytes_per_step = by;
    return ESBGK_OK;
}

int esbgk_batch_read_moments(esbgk_batch_t *b, int k, double *rho, double *u, double *T, double *P) {
    clear_error();
    if (int rc = bcheck_k(b, k)) return rc;
    if (!b->inited[k]) {
        set_error("domain %d has no state", k);
        return ESBGK_ESTATE;
    }
    const DomainSetup &s = b->su[k];
    const uint64_t n = s.geom.ncell;
    const int D = b->D, np = D * (D + 1) / 2;
    const uint64_t planes = 2 + D + (P ? np : 0);
    float *tmp = nullptr;
    ESBGK_HIP(hipMalloc(&tmp, planes * n * sizeof(float)));
    b->ops->moments(b->fb(k), b->gb(k), (uint32_t)s.plane_bytes, (uint32_t)(s.plane_bytes * b->Q), s.geom, s.coll,
                    b->lay(), s.npop == 2, tmp, P != nullptr, b->stream);
    std::vector<float> host;
    if (int rc = host_buffer(host, planes * n)) return rc;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), tmp, host.size() * sizeof(float), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) {
        set_error("read_moments failed: %s", hipGetErrorString(e));
        return ESBGK_EDEVICE;
    }
    for (uint64_t c = 0; c < n; c++) {
        if (rho) rho[c] = 1.0 + (double)host[c];
        if (T) T[c] = 1.0 + (double)host[(1 + D) * n + c];
    }
    if (u)
        for (uint64_t c = 0; c < (uint64_t)D * n; c++) u[c] = (double)host[n + c];
    if (P) {
        int q = 0;
        for (int a = 0; a < D; a++)
            for (int bb = a; bb < D; bb++, q++)
                for (uint64_t c = 0; c < n; c++) P[q * n + c] = (a == bb ? 1.0 : 0.0) + (double)host[(2 + D + q) * n + c];
    }
    return ESBGK_OK;
}

int esbgk_batch_totals(esbgk_batch_t *b, int k, double *out) {
    clear_error();
    if (int rc = bcheck_k(b, k)) return rc;
    if (!out || !b->inited[k]) {
        set_error("out is NULL or domain %d has no state", k);
        return ESBGK_EINVAL;
    }
    const DomainSetup &s = b->su[k];
    const uint32_t nchunks = std::max<uint32_t>(1, std::min<uint32_t>(256, (s.geom.ncell + 65535) / 65536));
    double *part = nullptr, *tot = nullptr;
    ESBGK_HIP(hipMalloc(&part, sizeof(double) * 2 * b->Q * nchunks));
    hipError_t e = hipMalloc(&tot, sizeof(double) * 8);
    if (e == hipSuccess) {
        b->ops->plane_sums(b->fb(k), b->gb(k), (uint32_t)s.plane_bytes, (uint32_t)(s.plane_bytes * b->Q),
                           s.geom.ncell, b->Q, s.npop == 2, part, nchunks, b->stream);
        launch_totals_final(part, nchunks, s.lc, s.npop, b->lay() == LAY_ODD, s.geom.ncell,
                            0.5 * b->desc[k].N_f, tot, b->stream);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(out, tot, sizeof(double) * (2 + b->D), hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    }
    (void)hipFree(part);
    if (tot) (void)hipFree(tot);
    if (e != hipSuccess) {
        set_error("batch totals failed: %s", hipGetErrorString(e));
        return ESBGK_EDEVICE;
    }
    return ESBGK_OK;
}

int esbgk_batch_read_populations(esbgk_batch_t *b, int k, double *f, double *g) {
    clear_error();
    if (int rc = bcheck_k(b, k)) return rc;
    if (!f || !b->inited[k]) {
        set_error("f is NULL or domain %d has no state", k);
        return ESBGK_EINVAL;
    }
    const DomainSetup &s = b->su[k];
    const uint64_t n = s.geom.ncell;
    const int Q = b->Q, npop = s.npop;
    float *tmp = nullptr;
    ESBGK_HIP(hipMalloc(&tmp, n * Q * npop * sizeof(float)));
    b->ops->cells(b->fb(k), b->gb(k), (uint32_t)s.plane_bytes, (uint32_t)(s.plane_bytes * Q), s.geom, s.coll,
                  b->lay(), npop == 2, nullptr, (uint32_t)n, tmp, b->stream);
    std::vector<float> host;
    if (int rc = host_buffer(host, n * Q * npop)) return rc;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), tmp, host.size() * sizeof(float), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) {
        set_error("read_populations failed: %s", hipGetErrorString(e));
        return ESBGK_EDEVICE;
    }
    const LatticeConsts &lc = s.lc;
    for (int i = 0; i < Q; i++) {
        const double w = lc.wshell[lc.shell_of[i]];
        for (uint64_t c = 0; c < n; c++) {
            f[i * n + c] = w + (double)host[i * n + c];
            if (g && npop == 2) g[i * n + c] = 0.5 * b->desc[k].N_f * w + (double)host[(Q + i) * n + c];
        }
    }
    return ESBGK_OK;
}

int esbgk_batch_autotune(esbgk_batch_t *b, double budget_ms, const char *cache_path) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (int rc = all_inited(b)) return rc;
    int64_t cells = 0;
    for (int k = 0; k < b->n; k++) cells += b->su[k].geom.ncell;
    char key[160];
    snprintf(key, sizeof key, "batch D%dQ%d st%d n%d log2cells%d", b->D, b->Q, b->storage, b->n,
             (int)std::floor(std::log2((double)cells)));
    const int window = (int)b->window;
    const double gbytes = b->group_bytes;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        const std::string k0 = std::string(key) + " ";
        while (std::getline(in, line)) {
            int blk, pol;
            if (line.rfind(k0, 0) == 0 && sscanf(line.c_str() + k0.size(), "block %d policy %d", &blk, &pol) == 2 &&
                esbgk_batch_set_tile(b, blk, pol, window, gbytes) == ESBGK_OK)
                return ESBGK_OK;
        }
        clear_error();
    }
    // time the persistent mode over a few steps per candidate, on a copy of
    // the state that is put back afterwards
    void *save = nullptr;
    if (hipMalloc(&save, b->bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("autotune needs a second copy of the batch storage (%llu bytes)", (unsigned long long)b->bytes);
        return ESBGK_ENOMEM;
    }
    const int64_t steps0 = b->steps;
    int rc = ESBGK_OK;
    if (hipMemcpyAsync(save, b->buf, b->bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess) rc = ESBGK_EDEVICE;
    const int old_block = b->block, old_policy = b->policy == 1 ? 2 : b->policy == 2 ? 3 : 0;
    int best_block = old_block, best_policy = old_policy;
    double best = 1e30;
    const auto t0 = std::chrono::steady_clock::now();
    for (int blk : {256, 512, 128})
        for (int pol : {0, 2, 3}) {
            const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rc || (budget_ms > 0 && el > budget_ms && best < 1e30)) continue;
            if ((rc = esbgk_batch_set_tile(b, blk, pol, window, gbytes))) break;
            double ms = 0;
            if ((rc = esbgk_batch_step(b, 4, 0))) break;                // captures the graph
            if ((rc = esbgk_batch_step_timed(b, 4, 0, &ms))) break;
            int status = 0;
            if ((rc = esbgk_batch_status(b, &status))) break;
            if (status == 0 && ms < best) {
                best = ms;
                best_block = blk;
                best_policy = pol;
            }
        }
    if (hipMemcpyAsync(b->buf, save, b->bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess && !rc) rc = ESBGK_EDEVICE;
    if (hipStreamSynchronize(b->stream) != hipSuccess && !rc) rc = ESBGK_EDEVICE;
    (void)hipFree(save);
    b->steps = steps0;
    if (rc) {
        if (rc == ESBGK_EDEVICE) set_error("device error during batch autotune");
        (void)esbgk_batch_set_tile(b, old_block, old_policy, window, gbytes);
        return rc;
    }
    if (int r2 = esbgk_batch_set_tile(b, best_block, best_policy, window, gbytes)) return r2;
    if (cache_path) {
        FILE *fp = std::fopen(cache_path, "a");
        if (!fp) {
            set_error("cannot append to %s", cache_path);
            return ESBGK_EIO;
        }
        std::fprintf(fp, "%s block %d policy %d\n", key, best_block, best_policy);
        std::fclose(fp);
    }
    return ESBGK_OK;
}

int esbgk_batch_get_tile(const esbgk_batch_t *b, int *block, int *policy) {
    clear_error();
    if (int rc = bcheck(b)) return rc;
    if (block) *block = b->block;
    if (policy) *policy = b->policy == 1 ? 2 : b->policy == 2 ? 3 : 0;
    return ESBGK_OK;
}

void esbgk_batch_destroy(esbgk_batch_t *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->buf) (void)hipFree(b->buf);
    if (b->d_doms) (void)hipFree(b->d_doms);
    if (b->d_tile_dom) (void)hipFree(b->d_tile_dom);
    if (b->d_tile_cell) (void)hipFree(b->d_tile_cell);
    if (b->d_groups) (void)hipFree(b->d_groups);
    if (b->d_ctr) (void)hipFree(b->d_ctr);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
