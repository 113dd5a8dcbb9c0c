// Batched stream-collide over many independent periodic domains.
//
// Work unit: a tile of `block` consecutive cells of one domain.  The tiles of
// all domains form one list per step (domain by domain).
//
// Persistent mode: one launch of co-resident work-groups that claim tickets
// from a global counter.  Tickets enumerate (step, tile) items in windows of
// W steps: within a window, domain group by domain group (groups are runs of
// consecutive domains whose storage fits a byte budget), and within a group
// step by step.  A work-group may start tile k of domain d at step s only
// when domain d has finished every tile of step s-1 (a per-domain counter of
// finished tiles, released/acquired at device scope).  Every wait is on an
// item with a smaller ticket, so the earliest unfinished ticket can always
// proceed; the waits are also bounded, and a timed-out wait stops the launch
// with a status flag instead of hanging.
#pragma once

#include "runtime.hpp"

namespace esbgk {

struct DomDev {
    uint64_t f_off, g_off;   // byte offsets of the f and g sets in the batch buffer
    uint32_t pb, sb;         // bytes per plane / per set
    uint32_t ntiles;         // tiles per step
    uint32_t has_g;
    Geom geom;
    Coll coll;
};

struct GroupDev {
    uint32_t tile_begin, tile_end;   // tile range of the group within one step
};

struct BatchDev {
    const DomDev *doms;
    const uint32_t *tile_dom;     // tile -> domain
    const uint32_t *tile_cell;    // tile -> first cell in its domain
    const GroupDev *groups;
    uint32_t ngroups;
    uint32_t tiles;               // tiles per step (all domains)
    uint32_t nsteps;              // steps of this launch
    uint32_t window;              // W
    uint32_t parity0;             // parity of the step count at launch
    uint32_t *ticket;             // global ticket counter
    uint32_t *done;               // per-domain finished tiles
    uint32_t *status;             // 0 ok, 1 timed out
};

// Process one tile of one domain at the given parity.
template <class L, int S, int CP, bool ODD, bool HAS_G>
__device__ __forceinline__ void tile_step(char *base, const DomDev &dd, uint32_t cell) {
    if (cell >= dd.geom.ncell) return;
    Nbr<L, S> nb;
    if constexpr (ODD) nb.init(cell, dd.geom);
    else nb.own = cell * StoreBytes<S>::value;
    const Sets R(base + dd.f_off, HAS_G ? base + dd.g_off : nullptr, dd.pb, dd.sb);
    float F[L::Q], E[HAS_G ? L::Q : 1];
    gather<L, S, ODD, HAS_G, CP>(R, nb, F, E);
    collide<L, HAS_G>(dd.coll, F, E);
    scatter<L, S, ODD, HAS_G, CP>(R, nb, F, E);
}

template <class L, int S, int CP>
__device__ __forceinline__ void tile_dispatch(char *base, const DomDev &dd, uint32_t cell, bool odd) {
    if (odd) {
        if (dd.has_g) tile_step<L, S, CP, true, true>(base, dd, cell);
        else tile_step<L, S, CP, true, false>(base, dd, cell);
    } else {
        if (dd.has_g) tile_step<L, S, CP, false, true>(base, dd, cell);
        else tile_step<L, S, CP, false, false>(base, dd, cell);
    }
}

// One launch per step: block b processes tile b.
template <class L, int S, int CP>
__global__ __launch_bounds__(512) void k_batch_step(char *base, const DomDev *doms, const uint32_t *tile_dom,
                                                    const uint32_t *tile_cell, uint32_t odd) {
    const uint32_t t = blockIdx.x;
    const DomDev &dd = doms[tile_dom[t]];
    tile_dispatch<L, S, CP>(base, dd, tile_cell[t] + threadIdx.x, odd != 0);
}

// Map a ticket to (step within the launch, tile).
__device__ __forceinline__ void ticket_item(const BatchDev &b, uint32_t t, uint32_t &step, uint32_t &tile) {
    const uint64_t per_window = (uint64_t)b.window * b.tiles;
    const uint32_t nfull = b.nsteps / b.window;
    uint32_t w0, W;
    uint64_t r;
    if ((uint64_t)t < (uint64_t)nfull * per_window) {
        w0 = (uint32_t)(t / per_window) * b.window;
        r = t % per_window;
        W = b.window;
    } else {
        w0 = nfull * b.window;
        r = (uint64_t)t - (uint64_t)nfull * per_window;
        W = b.nsteps - w0;
    }
    // groups are laid out consecutively, each taking W * (its tiles) tickets
    uint32_t g = 0;
    for (; g + 1 < b.ngroups; g++)
        if (r < (uint64_t)W * b.groups[g + 1].tile_begin) break;
    const uint32_t tb = b.groups[g].tile_begin, tg = b.groups[g].tile_end - tb;
    const uint64_t local = r - (uint64_t)W * tb;
    step = w0 + (uint32_t)(local / tg);
    tile = tb + (uint32_t)(local % tg);
}

template <class L, int S, int CP>
__global__ __launch_bounds__(512) void k_batch_persistent(char *base, BatchDev b) {
    __shared__ uint32_t sh_t, sh_abort;
    const uint32_t total = b.nsteps * b.tiles;
    for (;;) {
        if (threadIdx.x == 0) {
            sh_t = atomicAdd(b.ticket, 1u);
            sh_abort = __hip_atomic_load(b.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const uint32_t t = sh_t;
        const bool abort = sh_abort != 0;
        __syncthreads();
        if (t >= total || abort) break;
        uint32_t s, k;
        ticket_item(b, t, s, k);
        const uint32_t d = b.tile_dom[k];
        const DomDev &dd = b.doms[d];
        if (threadIdx.x == 0 && s > 0) {
            // bounded wait: about 2^20 polls (well under a second); every 256
            // polls also look at the launch-wide abort flag so that one
            // timed-out wait stops every work-group quickly
            const uint32_t need = s * dd.ntiles;
            uint32_t spins = 0;
            while (__hip_atomic_load(b.done + d, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                __builtin_amdgcn_s_sleep(2);
                ++spins;
                if ((spins & 255u) == 0 &&
                    __hip_atomic_load(b.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    sh_abort = 1;
                    break;
                }
                if (spins > (1u << 20)) {
                    __hip_atomic_store(b.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    sh_abort = 1;
                    break;
                }
            }
        }
        __syncthreads();
        if (sh_abort) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every wave sees the finished step
        tile_dispatch<L, S, CP>(base, dd, b.tile_cell[k] + threadIdx.x, ((b.parity0 + s) & 1u) != 0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // every wave's stores are visible device-wide
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(b.done + d, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

struct BatchOps {
    void (*step)(char *base, const DomDev *doms, const uint32_t *tile_dom, const uint32_t *tile_cell, uint32_t tiles,
                 int block, bool odd, int policy, hipStream_t s);
    void (*persistent)(char *base, const BatchDev &b, uint32_t grid, int block, int policy, hipStream_t s);
    int (*occupancy)(int block, int policy, int *blocks_per_cu);
};

template <class L, int S>
struct BatchOpsImpl {
    static void step(char *base, const DomDev *doms, const uint32_t *tile_dom, const uint32_t *tile_cell,
                     uint32_t tiles, int block, bool odd, int policy, hipStream_t s) {
        if (policy) k_batch_step<L, S, 2><<<tiles, block, 0, s>>>(base, doms, tile_dom, tile_cell, odd ? 1u : 0u);
        else k_batch_step<L, S, 0><<<tiles, block, 0, s>>>(base, doms, tile_dom, tile_cell, odd ? 1u : 0u);
    }
    static void persistent(char *base, const BatchDev &b, uint32_t grid, int block, int policy, hipStream_t s) {
        if (policy) k_batch_persistent<L, S, 2><<<grid, block, 0, s>>>(base, b);
        else k_batch_persistent<L, S, 0><<<grid, block, 0, s>>>(base, b);
    }
    static int occupancy(int block, int policy, int *blocks_per_cu) {
        hipError_t e = policy ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                                             k_batch_persistent<L, S, 2>, block, 0)
                              : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                                             k_batch_persistent<L, S, 0>, block, 0);
        return e == hipSuccess ? 0 : -1;
    }
    static constexpr BatchOps ops{&step, &persistent, &occupancy};
};

}  // namespace esbgk

#define ESBGK_INSTANTIATE_BATCH(LAT, NAME)                                                  \
    namespace esbgk {                                                                       \
    const BatchOps *batch_ops_##NAME(int storage) {                                         \
        static constexpr BatchOps o32 = BatchOpsImpl<LAT, ST_F32>::ops;                     \
        static constexpr BatchOps o16 = BatchOpsImpl<LAT, ST_F16>::ops;                     \
        static constexpr BatchOps ob16 = BatchOpsImpl<LAT, ST_BF16>::ops;                   \
        return storage == ST_F32 ? &o32 : storage == ST_F16 ? &o16 : &ob16;                 \
    }                                                                                       \
    }
