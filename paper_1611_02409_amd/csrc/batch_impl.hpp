// Batched stream-collide over many independent periodic domains.
//
// Work unit: a tile of `block` consecutive cells of one domain.  The tiles of
// all domains form one list per step (domain by domain); consecutive domains
// are grouped so that a group's storage fits a byte budget.
//
// Persistent mode: one launch of co-resident work-groups loops over windows
// of W steps; inside a window it takes one domain group at a time through
// its W steps.  Each (group, step) is split over the work-groups by a
// launch-wide ticket counter over the group's tiles and closed by a
// grid-wide barrier: every wave drains its stores, the work-group's first
// thread writes back the XCD's L2 (release at device scope), arrives on a
// global counter and polls it with relaxed loads; once all work-groups have
// arrived it invalidates its caches (acquire) once.  Both streaming schemes
// (A-A in place, two-copy pull) need exactly this ordering between
// consecutive steps of one domain: a step reads what the neighbouring tiles
// wrote in the step before.  The wait is bounded by
// the shader clock; a timeout sets a status flag, and every work-group that
// sees the flag leaves, so the launch always drains.
#pragma once

#include "runtime.hpp"

namespace esbgk {

struct DomDev {
    uint64_t f_off, g_off;   // byte offsets of the f and g sets in the batch buffer
    uint64_t copy_off;       // two-copy pull layout: bytes from copy 0 to copy 1
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
    uint32_t *arrive;             // grid-barrier arrival counter
    uint32_t *status;             // 0 ok, 1 a barrier wait timed out
    uint32_t *claim;              // tile tickets claimed so far in this launch
};

// A record every lane of the wave reads at the same address, returned in
// scalar registers (the compiler cannot prove that a table load is uniform;
// without this every population access becomes a waterfall loop over a
// per-lane buffer descriptor).
template <class T>
__device__ __forceinline__ T uniform_load(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "record must be a whole number of words");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, p, sizeof(T));
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; i++) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

__device__ __forceinline__ uint32_t uniform_u32(const uint32_t *p) { return __builtin_amdgcn_readfirstlane(*p); }

// Process one tile of one domain at the given parity of the step count.
// A-A (PULL false): in place, even or odd layout.  Two-copy pull: the state
// of an even step count is in copy 0 and the step writes copy 1, and the
// other way round on odd counts.
template <class L, int S, int CP, bool ODD, bool HAS_G, bool PULL>
__device__ __forceinline__ void tile_step(char *base, const DomDev &dd, uint32_t cell) {
    if (cell >= dd.geom.ncell) return;
    Nbr<L, kElemBytes<S, HAS_G>> nb;
    if constexpr (ODD || PULL) nb.init(cell, dd.geom);
    else nb.own = cell * kElemBytes<S, HAS_G>;
    const uint64_t rd = PULL && ODD ? dd.copy_off : 0, wr = PULL && !ODD ? dd.copy_off : 0;
    const Sets R(base + dd.f_off + rd, HAS_G ? base + dd.g_off + rd : nullptr, dd.pb, dd.sb);
    float F[L::Q], E[HAS_G ? L::Q : 1];
    constexpr int LAY = PULL ? LAY_PULL : ODD ? LAY_ODD : LAY_EVEN;
    gather<L, S, LAY, HAS_G, load_aux(CP)>(R, nb, F, E);
    collide<L, HAS_G, TargetReal<S>>(dd.coll, F, E);
    if constexpr (PULL) {
        const Sets W(base + dd.f_off + wr, HAS_G ? base + dd.g_off + wr : nullptr, dd.pb, dd.sb);
        scatter<L, S, LAY, HAS_G, store_aux(CP)>(W, nb, F, E);
    } else {
        scatter<L, S, LAY, HAS_G, store_aux(CP)>(R, nb, F, E);
    }
}

template <class L, int S, int CP, bool PULL>
__device__ __forceinline__ void tile_dispatch(char *base, const DomDev &dd, uint32_t cell, bool odd) {
    if (odd) {
        if (dd.has_g) tile_step<L, S, CP, true, true, PULL>(base, dd, cell);
        else tile_step<L, S, CP, true, false, PULL>(base, dd, cell);
    } else {
        if (dd.has_g) tile_step<L, S, CP, false, true, PULL>(base, dd, cell);
        else tile_step<L, S, CP, false, false, PULL>(base, dd, cell);
    }
}

// One launch per step: block b processes tile b.
template <class L, int S, int CP, bool PULL>
__global__ __launch_bounds__(512) void k_batch_step(char *base, const DomDev *doms, const uint32_t *tile_dom,
                                                    const uint32_t *tile_cell, uint32_t odd) {
    const uint32_t t = blockIdx.x;
    const DomDev dd = uniform_load(doms + uniform_u32(tile_dom + t));
    tile_dispatch<L, S, CP, PULL>(base, dd, uniform_u32(tile_cell + t) + threadIdx.x, odd != 0);
}

// Grid-wide barrier number `round` (0-based) of a launch with `nblocks`
// work-groups.  Returns false if the launch must stop.
__device__ __forceinline__ bool grid_barrier(const BatchDev &b, uint32_t round, uint32_t nblocks, uint32_t *sh_abort) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(b.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = (round + 1) * nblocks;
        const uint64_t t0 = clock64();
        uint32_t polls = 0;
        while (__hip_atomic_load(b.arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if ((++polls & 63u) == 0) {
                if (__hip_atomic_load(b.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    *sh_abort = 1;
                    break;
                }
                if (clock64() - t0 > (1ull << 31)) {   // ~1 s of shader clock
                    __hip_atomic_store(b.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    *sh_abort = 1;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return *sh_abort == 0;
}

template <class L, int S, int CP, bool PULL>
__device__ __forceinline__ void persistent_body(char *base, const BatchDev &b) {
    __shared__ uint32_t sh_abort, sh_t;
    if (threadIdx.x == 0) sh_abort = 0;
    __syncthreads();
    const uint32_t G = gridDim.x;
    uint32_t round = 0;
    // Tiles of a round are handed out by a launch-wide ticket counter, so a
    // work-group that drew cheap tiles (N_f = 0 domains, partial tiles) takes
    // more of them.  Every work-group ends a round with exactly one failing
    // draw, so the round's last ticket is known to all: next = first + tiles + G.
    uint32_t first = 0;
    for (uint32_t w0 = 0; w0 < b.nsteps; w0 += b.window) {
        const uint32_t W = min(b.window, b.nsteps - w0);
        for (uint32_t g = 0; g < b.ngroups; g++) {
            const GroupDev grp = uniform_load(b.groups + g);
            const uint32_t tb = grp.tile_begin, nt = grp.tile_end - grp.tile_begin;
            for (uint32_t s = w0; s < w0 + W; s++) {
                const bool odd = ((b.parity0 + s) & 1u) != 0;
                for (;;) {
                    if (threadIdx.x == 0) sh_t = atomicAdd(b.claim, 1u) - first;
                    __syncthreads();
                    const uint32_t k = sh_t;
                    __syncthreads();
                    if (k >= nt) break;
                    const uint32_t t = tb + k;
                    const DomDev dd = uniform_load(b.doms + uniform_u32(b.tile_dom + t));
                    tile_dispatch<L, S, CP, PULL>(base, dd, uniform_u32(b.tile_cell + t) + threadIdx.x, odd);
                }
                first += nt + G;
                if (!grid_barrier(b, round++, G, &sh_abort)) return;
            }
        }
    }
}

// Register budget: three waves per SIMD where the code fits in 168 VGPRs
// without spilling (BF16); FP32 storage (FP64 target) and FP16 storage keep
// the compiler's choice.
template <class L, int S, int CP, bool PULL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(S == ST_BF16 && L::Q <= 37 ? 3 : 1))) void k_batch_persistent(
    char *base, BatchDev b) {
    persistent_body<L, S, CP, PULL>(base, b);
}

template <class L, int S, int CP, bool PULL>
__global__ __launch_bounds__(512) void k_batch_persistent_f16(char *base, BatchDev b) {
    persistent_body<L, S, CP, PULL>(base, b);
}

// policy: 0 default, 1 non-temporal loads and stores, 2 non-temporal stores;
// pull: two-copy pull layout (else A-A in place)
struct BatchOps {
    void (*step)(char *base, const DomDev *doms, const uint32_t *tile_dom, const uint32_t *tile_cell, uint32_t tiles,
                 int block, bool odd, int policy, bool pull, hipStream_t s);
    void (*persistent)(char *base, const BatchDev &b, uint32_t grid, int block, int policy, bool pull,
                       hipStream_t s);
    int (*occupancy)(int block, int policy, bool pull, int *blocks_per_cu);
};

template <class L, int S>
struct BatchOpsImpl {
    template <int CP, bool PULL>
    static void step_k(char *base, const DomDev *doms, const uint32_t *tile_dom, const uint32_t *tile_cell,
                       uint32_t tiles, int block, bool odd, hipStream_t s) {
        k_batch_step<L, S, CP, PULL><<<tiles, block, 0, s>>>(base, doms, tile_dom, tile_cell, odd ? 1u : 0u);
    }
    static void step(char *base, const DomDev *doms, const uint32_t *tile_dom, const uint32_t *tile_cell,
                     uint32_t tiles, int block, bool odd, int policy, bool pull, hipStream_t s) {
        auto k = pull ? (policy == 1 ? &step_k<2, true> : policy == 2 ? &step_k<3, true> : &step_k<0, true>)
                      : (policy == 1 ? &step_k<2, false> : policy == 2 ? &step_k<3, false> : &step_k<0, false>);
        k(base, doms, tile_dom, tile_cell, tiles, block, odd, s);
    }
    template <int CP, bool PULL>
    static auto kernel() {
        if constexpr (S == ST_F16) return &k_batch_persistent_f16<L, S, CP, PULL>;
        else return &k_batch_persistent<L, S, CP, PULL>;
    }
    static auto pick(int policy, bool pull) {
        return pull ? (policy == 1 ? kernel<2, true>() : policy == 2 ? kernel<3, true>() : kernel<0, true>())
                    : (policy == 1 ? kernel<2, false>() : policy == 2 ? kernel<3, false>() : kernel<0, false>());
    }
    static void persistent(char *base, const BatchDev &b, uint32_t grid, int block, int policy, bool pull,
                           hipStream_t s) {
        pick(policy, pull)<<<grid, block, 0, s>>>(base, b);
    }
    static int occupancy(int block, int policy, bool pull, int *blocks_per_cu) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pick(policy, pull), block, 0) == hipSuccess
                   ? 0
                   : -1;
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
