// Kernel entry points of the single-domain path and their launchers for one
// (lattice, storage) combination.  Included by one translation unit per
// lattice.
#pragma once

#include "runtime.hpp"

namespace esbgk {

// ---------------------------------------------------------------- step
// One fused collide-and-stream step of the cells of one domain.  The state is
// read in layout LAY from (fb, gb) and written to (wfb, wgb): the same
// storage for the A-A layouts, the other copy for LAY_PULL.
// One work-group sweeps cpi consecutive chunks of blockDim.x cells.
// ROW: every wave lies inside one x-row (nx % 64 == 0); see RowNbr.
template <class L, int S, int LAY, bool HAS_G, int CP, bool ROW>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(ROW && S != ST_F32 ? (L::Q <= 37 ? 4 : 3) : 1))) void k_step(
    char *fb, char *gb, char *wfb, char *wgb, uint32_t pb, uint32_t sb, Geom g, Coll cp, uint32_t remap,
    uint32_t cpi) {
    const uint32_t blk = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const Sets R(fb, gb, pb, sb);
    const Sets W = LAY == LAY_PULL ? Sets(wfb, wgb, pb, sb) : R;
    const uint32_t first = blk * blockDim.x * cpi + threadIdx.x;
    for (uint32_t k = 0; k < cpi; k++) {
        const uint32_t cell = first + k * blockDim.x;
        if (cell >= g.ncell) return;
        float F[L::Q], E[HAS_G ? L::Q : 1];
        if constexpr (ROW) {
            RowNbr<L, kElemBytes<S, HAS_G>> nb;
            nb.init(cell, g);
            if (nb.inner) gather<L, S, LAY, HAS_G, load_aux(CP)>(R, nb.v, F, E);
            else gather<L, S, LAY, HAS_G, load_aux(CP)>(R, nb.edge(), F, E);
            collide<L, HAS_G, TargetReal<S>>(cp, F, E);
            if constexpr (LAY == LAY_PULL) {
                scatter<L, S, LAY, HAS_G, store_aux(CP)>(W, nb.v, F, E);   // own cell only
            } else {
                if (nb.inner) scatter<L, S, LAY, HAS_G, store_aux(CP)>(W, nb.v, F, E);
                else scatter<L, S, LAY, HAS_G, store_aux(CP)>(W, nb.edge(), F, E);
            }
        } else {
            Nbr<L, kElemBytes<S, HAS_G>> nb;
            if constexpr (LAY != LAY_EVEN) nb.init(cell, g);
            else nb.own = cell * kElemBytes<S, HAS_G>;
            gather<L, S, LAY, HAS_G, load_aux(CP)>(R, nb, F, E);
            collide<L, HAS_G, TargetReal<S>>(cp, F, E);
            scatter<L, S, LAY, HAS_G, store_aux(CP)>(W, nb, F, E);
        }
    }
}

// ---------------------------------------------------------------- init
// fields: [rho - 1 | u_x | u_y (| u_z) | T - 1], ncell floats each.  Writes
// the equilibrium of each cell in layout LAY (LAY_EVEN or LAY_PULL).
template <class L, int S, int LAY, bool HAS_G>
__global__ __launch_bounds__(256) void k_init(char *fb, char *gb, uint32_t pb, uint32_t sb, Geom g, Coll cp,
                                              const float *fields) {
    const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ncell = g.ncell;
    if (cell >= ncell) return;
    constexpr int D = L::D;
    float u[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; a++) u[a] = fields[(1 + a) * (uint64_t)ncell + cell];
    float F[L::Q], E[HAS_G ? L::Q : 1];
    equilibrium<L, HAS_G>(cp, fields[cell], u, fields[(1 + D) * (uint64_t)ncell + cell], F, E);
    const Sets R(fb, gb, pb, sb);
    Nbr<L, kElemBytes<S, HAS_G>> nb;
    nb.init(cell, g);
    st<S>(F[0], R.f, nb.own, 0);
    if constexpr (HAS_G) st<S>(E[0], R.g, nb.own, 0);
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int a = 2 * p + 1, b = 2 * p + 2;
        // direction a of this cell lives at (x - c_a, plane a) in the pull layout
        const uint32_t la = LAY == LAY_PULL ? nb.template at<-cx, -cy, -cz>().v : nb.own;
        const uint32_t lb = LAY == LAY_PULL ? nb.template at<cx, cy, cz>().v : nb.own;
        st<S>(F[a], R.f, la, R.so(a));
        st<S>(F[b], R.f, lb, R.so(b));
        if constexpr (HAS_G) {
            st<S>(E[a], R.g, la, R.so(a));
            st<S>(E[b], R.g, lb, R.so(b));
        }
    });
}

// ---------------------------------------------------------------- moments
// out: [rho - 1 | u (D) | T_eq - 1 | P - delta (D(D+1)/2, if with_P)]
template <class L, int S, int LAY, bool HAS_G>
__global__ __launch_bounds__(256) void k_moments(char *fb, char *gb, uint32_t pb, uint32_t sb, Geom g, Coll cp,
                                                 float *out, int with_P) {
    const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    constexpr int D = L::D;
    Nbr<L, kElemBytes<S, HAS_G>> nb;
    nb.init(cell, g);
    const Sets R(fb, gb, pb, sb);
    float F[L::Q], E[HAS_G ? L::Q : 1];
    gather<L, S, LAY, HAS_G>(R, nb, F, E);
    const CellState<D> cs = cell_moments<L, HAS_G>(cp, F, E);
    const uint64_t n = g.ncell;
    const float r = __builtin_sqrtf(cp.r2);
    out[cell] = cs.drho;
#pragma unroll
    for (int a = 0; a < D; a++) out[(1 + a) * n + cell] = r * cs.J[a] * cs.irho;
    out[(1 + D) * n + cell] = cs.Teq1;
    if (with_P) {
        int q = 0;
#pragma unroll
        for (int a = 0; a < D; a++)
#pragma unroll
            for (int b = a; b < D; b++) {
                // central pressure tensor rho sigma = r^2 M + delta (rho - drho = 1)
                out[(2 + D + q) * n + cell] = cp.r2 * cs.M[sym_idx(a, b)];
                q++;
            }
    }
}

// ---------------------------------------------------------------- read cells
// out[k*Q + i] = f_i - w_i of listed cell k (unscaled, FP32); g after the f
// block at offset n*Q.  list == nullptr: all cells, output as planes
// out[i*ncell + k].
template <class L, int S, int LAY, bool HAS_G>
__global__ __launch_bounds__(256) void k_cells(char *fb, char *gb, uint32_t pb, uint32_t sb, Geom g, Coll cp,
                                               const uint32_t *list, uint32_t n, float *out) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t cell = list ? list[k] : k;
    if (cell >= g.ncell) return;
    Nbr<L, kElemBytes<S, HAS_G>> nb;
    nb.init(cell, g);
    const Sets R(fb, gb, pb, sb);
    float F[L::Q], E[HAS_G ? L::Q : 1];
    gather<L, S, LAY, HAS_G>(R, nb, F, E);
    int sh[L::Q];
    sh[0] = 0;
#pragma unroll
    for (int p = 0; p < L::NP; p++) sh[2 * p + 1] = sh[2 * p + 2] = L::P[p].shell;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        const float is = cp.isc[sh[i]];
        if (list) {
            out[(uint64_t)k * L::Q + i] = F[i] * is;
            if constexpr (HAS_G) out[(uint64_t)n * L::Q + (uint64_t)k * L::Q + i] = E[i] * is;
        } else {
            out[(uint64_t)i * n + k] = F[i] * is;
            if constexpr (HAS_G) out[(uint64_t)(L::Q + i) * n + k] = E[i] * is;
        }
    }
}

// ---------------------------------------------------------------- write populations
// in: scaled deviations as planes in natural order ([f planes | g planes]),
// stored in layout LAY.
template <class L, int S, int LAY, bool HAS_G>
__global__ __launch_bounds__(256) void k_write(char *fb, char *gb, uint32_t pb, uint32_t sb, Geom g,
                                               const float *in) {
    const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    Nbr<L, kElemBytes<S, HAS_G>> nb;
    nb.init(cell, g);
    const uint64_t n = g.ncell;
    const Sets R(fb, gb, pb, sb);
    st<S>(in[cell], R.f, nb.own, 0);
    if constexpr (HAS_G) st<S>(in[L::Q * n + cell], R.g, nb.own, 0);
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int a = 2 * p + 1, b = 2 * p + 2;
        // direction a of this cell lives at (x - c_a) in the odd and pull layouts
        constexpr bool SHIFT = LAY != LAY_EVEN;
        constexpr int pa = LAY == LAY_ODD ? b : a, pb_ = LAY == LAY_ODD ? a : b;
        const uint32_t la = SHIFT ? nb.template at<-cx, -cy, -cz>().v : nb.own;
        const uint32_t lb = SHIFT ? nb.template at<cx, cy, cz>().v : nb.own;
        st<S>(in[a * n + cell], R.f, la, R.so(pa));
        st<S>(in[b * n + cell], R.f, lb, R.so(pb_));
        if constexpr (HAS_G) {
            st<S>(in[(L::Q + a) * n + cell], R.g, la, R.so(pa));
            st<S>(in[(L::Q + b) * n + cell], R.g, lb, R.so(pb_));
        }
    });
}

// ---------------------------------------------------------------- plane sums (FP64)
// partials[plane * nchunks + chunk] = sum over the chunk's cells of the stored
// value of that plane (raw scaled value, in double).
// estride: bytes from one cell's element to the next (paired or not).
template <int S>
__global__ __launch_bounds__(256) void k_plane_sums(char *fb, char *gb, uint32_t pb, uint32_t sb, uint32_t ncell,
                                                    int q, uint32_t estride, double *partials) {
    const uint32_t chunk = blockIdx.x, nchunks = gridDim.x;
    const int plane = blockIdx.y;
    const auto r = set_rsrc(plane < q ? fb : gb, sb);
    const uint32_t so = uint32_t(plane < q ? plane : plane - q) * pb;
    const uint32_t per = (ncell + nchunks - 1) / nchunks;
    const uint32_t lo = chunk * per, hi = min(ncell, lo + per);
    double s = 0;
    for (uint32_t c = lo + threadIdx.x; c < hi; c += blockDim.x) s += (double)ld<S>(r, c * estride, so);
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(uint64_t)plane * nchunks + chunk] = red[0];
}

// ---------------------------------------------------------------- walls
// After each step of a domain with walls, on the state it wrote (two-copy
// pull layout; (fb, gb) is that copy, whose value of direction i at cell p is
// what p streams along c_i in the next step): one thread per ghost column
// (x, z) and wall.  It sums, in FP64, the mass the gas will stream into the
// column's ghost rows (gas cells (x - c_x, y, z - c_z) within |c_y| rows of
// the wall, wall-bound directions) and divides by the wall's emission per
// unit density: rho_w.  The column's ghost cells then hold rho_w G_i(wall)
// (g: rho_w (N_f/2) T_w G_i) in the gas-bound directions, which is what the
// gas cells read in that stream, and the unit-density wall state in the
// others.  Diffuse reflection: what a wall receives it re-emits at its
// velocity and temperature.
template <class L, int S, bool HAS_G>
__global__ __launch_bounds__(256) void k_walls(char *fb, char *gb, uint32_t pb, uint32_t sb, Geom g, Coll cp,
                                               WallSet ws) {
    const uint32_t ncol = g.nx * g.nz;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * ncol) return;
    const int w = idx < ncol ? 0 : 1;
    const uint32_t col = idx - (w ? ncol : 0);
    const int x = int(col % g.nx), z = int(col / g.nx);
    const int nx = int(g.nx), ny = int(g.ny), nz = int(g.nz), R = ws.reach;
    constexpr uint32_t B = kElemBytes<S, HAS_G>;
    const Sets W(fb, gb, pb, sb);
    auto at = [&](int xx, int yy, int zz) {
        xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
        zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
        return uint32_t((zz * ny + yy) * nx + xx) * B;
    };
    // mass received: rest part + sum of stored deviations / scale
    double in = ws.rest[w];
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int sh = L::P[p].shell;
        static_for<2>([&](auto ss) {
            constexpr int sgn = decltype(ss)::value == 0 ? 1 : -1;
            constexpr int cx = sgn * L::P[p].c[0], cy = sgn * L::P[p].c[1], cz = sgn * L::P[p].c[2];
            constexpr int i = decltype(ss)::value == 0 ? 2 * p + 1 : 2 * p + 2;
            if constexpr (cy != 0) {
                if ((w == 0 && cy < 0) || (w == 1 && cy > 0)) {
                    constexpr int ay = cy < 0 ? -cy : cy;
                    for (int k = 0; k < ay; k++) {
                        const int y = w == 0 ? R + k : ny - R - 1 - k;
                        in += double(ld<S>(W.f, at(x - cx, y, z - cz), W.so(i))) * double(cp.isc[sh]);
                    }
                }
            }
        });
    });
    const double rw = in / ws.emit[w];
    const double hN = double(cp.hN);
    for (int k = 0; k < R; k++) {
        const int y = w == 0 ? k : ny - R + k;
        const uint32_t o = at(x, y, z);
        static_for<L::Q>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            constexpr int sh = i == 0 ? 0 : L::P[(i - 1) / 2].shell;
            constexpr int cy = i == 0 ? 0 : ((i & 1) ? L::P[(i - 1) / 2].c[1] : -L::P[(i - 1) / 2].c[1]);
            const bool into_gas = (w == 0 && cy > 0) || (w == 1 && cy < 0);
            const double wi = (double(cp.wh[sh]) + double(cp.wl[sh])) * double(cp.isc[sh]);
            const double sc = 1.0 / double(cp.isc[sh]);
            const double G = (into_gas ? rw : 1.0) * ws.G[w][i];
            st<S>(float((G - wi) * sc), W.f, o, W.so(i));
            if constexpr (HAS_G) st<S>(float((hN * ws.T[w] * G - hN * wi) * sc), W.g, o, W.so(i));
        });
    }
}

// Open (zero-gradient) ends along x, after each step of a domain with open
// ends (two-copy pull layout; (fb, gb) is the copy the step wrote): the
// first and last rx columns are ghost columns, and every ghost cell takes a
// raw copy of all stored values of the nearest gas cell of its row (x = rx
// or nx - rx - 1).  The gas cells next to an end then stream in the
// post-collision populations of the end column, as if the gas continued
// unchanged past it.  One thread per ghost cell.
template <class L, int S, bool HAS_G>
__global__ __launch_bounds__(256) void k_open_x(char *fb, char *gb, uint32_t pb, uint32_t sb, Geom g, uint32_t rx) {
    const uint32_t nrow = g.ny * g.nz;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * rx * nrow) return;
    const uint32_t row = idx / (2 * rx), k = idx % (2 * rx);
    const bool right = k >= rx;
    const uint32_t x = right ? g.nx - 2 * rx + k : k;
    const uint32_t xs = right ? g.nx - rx - 1 : rx;
    constexpr uint32_t B = kElemBytes<S, HAS_G>;
    const uint32_t dst = (row * g.nx + x) * B, src = (row * g.nx + xs) * B;
    auto copy_set = [&](char *base) {
        const auto r = set_rsrc(base, sb);
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            const uint32_t so = uint32_t(i) * pb;
            if constexpr (B == 4)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_raw_buffer_load_b32(r, (int)src, (int)so, 0), r,
                                                      (int)dst, (int)so, 0);
            else
                __builtin_amdgcn_raw_buffer_store_b16(__builtin_amdgcn_raw_buffer_load_b16(r, (int)src, (int)so, 0), r,
                                                      (int)dst, (int)so, 0);
        }
    };
    copy_set(fb);
    if constexpr (HAS_G && !kPaired<S, HAS_G>) copy_set(gb);   // paired elements carry g already
}

// G_i(1, u, (1 + dT) delta) of one cell in FP64 (the target evaluated as in
// the collision, at unit density): the walls' emission per unit density.
template <class L>
__global__ void k_equilibrium_one(Coll cp, double ux, double uy, double uz, double dT, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    constexpr int D = L::D;
    const double A[6] = {dT, 0, 0, dT, 0, D == 3 ? dT : 0.0};
    const double r = __builtin_sqrt(double(cp.r2) + double(cp.r2_lo));
    const double ut[3] = {ux / r, uy / r, D == 3 ? uz / r : 0.0};
    const TargetInv<D, double> T = target_inv<D, double, double>(A, ut, cp.r2, cp.r2_lo);
    auto w_of = [&](int sh) { return (double(cp.wh[sh]) + double(cp.wl[sh])) * double(cp.isc[sh]); };
    out[0] = w_of(0) + target_x<double>(target_rest<D, double>(T), 1.0f, 0.0f, cp.wh[0], cp.wl[0]) * double(cp.isc[0]);
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int sh = L::P[p].shell;
        double Em1, O;
        target_pair<D, cx, cy, cz, double>(T, Em1, O);
        const double X = target_x<double>(Em1, 1.0f, 0.0f, cp.wh[sh], cp.wl[sh]);
        const double Y = target_y<double>(O, 1.0f, cp.wh[sh], cp.wl[sh]);
        out[2 * p + 1] = w_of(sh) + (X + Y) * double(cp.isc[sh]);
        out[2 * p + 2] = w_of(sh) + (X - Y) * double(cp.isc[sh]);
    });
}

// ---------------------------------------------------------------- launchers
inline uint32_t nblocks(uint64_t n, int block) { return (uint32_t)((n + block - 1) / block); }

template <class L, int S>
struct OpsImpl {
    // Calls K<LAY>() with the layout as a template argument.
    template <class K>
    static void by_layout(int lay, K &&k) {
        if (lay == LAY_ODD) k(std::integral_constant<int, LAY_ODD>{});
        else if (lay == LAY_PULL) k(std::integral_constant<int, LAY_PULL>{});
        else k(std::integral_constant<int, LAY_EVEN>{});
    }
    template <int CP>
    static void step_cp(char *fb, char *gb, char *wfb, char *wgb, uint32_t pb, uint32_t sb, const Geom &g,
                        const Coll &c, int lay, bool has_g, int block, int remap, int cpi, hipStream_t s) {
        const uint32_t nb = nblocks(g.ncell, block * cpi);
        const uint32_t k = (uint32_t)cpi;
        // waves start at multiples of 64 cells (block is a multiple of 64)
        const bool row = g.nx % 64 == 0 && lay != LAY_EVEN;
        by_layout(lay, [&](auto ly) {
            constexpr int LY = decltype(ly)::value;
            if (row) {
                if constexpr (LY != LAY_EVEN) {
                    if (has_g) k_step<L, S, LY, true, CP, true><<<nb, block, 0, s>>>(fb, gb, wfb, wgb, pb, sb, g, c, remap, k);
                    else k_step<L, S, LY, false, CP, true><<<nb, block, 0, s>>>(fb, gb, wfb, wgb, pb, sb, g, c, remap, k);
                }
            } else {
                if (has_g) k_step<L, S, LY, true, CP, false><<<nb, block, 0, s>>>(fb, gb, wfb, wgb, pb, sb, g, c, remap, k);
                else k_step<L, S, LY, false, CP, false><<<nb, block, 0, s>>>(fb, gb, wfb, wgb, pb, sb, g, c, remap, k);
            }
        });
    }
    // Tile::policy 0: default caching; 1: non-temporal loads and stores;
    // 2: non-temporal stores only (kernel policy codes 0, 2, 3)
    static void step(char *fb, char *gb, char *wfb, char *wgb, uint32_t pb, uint32_t sb, const Geom &g,
                     const Coll &c, int lay, bool has_g, const Tile &t, hipStream_t s) {
        if (t.policy == 1) step_cp<2>(fb, gb, wfb, wgb, pb, sb, g, c, lay, has_g, t.block, t.remap, t.cpi, s);
        else if (t.policy == 2) step_cp<3>(fb, gb, wfb, wgb, pb, sb, g, c, lay, has_g, t.block, t.remap, t.cpi, s);
        else step_cp<0>(fb, gb, wfb, wgb, pb, sb, g, c, lay, has_g, t.block, t.remap, t.cpi, s);
    }
    static void init(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, const float *fields,
                     int lay, bool has_g, hipStream_t s) {
        const uint32_t nb = nblocks(g.ncell, 256);
        if (lay == LAY_PULL) {
            if (has_g) k_init<L, S, LAY_PULL, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, fields);
            else k_init<L, S, LAY_PULL, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, fields);
        } else {
            if (has_g) k_init<L, S, LAY_EVEN, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, fields);
            else k_init<L, S, LAY_EVEN, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, fields);
        }
    }
    static void moments(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, int lay, bool has_g,
                        float *out, bool with_P, hipStream_t s) {
        const uint32_t nb = nblocks(g.ncell, 256);
        const int wp = with_P ? 1 : 0;
        by_layout(lay, [&](auto ly) {
            constexpr int LY = decltype(ly)::value;
            if (has_g) k_moments<L, S, LY, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, out, wp);
            else k_moments<L, S, LY, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, out, wp);
        });
    }
    static void cells(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, int lay, bool has_g,
                      const uint32_t *list, uint32_t n, float *out, hipStream_t s) {
        const uint32_t nb = nblocks(n, 256);
        by_layout(lay, [&](auto ly) {
            constexpr int LY = decltype(ly)::value;
            if (has_g) k_cells<L, S, LY, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, list, n, out);
            else k_cells<L, S, LY, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, list, n, out);
        });
    }
    static void write(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, int lay, bool has_g, const float *in,
                      hipStream_t s) {
        const uint32_t nb = nblocks(g.ncell, 256);
        by_layout(lay, [&](auto ly) {
            constexpr int LY = decltype(ly)::value;
            if (has_g) k_write<L, S, LY, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, in);
            else k_write<L, S, LY, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, in);
        });
    }
    static void plane_sums(char *fb, char *gb, uint32_t pb, uint32_t sb, uint32_t ncell, int q, bool has_g, double *partials,
                           uint32_t nchunks, hipStream_t s) {
        dim3 grid(nchunks, has_g ? 2 * q : q);
        const uint32_t estride = has_g ? kElemBytes<S, true> : kElemBytes<S, false>;
        k_plane_sums<S><<<grid, 256, 0, s>>>(fb, gb, pb, sb, ncell, q, estride, partials);
    }
    static void walls(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, const WallSet &ws,
                      bool has_g, hipStream_t s) {
        const uint32_t nb = nblocks(2ull * g.nx * g.nz, 256);
        if (has_g) k_walls<L, S, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, ws);
        else k_walls<L, S, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, c, ws);
    }
    static void open_x(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, uint32_t rx, bool has_g,
                       hipStream_t s) {
        const uint32_t nb = nblocks(2ull * rx * g.ny * g.nz, 256);
        if (has_g) k_open_x<L, S, true><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, rx);
        else k_open_x<L, S, false><<<nb, 256, 0, s>>>(fb, gb, pb, sb, g, rx);
    }
    static void equilibrium_one(const Coll &c, const double *u, double dT, double *out, hipStream_t s) {
        k_equilibrium_one<L><<<1, 64, 0, s>>>(c, u[0], u[1], u[2], dT, out);
    }
    static constexpr Ops ops{&step, &init, &moments, &cells, &write, &plane_sums, &walls, &equilibrium_one, &open_x};
};

}  // namespace esbgk

#define ESBGK_INSTANTIATE_LATTICE(LAT, NAME)                                               \
    namespace esbgk {                                                                      \
    const Ops *ops_##NAME(int storage) {                                                   \
        static constexpr Ops o32 = OpsImpl<LAT, ST_F32>::ops;                              \
        static constexpr Ops o16 = OpsImpl<LAT, ST_F16>::ops;                              \
        static constexpr Ops ob16 = OpsImpl<LAT, ST_BF16>::ops;                            \
        return storage == ST_F32 ? &o32 : storage == ST_F16 ? &o16 : &ob16;                \
    }                                                                                      \
    }
