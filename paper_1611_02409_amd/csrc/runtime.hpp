// Host-side runtime shared by the single-domain and batched entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/esbgk.h"
#include "kernels.hpp"
#include "lattice.hpp"

namespace esbgk {

// Thread-local error message and status helpers.
void set_error(const char *fmt, ...);
void clear_error();

#define ESBGK_HIP(call)                                                                                  \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) {                                                                          \
            ::esbgk::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return e_ == hipErrorOutOfMemory ? ESBGK_ENOMEM : ESBGK_EDEVICE;                             \
        }                                                                                                \
    } while (0)

// Sizes a host buffer for a C ABI call; a failed allocation becomes
// ESBGK_ENOMEM with the message set instead of an exception that would
// cross the C boundary.
template <class T>
int host_buffer(std::vector<T> &v, uint64_t n) {
    try {
        v.resize(n);
    } catch (...) {
        set_error("host allocation of %llu bytes failed", (unsigned long long)(n * sizeof(T)));
        return ESBGK_ENOMEM;
    }
    return ESBGK_OK;
}

FastDiv make_fastdiv(uint32_t d);

// Parts of a storage argument: the codec (ESBGK_F32, ESBGK_F16_DEV or
// ESBGK_BF16_DEV) and the plane padding in bytes.
inline int storage_codec(int storage) { return storage & 3; }
inline uint64_t storage_plane_pad(int storage) { return (uint64_t)((storage >> 8) & 0xff) * 4096u; }
inline int storage_unpadded(int storage) { return storage & ~ESBGK_PLANE_PAD(0xff); }

// Validate (D, Q, N_f, Pr, tau, kappa, dims, storage) and fill the derived
// constants.  Returns ESBGK_OK or an error code with the message set.
struct DomainSetup {
    LatticeConsts lc;
    double prm[4];  // omega, omega_s, nu, gamma
    Coll coll;
    Geom geom;
    int npop;
    int codec;       // ESBGK_F32, ESBGK_F16_DEV or ESBGK_BF16_DEV
    int copies;      // 1: A-A in place; 2: two-copy pull
    uint32_t esize;        // bytes per stored value
    bool paired;           // f_i and g_i side by side in one element (FP16/BF16 storage, N_f > 0)
    uint64_t plane_bytes;  // bytes from one direction's plane to the next: the values of all
                           // cells (both populations when paired) plus plane_pad
    uint64_t plane_pad;    // padding after each plane (a multiple of 256; 0 unless chosen)
    uint64_t set_stride;   // bytes of a population set (256-byte aligned)
    uint64_t g_off;        // bytes from f to g: the next set, or 2 within a paired element
    uint64_t copy_bytes;   // bytes of one copy of the state
    uint64_t bytes;        // all population storage
};

int setup_domain(int D, int Q, int Nf, double Pr, double tau, double kappa, const int64_t *dims, int storage,
                 DomainSetup &out);

// Recompute the storage sizes of a set-up domain for another plane padding
// (bytes, a multiple of 256).  ESBGK_EUNSUPPORTED if a set would exceed 4 GiB.
int set_layout(DomainSetup &su, uint64_t plane_pad);

// Enqueue a copy of the population storage from one layout of a domain to
// another (same domain, planes padded differently): `copies` copies of the
// state, every set and plane.  Plane padding is not copied.
int copy_layout(char *dst, const DomainSetup &dl, const char *src, const DomainSetup &sl, int copies,
                hipMemcpyKind kind, hipStream_t s);

// Collision constants for the given parameters.
Coll make_coll(const LatticeConsts &lc, const double prm[4], int D, int Nf, double kappa);

// Host-side field conversion to the FP32 deviations the init kernel reads:
// out = [rho - 1 | u (D planes) | T - 1], each ncell floats.
int fields_to_dev(const double *rho, const double *u, const double *T, int D, uint64_t ncell, float *out);

// Launch shape of one step kernel.
struct Tile {
    int block = 256;   // work-group size
    int remap = 0;     // 1: contiguous cell runs per XCD
    int policy = 0;    // 0 default caching; 1 non-temporal population loads and stores; 2 non-temporal stores only
    int cpi = 1;       // chunks of `block` cells per work-group
};

// Kernel dispatch of one (lattice, storage) combination.  lay is the layout
// of the stored state (LAY_EVEN, LAY_ODD or LAY_PULL); a step reads (fb, gb)
// and writes (wfb, wgb), which are the same storage except for LAY_PULL.
struct Ops {
    void (*step)(char *fb, char *gb, char *wfb, char *wgb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c,
                 int lay, bool has_g, const Tile &t, hipStream_t s);
    void (*init)(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, const float *fields,
                 int lay, bool has_g, hipStream_t s);
    void (*moments)(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, int lay, bool has_g,
                    float *out, bool with_P, hipStream_t s);
    void (*cells)(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, int lay, bool has_g,
                  const uint32_t *list, uint32_t n, float *out, hipStream_t s);
    void (*write)(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, int lay, bool has_g, const float *in,
                  hipStream_t s);
    void (*plane_sums)(char *fb, char *gb, uint32_t pb, uint32_t sb, uint32_t ncell, int nplanes_per_set, bool has_g,
                       double *partials, uint32_t nchunks, hipStream_t s);
    // wall emissions of the current pull-layout copy (see k_walls)
    void (*walls)(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, const Coll &c, const WallSet &ws,
                  bool has_g, hipStream_t s);
    // G_i(1, u, T delta) of one cell (physical u[3], dT = T - 1) into out[Q] (device, FP64)
    void (*equilibrium_one)(const Coll &c, const double *u, double dT, double *out, hipStream_t s);
    // open x ends of the current pull-layout copy (see k_open_x)
    void (*open_x)(char *fb, char *gb, uint32_t pb, uint32_t sb, const Geom &g, uint32_t rx, bool has_g,
                   hipStream_t s);
};

const Ops *get_ops(int D, int Q, int storage);

// Final FP64 reduction of plane sums into totals (one block on the GPU).
void launch_totals_final(const double *partials, uint32_t nchunks, const LatticeConsts &lc, int npop, bool opp_planes,
                         uint64_t ncell, double hN, double *out, hipStream_t s);

}  // namespace esbgk
