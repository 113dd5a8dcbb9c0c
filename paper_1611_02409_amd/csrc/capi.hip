// C ABI of the single-domain ES-BGK lattice (see include/esbgk.h) and the
// runtime pieces shared with the batched path.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

namespace esbgk {

const Ops *ops_d2q37(int storage);
const Ops *ops_d2q33(int storage);
const Ops *ops_d3q39(int storage);

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{d, 0, 0};
    uint32_t s = 0;
    while ((1ull << s) < d) s++;
    f.s = s;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
}

// storage: the codec part of a storage argument (ESBGK_F32, ESBGK_F16_DEV or
// ESBGK_BF16_DEV)
const Ops *get_ops(int D, int Q, int storage) {
    if (storage < 0 || storage > 2) return nullptr;
    if (D == 2 && Q == 37) return ops_d2q37(storage);
    if (D == 2 && Q == 33) return ops_d2q33(storage);
    if (D == 3 && Q == 39) return ops_d3q39(storage);
    return nullptr;
}

Coll make_coll(const LatticeConsts &lc, const double prm[4], int D, int Nf, double kappa) {
    Coll c{};
    c.omega = (float)prm[0];
    c.kappa = (float)kappa;
    c.nu = (float)prm[2];
    const double r2 = lc.r * lc.r;
    c.r2 = (float)r2;
    c.r2_lo = (float)(r2 - (double)c.r2);
    c.hN = (float)(0.5 * Nf);
    const double tnf = Nf > 0 ? 2.0 / Nf : 0.0;
    c.two_over_nf = (float)tnf;
    c.two_over_nf_lo = (float)(tnf - (double)c.two_over_nf);
    c.cD = (float)(double(D) / double(D + Nf));
    c.cN = (float)(double(Nf) / double(D + Nf));
    for (int s = 0; s < MAX_SHELL; s++) {
        if (s < lc.nshell) {
            const double w = std::ldexp(lc.wshell[s], lc.scale_exp[s]);
            c.wh[s] = (float)w;
            c.wl[s] = (float)(w - (double)c.wh[s]);
            c.isc[s] = (float)std::ldexp(1.0, -lc.scale_exp[s]);
        } else {
            c.wh[s] = c.wl[s] = 0.f;
            c.isc[s] = 0.f;
        }
    }
    return c;
}

int setup_domain(int D, int Q, int Nf, double Pr, double tau, double kappa, const int64_t *dims, int storage,
                 DomainSetup &out) {
    if (!dims) {
        set_error("dims is NULL");
        return ESBGK_EINVAL;
    }
    const int codec = storage_codec(storage);
    if (storage < 0 || (storage & ~(3 | ESBGK_PULL | ESBGK_PLANE_PAD(0xff))) || codec > 2) {
        set_error("unknown storage mode %d", storage);
        return ESBGK_EINVAL;
    }
    out.codec = codec;
    out.copies = (storage & ESBGK_PULL) ? 2 : 1;
    if (!lattice_consts(D, Q, out.lc)) {
        set_error("unsupported lattice D%dQ%d (supported: D2Q37, D2Q33, D3Q39)", D, Q);
        return ESBGK_EUNSUPPORTED;
    }
    char msg[256];
    int rc = derive_params(D, Nf, Pr, tau, kappa, out.prm, msg, sizeof msg);
    if (rc) {
        set_error("%s", msg);
        return rc;
    }
    uint64_t ncell = 1;
    int64_t nd[3] = {1, 1, 1};
    for (int d = 0; d < D; d++) {
        if (dims[d] < out.lc.reach || dims[d] > (int64_t)1 << 30) {
            set_error("dims[%d] = %lld must be in [%d, 2^30] (the lattice reach)", d, (long long)dims[d], out.lc.reach);
            return ESBGK_EINVAL;
        }
        nd[d] = dims[d];
        ncell *= (uint64_t)dims[d];
        if (ncell > ((uint64_t)1 << 31)) {
            set_error("too many cells (%llu)", (unsigned long long)ncell);
            return ESBGK_EUNSUPPORTED;
        }
    }
    out.esize = codec == ESBGK_F32 ? 4 : 2;
    out.npop = Nf > 0 ? 2 : 1;
    out.paired = codec != ESBGK_F32 && out.npop == 2;
    out.geom.ncell = (uint32_t)ncell;
    if (int rc2 = set_layout(out, storage_plane_pad(storage))) return rc2;
    out.coll = make_coll(out.lc, out.prm, D, Nf, kappa);
    Geom &g = out.geom;
    g.nx = (uint32_t)nd[0];
    g.ny = (uint32_t)nd[1];
    g.nz = (uint32_t)nd[2];
    g.by_nx = make_fastdiv(g.nx);
    g.by_nxy = make_fastdiv(g.nx * g.ny);
    return ESBGK_OK;
}

int set_layout(DomainSetup &su, uint64_t plane_pad) {
    const uint64_t ncell = su.geom.ncell;
    const int Q = su.lc.Q;
    const uint64_t ebytes = su.esize * (su.paired ? 2 : 1);
    if (plane_pad & 255) {
        set_error("plane padding must be a multiple of 256 bytes");
        return ESBGK_EINVAL;
    }
    const uint64_t plane = ncell * ebytes + plane_pad;
    const uint64_t set_bytes = plane * (uint64_t)Q;
    if (set_bytes >= ((uint64_t)1 << 32)) {
        set_error("one population set would take %llu bytes; the limit is 4 GiB per set (%llu cells for this "
                  "lattice, storage and N_f)",
                  (unsigned long long)set_bytes, (unsigned long long)((((uint64_t)1 << 32) - 1) / (ebytes * Q)));
        return ESBGK_EUNSUPPORTED;
    }
    su.plane_pad = plane_pad;
    su.plane_bytes = plane;
    // planes are 256-byte aligned inside a set only through the cell count;
    // sets and copies start 256-byte aligned
    su.set_stride = (set_bytes + 255) & ~uint64_t(255);
    const int nsets = su.paired ? 1 : su.npop;
    su.g_off = su.npop == 2 ? (su.paired ? su.esize : su.set_stride) : 0;
    su.copy_bytes = su.set_stride * nsets;
    su.bytes = su.copy_bytes * su.copies;
    return ESBGK_OK;
}

int copy_layout(char *dst, const DomainSetup &dl, const char *src, const DomainSetup &sl, int copies,
                hipMemcpyKind kind, hipStream_t s) {
    const uint64_t width = (uint64_t)dl.geom.ncell * dl.esize * (dl.paired ? 2 : 1);
    const int nsets = dl.paired ? 1 : dl.npop;
    for (int c = 0; c < copies; c++)
        for (int k = 0; k < nsets; k++)
            ESBGK_HIP(hipMemcpy2DAsync(dst + c * dl.copy_bytes + k * dl.set_stride, dl.plane_bytes,
                                       src + c * sl.copy_bytes + k * sl.set_stride, sl.plane_bytes, width, dl.lc.Q,
                                       kind, s));
    return ESBGK_OK;
}

int fields_to_dev(const double *rho, const double *u, const double *T, int D, uint64_t ncell, float *out) {
    if (!rho || !u || !T) {
        set_error("rho, u and T must not be NULL");
        return ESBGK_EINVAL;
    }
    for (uint64_t k = 0; k < ncell; k++) {
        if (!std::isfinite(rho[k]) || !std::isfinite(T[k])) {
            set_error("non-finite rho or T at cell %llu", (unsigned long long)k);
            return ESBGK_ENONFINITE;
        }
        if (!(rho[k] > 0) || !(T[k] > 0)) {
            set_error("rho and T must be positive (cell %llu: rho %g, T %g)", (unsigned long long)k, rho[k], T[k]);
            return ESBGK_EINVAL;
        }
        out[k] = (float)(rho[k] - 1.0);
        out[(1 + D) * ncell + k] = (float)(T[k] - 1.0);
    }
    for (uint64_t k = 0; k < (uint64_t)D * ncell; k++) {
        if (!std::isfinite(u[k])) {
            set_error("non-finite u at index %llu", (unsigned long long)k);
            return ESBGK_ENONFINITE;
        }
        out[ncell + k] = (float)u[k];
    }
    return ESBGK_OK;
}

// ---------------------------------------------------------------- FP64 totals
struct TotConsts {
    int Q, D, npop, odd;
    int c[MAX_Q][3];
    double isc[MAX_Q];
    double r;
    double ncell;
    double hN;
};

// One block: sum the per-chunk plane partials in a fixed order, then weight
// each plane by its velocity: mass = sum d, momentum = r sum c d (sign flipped
// in the A-A odd layout, where plane i holds direction opp(i)), energy =
// sum r^2 |c|^2 d / 2 + sum g_d, plus the rest-state contributions.
__global__ __launch_bounds__(256) void k_totals_final(const double *partials, uint32_t nchunks, TotConsts tc,
                                                      double *out) {
    __shared__ double plane[2 * MAX_Q];
    const int nplanes = tc.Q * tc.npop;
    for (int p = threadIdx.x; p < nplanes; p += blockDim.x) {
        double s = 0;
        for (uint32_t k = 0; k < nchunks; k++) s += partials[(uint64_t)p * nchunks + k];
        plane[p] = s * tc.isc[p % tc.Q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mass = 0, mom[3] = {0, 0, 0}, en = 0;
        const double sgn = tc.odd ? -1.0 : 1.0;
        for (int i = 0; i < tc.Q; i++) {
            const double d = plane[i];
            mass += d;
            double c2 = 0;
            for (int a = 0; a < tc.D; a++) {
                mom[a] += sgn * tc.r * tc.c[i][a] * d;
                c2 += double(tc.c[i][a]) * tc.c[i][a];
            }
            en += 0.5 * tc.r * tc.r * c2 * d;
            if (tc.npop == 2) en += plane[tc.Q + i];
        }
        out[0] = tc.ncell + mass;
        for (int a = 0; a < tc.D; a++) out[1 + a] = mom[a];
        // rest state: sum w xi^2 / 2 = D/2 per cell, sum w N_f/2 = N_f/2
        out[1 + tc.D] = tc.ncell * (0.5 * tc.D + tc.hN) + en;
    }
}

void launch_totals_final(const double *partials, uint32_t nchunks, const LatticeConsts &lc, int npop, bool opp_planes,
                         uint64_t ncell, double hN, double *out, hipStream_t s) {
    TotConsts tc{};
    tc.Q = lc.Q;
    tc.D = lc.D;
    tc.npop = npop;
    tc.odd = opp_planes ? 1 : 0;
    for (int i = 0; i < lc.Q; i++) {
        for (int a = 0; a < 3; a++) tc.c[i][a] = lc.c[i][a];
        tc.isc[i] = std::ldexp(1.0, -lc.scale_exp[lc.shell_of[i]]);
    }
    tc.r = lc.r;
    tc.ncell = (double)ncell;
    tc.hN = hN;
    k_totals_final<<<1, 256, 0, s>>>(partials, nchunks, tc, out);
}

}  // namespace esbgk

using namespace esbgk;

// ============================================================== handle
struct esbgk_lattice {
    int D = 0, Q = 0, Nf = 0, storage = 0;
    double Pr = 0, tau = 0, kappa = 0.2;
    int64_t dims[3] = {1, 1, 1};
    DomainSetup su;
    const Ops *ops = nullptr;
    char *buf = nullptr;
    bool owns_buf = false;
    hipStream_t stream = nullptr;
    int64_t steps = 0;
    bool initialized = false;
    Tile tile[2];   // launch shape of the even- and odd-layout step kernels
    double *d_partials = nullptr;
    double *d_totals = nullptr;
    uint32_t nchunks = 0;
    bool walls = false;   // diffusely reflecting walls at low and high y
    WallSet ws{};
    bool open_x = false;  // zero-gradient ends along x
    uint32_t rx = 0;      // ghost columns per end
    // The current state was written by a step (its values are post-collision
    // and the walls take part in its stream), not laid down by init or
    // write_populations (which stream into the given pre-collision state,
    // wall neighbours included).
    bool from_step = false;

    void apply_walls() { ops->walls(fb(), gb(), pb(), sb(), su.geom, su.coll, ws, has_g(), stream); }
    void apply_open_x() { ops->open_x(fb(), gb(), pb(), sb(), su.geom, rx, has_g(), stream); }
    void launch_step() {
        ops->step(fb(), gb(), wfb(), wgb(), pb(), sb(), su.geom, su.coll, lay(), has_g(), tile[odd() ? 1 : 0],
                  stream);
        steps++;
        from_step = true;
        // the new state's ghost rows take the walls' emission, so that every
        // reader of the state (moments, populations, checkpoints, the next
        // step) sees what the gas receives in its next stream
        if (walls) apply_walls();
        if (open_x) apply_open_x();
    }
    // storage of the current state and of the state a step writes (the same
    // storage for A-A; the other copy for two-copy pull)
    char *copy(int64_t s) const { return buf + (su.copies == 2 ? (uint64_t)(s & 1) * su.copy_bytes : 0); }
    char *fb() const { return copy(steps); }
    char *gb() const { return su.npop == 2 ? fb() + su.g_off : nullptr; }
    char *wfb() const { return copy(steps + 1); }
    char *wgb() const { return su.npop == 2 ? wfb() + su.g_off : nullptr; }
    uint32_t pb() const { return (uint32_t)su.plane_bytes; }
    uint32_t sb() const { return (uint32_t)(su.plane_bytes * (uint64_t)Q); }
    bool odd() const { return (steps & 1) != 0; }
    int lay() const { return su.copies == 2 ? LAY_PULL : odd() ? LAY_ODD : LAY_EVEN; }
    bool has_g() const { return su.npop == 2; }
};

namespace {

int alloc_aux(esbgk_t *h) {
    h->nchunks = std::max<uint32_t>(1, std::min<uint32_t>(256, (h->su.geom.ncell + 65535) / 65536));
    ESBGK_HIP(hipMalloc(&h->d_partials, sizeof(double) * 2 * h->Q * h->nchunks));
    ESBGK_HIP(hipMalloc(&h->d_totals, sizeof(double) * 8));
    return ESBGK_OK;
}

int create_impl(int D, int Q, int Nf, double Pr, double tau, const int64_t *dims, int storage, void *dev_buf,
                size_t bytes, void *stream, bool external, esbgk_t **out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return ESBGK_EINVAL;
    }
    *out = nullptr;
    auto *h = new (std::nothrow) esbgk_lattice();
    if (!h) {
        set_error("host allocation failed");
        return ESBGK_ENOMEM;
    }
    int rc = setup_domain(D, Q, Nf, Pr, tau, 0.2, dims, storage, h->su);
    if (rc) {
        delete h;
        return rc;
    }
    h->D = D;
    h->Q = Q;
    h->Nf = Nf;
    h->storage = storage;
    h->Pr = Pr;
    h->tau = tau;
    for (int d = 0; d < D; d++) h->dims[d] = dims[d];
    h->ops = get_ops(D, Q, h->su.codec);
    h->stream = (hipStream_t)stream;
    if (external) {
        if (!dev_buf || bytes < h->su.bytes || ((uintptr_t)dev_buf & 255)) {
            set_error("dev_buf must be non-NULL, 256-byte aligned and hold %llu bytes (got %zu)",
                      (unsigned long long)h->su.bytes, bytes);
            delete h;
            return ESBGK_EINVAL;
        }
        h->buf = (char *)dev_buf;
        h->owns_buf = false;
    } else {
        hipError_t e = hipMalloc(&h->buf, h->su.bytes);
        if (e != hipSuccess) {
            set_error("hipMalloc of %llu bytes failed: %s", (unsigned long long)h->su.bytes, hipGetErrorString(e));
            (void)hipGetLastError();
            delete h;
            return e == hipErrorOutOfMemory ? ESBGK_ENOMEM : ESBGK_EDEVICE;
        }
        h->owns_buf = true;
    }
    rc = alloc_aux(h);
    if (rc) {
        esbgk_destroy(h);
        return rc;
    }
    *out = h;
    return ESBGK_OK;
}

int check(const esbgk_t *h) {
    if (!h) {
        set_error("handle is NULL");
        return ESBGK_EINVAL;
    }
    return ESBGK_OK;
}

int check_init(const esbgk_t *h) {
    if (int rc = check(h)) return rc;
    if (!h->initialized) {
        set_error("lattice has no state yet: call esbgk_init_fields (or esbgk_load) first");
        return ESBGK_ESTATE;
    }
    return ESBGK_OK;
}

int launch_error() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("kernel launch failed: %s", hipGetErrorString(e));
        return ESBGK_EDEVICE;
    }
    return ESBGK_OK;
}

// HIP events owned by the call (destroyed on every return path).
struct Events {
    std::vector<hipEvent_t> e;
    ~Events() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
    int create(uint64_t n) {
        if (int rc = host_buffer(e, n)) return rc;
        for (auto &x : e) ESBGK_HIP(hipEventCreate(&x));
        return ESBGK_OK;
    }
};

// Device scratch of at least n bytes owned by the call.
struct DevTmp {
    void *p = nullptr;
    ~DevTmp() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" {

const char *esbgk_last_error(void) { return g_err; }

const char *esbgk_version(void) { return "esbgk-mi355x 0.1 (gfx950)"; }

int esbgk_lattice_info(int D, int Q, int *c, double *w, double *r, int *reach) {
    clear_error();
    LatticeConsts lc;
    if (!lattice_consts(D, Q, lc)) {
        set_error("unsupported lattice D%dQ%d", D, Q);
        return ESBGK_EUNSUPPORTED;
    }
    for (int i = 0; i < Q; i++) {
        if (c)
            for (int d = 0; d < 3; d++) c[3 * i + d] = lc.c[i][d];
        if (w) w[i] = lc.wshell[lc.shell_of[i]];
    }
    if (r) *r = lc.r;
    if (reach) *reach = lc.reach;
    return ESBGK_OK;
}

int esbgk_params(int D, int N_f, double Pr, double tau, double kappa, double out[4]) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return ESBGK_EINVAL;
    }
    char msg[256];
    int rc = derive_params(D, N_f, Pr, tau, kappa, out, msg, sizeof msg);
    if (rc) set_error("%s", msg);
    return rc;
}

int esbgk_storage_bytes(int D, int Q, int N_f, const int64_t *dims, int storage, size_t *bytes) {
    clear_error();
    DomainSetup su;
    int rc = setup_domain(D, Q, N_f, 1.0, 1.0, 0.2, dims, storage, su);
    if (rc) return rc;
    if (!bytes) {
        set_error("bytes is NULL");
        return ESBGK_EINVAL;
    }
    *bytes = su.bytes;
    return ESBGK_OK;
}

int esbgk_create(int D, int Q, int N_f, double Pr, double tau, const int64_t *dims, int storage, esbgk_t **out) {
    return create_impl(D, Q, N_f, Pr, tau, dims, storage, nullptr, 0, nullptr, false, out);
}

int esbgk_create_ex(int D, int Q, int N_f, double Pr, double tau, const int64_t *dims, int storage, void *dev_buf,
                    size_t bytes, void *hip_stream, esbgk_t **out) {
    return create_impl(D, Q, N_f, Pr, tau, dims, storage, dev_buf, bytes, hip_stream, true, out);
}

int esbgk_set_kappa(esbgk_t *h, double kappa) {
    clear_error();
    if (int rc = check(h)) return rc;
    double prm[4];
    char msg[256];
    int rc = derive_params(h->D, h->Nf, h->Pr, h->tau, kappa, prm, msg, sizeof msg);
    if (rc) {
        set_error("%s", msg);
        return rc;
    }
    h->kappa = kappa;
    std::memcpy(h->su.prm, prm, sizeof prm);
    h->su.coll = make_coll(h->su.lc, prm, h->D, h->Nf, kappa);
    return ESBGK_OK;
}

int esbgk_set_stream(esbgk_t *h, void *hip_stream) {
    clear_error();
    if (int rc = check(h)) return rc;
    h->stream = (hipStream_t)hip_stream;
    return ESBGK_OK;
}

int esbgk_init_fields(esbgk_t *h, const double *rho, const double *u, const double *T) {
    clear_error();
    if (int rc = check(h)) return rc;
    const uint64_t n = h->su.geom.ncell;
    std::vector<float> host;
    if (int rc = host_buffer(host, (2 + h->D) * n)) return rc;
    if (int rc = fields_to_dev(rho, u, T, h->D, n, host.data())) return rc;
    DevTmp tmp;
    ESBGK_HIP(hipMalloc(&tmp.p, host.size() * sizeof(float)));
    ESBGK_HIP(hipMemcpyAsync(tmp.p, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
    h->steps = 0;
    h->from_step = false;
    h->ops->init(h->fb(), h->gb(), h->pb(), h->sb(), h->su.geom, h->su.coll, (const float *)tmp.p, h->lay(),
                 h->has_g(), h->stream);
    if (int rc = launch_error()) return rc;
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    h->initialized = true;
    return ESBGK_OK;
}

int esbgk_step(esbgk_t *h, int64_t n) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    if (n < 0) {
        set_error("n must be >= 0");
        return ESBGK_EINVAL;
    }
    for (int64_t k = 0; k < n; k++) h->launch_step();
    return launch_error();
}

int esbgk_set_walls(esbgk_t *h, const double *bottom, const double *top) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (!bottom && !top) {
        h->walls = false;
        return ESBGK_OK;
    }
    if (!bottom || !top) {
        set_error("give both walls (or neither, to remove them)");
        return ESBGK_EINVAL;
    }
    if (h->su.copies != 2) {
        set_error("walls need the two-copy streaming scheme (storage | ESBGK_PULL)");
        return ESBGK_EINVAL;
    }
    if (h->open_x) {
        set_error("walls and open x ends cannot be combined");
        return ESBGK_EINVAL;
    }
    const LatticeConsts &lc = h->su.lc;
    int R = 0;
    for (int i = 0; i < h->Q; i++) R = std::max(R, lc.c[i][1]);
    if (h->dims[1] < 2 * R + 1) {
        set_error("walls need ny >= %d (%d ghost rows per wall and one gas row)", 2 * R + 1, R);
        return ESBGK_EINVAL;
    }
    const double *wv[2] = {bottom, top};
    for (int w = 0; w < 2; w++)
        for (int a = 0; a < 4; a++)
            if (!std::isfinite(wv[w][a]) || (a == 3 && !(wv[w][3] > 0))) {
                set_error("wall velocity must be finite and wall temperature finite and > 0");
                return ESBGK_EINVAL;
            }
    WallSet ws{};
    ws.reach = R;
    DevTmp tmp;
    ESBGK_HIP(hipMalloc(&tmp.p, sizeof(double) * 2 * MAX_Q));
    for (int w = 0; w < 2; w++) {
        const double u[3] = {wv[w][0], wv[w][1], h->D == 3 ? wv[w][2] : 0.0};
        h->ops->equilibrium_one(h->su.coll, u, wv[w][3] - 1.0, (double *)tmp.p + w * MAX_Q, h->stream);
    }
    if (int rc = launch_error()) return rc;
    ESBGK_HIP(hipMemcpyAsync(ws.G, tmp.p, sizeof ws.G, hipMemcpyDeviceToHost, h->stream));
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    for (int w = 0; w < 2; w++) {
        ws.T[w] = wv[w][3];
        for (int i = 0; i < h->Q; i++) {
            const int cy = lc.c[i][1];
            const bool into_gas = (w == 0 && cy > 0) || (w == 1 && cy < 0);
            const bool into_wall = (w == 0 && cy < 0) || (w == 1 && cy > 0);
            if (into_gas) ws.emit[w] += std::abs(cy) * ws.G[w][i];
            if (into_wall) ws.rest[w] += std::abs(cy) * lc.wshell[lc.shell_of[i]];
        }
    }
    h->ws = ws;
    h->walls = true;
    if (h->initialized && h->from_step) {
        h->apply_walls();
        if (int rc = launch_error()) return rc;
    }
    return ESBGK_OK;
}

int esbgk_set_open_x(esbgk_t *h, int on) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (!on) {
        h->open_x = false;
        return ESBGK_OK;
    }
    if (h->su.copies != 2) {
        set_error("open ends need the two-copy streaming scheme (storage | ESBGK_PULL)");
        return ESBGK_EINVAL;
    }
    if (h->walls) {
        set_error("walls and open x ends cannot be combined");
        return ESBGK_EINVAL;
    }
    int R = 0;
    for (int i = 0; i < h->Q; i++) R = std::max(R, h->su.lc.c[i][0]);
    if (h->dims[0] < 2 * R + 1) {
        set_error("open ends need nx >= %d (%d ghost columns per end and one gas column)", 2 * R + 1, R);
        return ESBGK_EINVAL;
    }
    h->rx = (uint32_t)R;
    h->open_x = true;
    if (h->initialized && h->from_step) {
        h->apply_open_x();
        if (int rc = launch_error()) return rc;
    }
    return ESBGK_OK;
}

int esbgk_plane_pad(const esbgk_t *h, int64_t *bytes) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (!bytes) {
        set_error("bytes is NULL");
        return ESBGK_EINVAL;
    }
    *bytes = (int64_t)h->su.plane_pad;
    return ESBGK_OK;
}

int esbgk_step_count(const esbgk_t *h, int64_t *n) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (!n) {
        set_error("n is NULL");
        return ESBGK_EINVAL;
    }
    *n = h->steps;
    return ESBGK_OK;
}

int esbgk_read_moments(esbgk_t *h, double *rho, double *u, double *T, double *P) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    const uint64_t n = h->su.geom.ncell;
    const int D = h->D, np = D * (D + 1) / 2;
    const uint64_t planes = 2 + D + (P ? np : 0);
    DevTmp tmp;
    ESBGK_HIP(hipMalloc(&tmp.p, planes * n * sizeof(float)));
    h->ops->moments(h->fb(), h->gb(), h->pb(), h->sb(), h->su.geom, h->su.coll, h->lay(), h->has_g(),
                    (float *)tmp.p, P != nullptr, h->stream);
    if (int rc = launch_error()) return rc;
    std::vector<float> host;
    if (int rc = host_buffer(host, planes * n)) return rc;
    ESBGK_HIP(hipMemcpyAsync(host.data(), tmp.p, host.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    for (uint64_t k = 0; k < n; k++) {
        if (rho) rho[k] = 1.0 + (double)host[k];
        if (T) T[k] = 1.0 + (double)host[(1 + D) * n + k];
    }
    if (u)
        for (uint64_t k = 0; k < (uint64_t)D * n; k++) u[k] = (double)host[n + k];
    if (P) {
        int q = 0;
        for (int a = 0; a < D; a++)
            for (int b = a; b < D; b++, q++)
                for (uint64_t k = 0; k < n; k++) P[q * n + k] = (a == b ? 1.0 : 0.0) + (double)host[(2 + D + q) * n + k];
    }
    return ESBGK_OK;
}

int esbgk_totals(esbgk_t *h, double *out) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    if (!out) {
        set_error("out is NULL");
        return ESBGK_EINVAL;
    }
    if (h->walls || h->open_x) {
        set_error("totals cover the whole periodic domain; with walls or open ends the ghost cells are not gas");
        return ESBGK_ESTATE;
    }
    h->ops->plane_sums(h->fb(), h->gb(), h->pb(), h->sb(), h->su.geom.ncell, h->Q, h->has_g(), h->d_partials,
                       h->nchunks, h->stream);
    launch_totals_final(h->d_partials, h->nchunks, h->su.lc, h->su.npop, h->lay() == LAY_ODD, h->su.geom.ncell,
                        0.5 * h->Nf, h->d_totals, h->stream);
    if (int rc = launch_error()) return rc;
    ESBGK_HIP(hipMemcpyAsync(out, h->d_totals, sizeof(double) * (2 + h->D), hipMemcpyDeviceToHost, h->stream));
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    return ESBGK_OK;
}

int esbgk_read_cells(esbgk_t *h, int64_t n, const int64_t *cells, double *f, double *g) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    if (n < 0 || (n > 0 && (!cells || !f))) {
        set_error("need n >= 0 and non-NULL cells and f");
        return ESBGK_EINVAL;
    }
    if (n == 0) return ESBGK_OK;
    if (n > (int64_t)1 << 28) {
        set_error("too many cells requested");
        return ESBGK_EINVAL;
    }
    std::vector<uint32_t> list;
    if (int rc = host_buffer(list, n)) return rc;
    for (int64_t k = 0; k < n; k++) {
        if (cells[k] < 0 || cells[k] >= (int64_t)h->su.geom.ncell) {
            set_error("cell index %lld out of range", (long long)cells[k]);
            return ESBGK_EINVAL;
        }
        list[k] = (uint32_t)cells[k];
    }
    const int Q = h->Q, npop = h->su.npop;
    DevTmp dl, dout;
    ESBGK_HIP(hipMalloc(&dl.p, n * sizeof(uint32_t)));
    ESBGK_HIP(hipMalloc(&dout.p, (size_t)n * Q * npop * sizeof(float)));
    ESBGK_HIP(hipMemcpyAsync(dl.p, list.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    h->ops->cells(h->fb(), h->gb(), h->pb(), h->sb(), h->su.geom, h->su.coll, h->lay(), h->has_g(),
                  (const uint32_t *)dl.p, (uint32_t)n, (float *)dout.p, h->stream);
    if (int rc = launch_error()) return rc;
    std::vector<float> host;
    if (int rc = host_buffer(host, (size_t)n * Q * npop)) return rc;
    ESBGK_HIP(hipMemcpyAsync(host.data(), dout.p, host.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    const LatticeConsts &lc = h->su.lc;
    for (int64_t k = 0; k < n; k++)
        for (int i = 0; i < Q; i++) {
            const double w = lc.wshell[lc.shell_of[i]];
            f[k * Q + i] = w + (double)host[(size_t)k * Q + i];
            if (g && npop == 2) g[k * Q + i] = 0.5 * h->Nf * w + (double)host[(size_t)n * Q + (size_t)k * Q + i];
        }
    return ESBGK_OK;
}

int esbgk_read_populations(esbgk_t *h, double *f, double *g) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    if (!f) {
        set_error("f is NULL");
        return ESBGK_EINVAL;
    }
    const uint64_t n = h->su.geom.ncell;
    const int Q = h->Q, npop = h->su.npop;
    DevTmp dout;
    ESBGK_HIP(hipMalloc(&dout.p, n * Q * npop * sizeof(float)));
    h->ops->cells(h->fb(), h->gb(), h->pb(), h->sb(), h->su.geom, h->su.coll, h->lay(), h->has_g(), nullptr,
                  (uint32_t)n, (float *)dout.p, h->stream);
    if (int rc = launch_error()) return rc;
    std::vector<float> host;
    if (int rc = host_buffer(host, n * Q * npop)) return rc;
    ESBGK_HIP(hipMemcpyAsync(host.data(), dout.p, host.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    const LatticeConsts &lc = h->su.lc;
    for (int i = 0; i < Q; i++) {
        const double w = lc.wshell[lc.shell_of[i]];
        for (uint64_t k = 0; k < n; k++) {
            f[i * n + k] = w + (double)host[i * n + k];
            if (g && npop == 2) g[i * n + k] = 0.5 * h->Nf * w + (double)host[(Q + i) * n + k];
        }
    }
    return ESBGK_OK;
}

int esbgk_write_populations(esbgk_t *h, const double *f, const double *g) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (!f || (h->su.npop == 2 && !g)) {
        set_error("f (and g when N_f > 0) must not be NULL");
        return ESBGK_EINVAL;
    }
    const uint64_t n = h->su.geom.ncell;
    const int Q = h->Q, npop = h->su.npop;
    const LatticeConsts &lc = h->su.lc;
    std::vector<float> host;
    if (int rc = host_buffer(host, n * Q * npop)) return rc;
    for (int i = 0; i < Q; i++) {
        const int sh = lc.shell_of[i];
        const double w = lc.wshell[sh];
        for (uint64_t k = 0; k < n; k++) {
            if (!std::isfinite(f[i * n + k]) || (npop == 2 && !std::isfinite(g[i * n + k]))) {
                set_error("non-finite population (plane %d, cell %llu)", i, (unsigned long long)k);
                return ESBGK_ENONFINITE;
            }
            host[i * n + k] = (float)std::ldexp(f[i * n + k] - w, lc.scale_exp[sh]);
            if (npop == 2) host[(Q + i) * n + k] = (float)std::ldexp(g[i * n + k] - 0.5 * h->Nf * w, lc.scale_exp[sh]);
        }
    }
    DevTmp din;
    ESBGK_HIP(hipMalloc(&din.p, host.size() * sizeof(float)));
    ESBGK_HIP(hipMemcpyAsync(din.p, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
    h->ops->write(h->fb(), h->gb(), h->pb(), h->sb(), h->su.geom, h->lay(), h->has_g(), (const float *)din.p,
                  h->stream);
    if (int rc = launch_error()) return rc;
    h->from_step = false;
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    h->initialized = true;
    return ESBGK_OK;
}

// ---------------------------------------------------------------- checkpoints
namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, D, Q, Nf, storage;
    int32_t flags;   // bit 0: the state was written by a step
    int64_t dims[3];
    int64_t steps;
    double Pr, tau, kappa;
    uint64_t bytes;
};
}  // namespace

int esbgk_save(esbgk_t *h, const char *path) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    if (!path) {
        set_error("path is NULL");
        return ESBGK_EINVAL;
    }
    // the current state only (one copy), in the unpadded layout
    DomainSetup su0 = h->su;
    if (int rc = set_layout(su0, 0)) return rc;
    std::vector<char> host;
    if (int rc = host_buffer(host, su0.copy_bytes)) return rc;
    if (int rc = copy_layout(host.data(), su0, h->fb(), h->su, 1, hipMemcpyDeviceToHost, h->stream)) return rc;
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    CkptHeader hd{};
    std::memcpy(hd.magic, "ESBGKCK2", 8);
    hd.version = 2;
    hd.D = h->D;
    hd.Q = h->Q;
    hd.Nf = h->Nf;
    hd.storage = storage_unpadded(h->storage);
    for (int d = 0; d < 3; d++) hd.dims[d] = h->dims[d];
    hd.steps = h->steps;
    hd.flags = h->from_step ? 1 : 0;
    hd.Pr = h->Pr;
    hd.tau = h->tau;
    hd.kappa = h->kappa;
    hd.bytes = su0.copy_bytes;
    FILE *fp = std::fopen(path, "wb");
    if (!fp) {
        set_error("cannot open %s for writing", path);
        return ESBGK_EIO;
    }
    bool ok = std::fwrite(&hd, sizeof hd, 1, fp) == 1 && std::fwrite(host.data(), 1, host.size(), fp) == host.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) {
        set_error("write to %s failed", path);
        return ESBGK_EIO;
    }
    return ESBGK_OK;
}

int esbgk_load(esbgk_t *h, const char *path) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (!path) {
        set_error("path is NULL");
        return ESBGK_EINVAL;
    }
    FILE *fp = std::fopen(path, "rb");
    if (!fp) {
        set_error("cannot open %s", path);
        return ESBGK_EIO;
    }
    CkptHeader hd{};
    if (std::fread(&hd, sizeof hd, 1, fp) != 1 || std::memcmp(hd.magic, "ESBGKCK2", 8) != 0) {
        std::fclose(fp);
        set_error("%s is not an esbgk checkpoint", path);
        return ESBGK_EIO;
    }
    DomainSetup su0 = h->su;   // the unpadded layout checkpoints are written in
    if (int rc = set_layout(su0, 0)) {
        std::fclose(fp);
        return rc;
    }
    bool same = hd.D == h->D && hd.Q == h->Q && hd.Nf == h->Nf && hd.storage == storage_unpadded(h->storage) &&
                hd.bytes == su0.copy_bytes;
    for (int d = 0; d < 3; d++) same = same && hd.dims[d] == h->dims[d];
    if (!same) {
        std::fclose(fp);
        set_error("checkpoint %s does not match this lattice (shape, N_f or storage)", path);
        return ESBGK_EINVAL;
    }
    if (hd.version != 2 || hd.steps < 0) {
        std::fclose(fp);
        set_error("%s has an unknown version or a negative step count", path);
        return ESBGK_EIO;
    }
    std::vector<char> host;
    if (int rc = host_buffer(host, hd.bytes)) {
        std::fclose(fp);
        return rc;
    }
    const bool ok = std::fread(host.data(), 1, host.size(), fp) == host.size();
    std::fclose(fp);
    if (!ok) {
        set_error("%s is truncated", path);
        return ESBGK_EIO;
    }
    // parameters of the checkpoint take effect
    double prm[4];
    char msg[256];
    if (int rc = derive_params(h->D, h->Nf, hd.Pr, hd.tau, hd.kappa, prm, msg, sizeof msg)) {
        set_error("%s", msg);
        return rc;
    }
    h->Pr = hd.Pr;
    h->tau = hd.tau;
    h->kappa = hd.kappa;
    std::memcpy(h->su.prm, prm, sizeof prm);
    h->su.coll = make_coll(h->su.lc, prm, h->D, h->Nf, hd.kappa);
    h->steps = hd.steps;
    h->from_step = (hd.flags & 1) != 0;
    if (int rc = copy_layout(h->fb(), h->su, host.data(), su0, 1, hipMemcpyHostToDevice, h->stream)) return rc;
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    h->initialized = true;
    return ESBGK_OK;
}

int esbgk_step_timed(esbgk_t *h, int64_t n, double *total_ms, double *per_launch_ms) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    if (n < 1 || !total_ms) {
        set_error("need n >= 1 and total_ms");
        return ESBGK_EINVAL;
    }
    Events events;
    if (int rc = events.create((uint64_t)n + 1)) return rc;
    std::vector<hipEvent_t> &ev = events.e;
    int rc = ESBGK_OK;
    ESBGK_HIP(hipEventRecord(ev[0], h->stream));
    for (int64_t k = 0; k < n; k++) {
        h->launch_step();
        ESBGK_HIP(hipEventRecord(ev[k + 1], h->stream));
    }
    rc = launch_error();
    ESBGK_HIP(hipEventSynchronize(ev[n]));
    float ms = 0;
    ESBGK_HIP(hipEventElapsedTime(&ms, ev[0], ev[n]));
    *total_ms = ms;
    if (per_launch_ms)
        for (int64_t k = 0; k < n; k++) {
            ESBGK_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            per_launch_ms[k] = ms;
        }
    return rc;
}

int esbgk_set_tile(esbgk_t *h, int parity, int block, int order, int policy, int cells_per_item) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (block == 0) block = 256;
    if (cells_per_item == 0) cells_per_item = 1;
    if (block < 64 || block > 512 || (block & 63)) {
        set_error("block must be a multiple of 64 in [64, 512] (got %d)", block);
        return ESBGK_EINVAL;
    }
    if (parity < -1 || parity > 1 || order < 0 || order > 2 || policy < 0 || policy > 3 || cells_per_item < 1 ||
        cells_per_item > 64) {
        set_error("need parity -1..1, order 0..2, policy 0..3, cells_per_item 1..64");
        return ESBGK_EINVAL;
    }
    Tile t;
    t.block = block;
    t.remap = order == 2 ? 1 : 0;
    t.policy = policy == 2 ? 1 : policy == 3 ? 2 : 0;
    t.cpi = cells_per_item;
    if (parity != 1) h->tile[0] = t;
    if (parity != 0) h->tile[1] = t;
    return ESBGK_OK;
}

int esbgk_get_tile(const esbgk_t *h, int parity, int *block, int *order, int *policy, int *cells_per_item) {
    clear_error();
    if (int rc = check(h)) return rc;
    if (parity < 0 || parity > 1) {
        set_error("parity must be 0 (even-layout kernel) or 1 (odd-layout kernel)");
        return ESBGK_EINVAL;
    }
    const Tile &t = h->tile[parity];
    if (block) *block = t.block;
    if (order) *order = t.remap ? 2 : 1;
    if (policy) *policy = t.policy + 1;
    if (cells_per_item) *cells_per_item = t.cpi;
    return ESBGK_OK;
}

namespace {
std::string tune_key(const esbgk_t *h) {
    int sc = 0;
    while ((1ull << (sc + 1)) <= h->su.geom.ncell) sc++;
    char k[128];
    snprintf(k, sizeof k, "D%dQ%d npop%d st%d log2n%d", h->D, h->Q, h->su.npop, storage_unpadded(h->storage), sc);
    return k;
}

// Plane paddings the autotuner times on library-owned storage (bytes).
constexpr uint64_t kPadCandidates[] = {0, 16384, 24576, 49152};

// Move library-owned storage to a new allocation laid out with plane
// padding `pad` (the state is copied across).  The old allocation is freed.
int relayout(esbgk_t *h, uint64_t pad) {
    DomainSetup nsu = h->su;
    if (int rc = set_layout(nsu, pad)) return rc;
    char *nb = nullptr;
    if (hipError_t e = hipMalloc(&nb, nsu.bytes); e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %llu bytes failed: %s", (unsigned long long)nsu.bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? ESBGK_ENOMEM : ESBGK_EDEVICE;
    }
    int rc = copy_layout(nb, nsu, h->buf, h->su, h->su.copies, hipMemcpyDeviceToDevice, h->stream);
    if (rc == ESBGK_OK && hipStreamSynchronize(h->stream) != hipSuccess) {
        set_error("copy to the new layout failed");
        rc = ESBGK_EDEVICE;
    }
    if (rc) {
        (void)hipFree(nb);
        return rc;
    }
    (void)hipFree(h->buf);
    h->buf = nb;
    h->su = nsu;
    return ESBGK_OK;
}
}  // namespace

int esbgk_autotune(esbgk_t *h, double budget_ms, const char *cache_path) {
    clear_error();
    if (int rc = check_init(h)) return rc;
    const std::string key = tune_key(h);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        bool got[2] = {false, false};
        long long pad = -1;
        while (std::getline(in, line)) {
            if (line.rfind(key + " ", 0) != 0) continue;
            int par, b, o, p, k;
            long long pd;
            if (sscanf(line.c_str() + key.size(), " parity %d block %d order %d policy %d cpi %d", &par, &b, &o, &p,
                       &k) == 5 &&
                (par == 0 || par == 1) && esbgk_set_tile(h, par, b, o, p, k) == ESBGK_OK)
                got[par] = true;
            else if (sscanf(line.c_str() + key.size(), " plane_pad %lld", &pd) == 1 && pd >= 0)
                pad = pd;
        }
        if (got[0] && got[1] && (!h->owns_buf || pad >= 0)) {
            clear_error();
            if (h->owns_buf && (uint64_t)pad != h->su.plane_pad) return relayout(h, (uint64_t)pad);
            return ESBGK_OK;
        }
        clear_error();
    }
    DevTmp save;
    ESBGK_HIP(hipMalloc(&save.p, h->su.bytes));
    ESBGK_HIP(hipMemcpyAsync(save.p, h->buf, h->su.bytes, hipMemcpyDeviceToDevice, h->stream));
    const DomainSetup su_entry = h->su;   // layout of the saved state
    const int64_t steps0 = h->steps;
    const bool from_step0 = h->from_step;
    Events events;
    if (int rc = events.create(7)) return rc;
    const std::vector<hipEvent_t> &ev = events.e;
    double best[2] = {1e30, 1e30};
    Tile bestt[2] = {h->tile[0], h->tile[1]};
    const auto t_start = std::chrono::steady_clock::now();
    int rc = ESBGK_OK;
    for (int block : {256, 512, 128})
        for (int remap : {0, 1})
            for (int policy : {0, 1, 2})
                for (int cpi : {1, 4, 16}) {
                    const double el =
                        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
                    if (rc || (budget_ms > 0 && el > budget_ms && best[1] < 1e30)) continue;
                    Tile t;
                    t.block = block;
                    t.remap = remap;
                    t.policy = policy;
                    t.cpi = cpi;
                    h->tile[0] = h->tile[1] = t;
                    h->launch_step();   // warm-up pair
                    h->launch_step();
                    for (int rep = 0; rep < 2; rep++) {
                        // six launches, each bracketed by events: three per parity
                        int par_of[6];
                        (void)hipEventRecord(ev[0], h->stream);
                        for (int k = 0; k < 6; k++) {
                            par_of[k] = h->odd() ? 1 : 0;
                            h->launch_step();
                            (void)hipEventRecord(ev[k + 1], h->stream);
                        }
                        if ((rc = launch_error())) break;
                        (void)hipEventSynchronize(ev[6]);
                        for (int k = 0; k < 6; k++) {
                            float ms = 0;
                            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
                            const int par = par_of[k];
                            if (ms < best[par]) {
                                best[par] = ms;
                                bestt[par] = t;
                            }
                        }
                    }
                }
    if (!rc) {
        h->tile[0] = bestt[0];
        h->tile[1] = bestt[1];
    }
    // Library-owned storage: time the plane paddings, each on an allocation
    // of its own, and keep the fastest allocation (where an allocation lands
    // in HBM matters as much as the padding itself).
    if (!rc && h->owns_buf) {
        auto time_now = [&](double *ms) -> int {
            h->launch_step();
            h->launch_step();
            (void)hipEventRecord(ev[0], h->stream);
            for (int k = 0; k < 6; k++) h->launch_step();
            (void)hipEventRecord(ev[1], h->stream);
            if (int r = launch_error()) return r;
            float f = 0;
            if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&f, ev[0], ev[1]) != hipSuccess) {
                set_error("timing events failed");
                return ESBGK_EDEVICE;
            }
            *ms = f;
            return ESBGK_OK;
        };
        double best_ms = 0;
        rc = time_now(&best_ms);
        char *best_buf = h->buf;
        DomainSetup best_su = h->su;
        const uint64_t pad0 = h->su.plane_pad;
        for (uint64_t pad : kPadCandidates) {
            if (rc || pad == pad0) continue;
            DomainSetup nsu = best_su;
            if (set_layout(nsu, pad) != ESBGK_OK) {
                clear_error();
                continue;
            }
            char *nb = nullptr;
            if (hipMalloc(&nb, nsu.bytes) != hipSuccess) {   // no room for a trial: keep what there is
                (void)hipGetLastError();
                break;
            }
            rc = copy_layout(nb, nsu, best_buf, best_su, best_su.copies, hipMemcpyDeviceToDevice, h->stream);
            h->buf = nb;
            h->su = nsu;
            double ms = 0;
            if (!rc) rc = time_now(&ms);
            (void)hipStreamSynchronize(h->stream);
            if (!rc && ms < best_ms) {
                (void)hipFree(best_buf);
                best_buf = nb;
                best_su = nsu;
                best_ms = ms;
            } else {
                (void)hipFree(nb);
                h->buf = best_buf;
                h->su = best_su;
            }
        }
    }
    // put the entry state back, in the (possibly new) layout
    if (int r = copy_layout(h->buf, h->su, (const char *)save.p, su_entry, su_entry.copies,
                            hipMemcpyDeviceToDevice, h->stream);
        r && !rc)
        rc = r;
    ESBGK_HIP(hipStreamSynchronize(h->stream));
    h->steps = steps0;
    h->from_step = from_step0;
    if (rc) return rc;
    if (cache_path) {
        FILE *fp = std::fopen(cache_path, "a");
        if (!fp) {
            set_error("cannot append to %s", cache_path);
            return ESBGK_EIO;
        }
        for (int par = 0; par < 2; par++)
            std::fprintf(fp, "%s parity %d block %d order %d policy %d cpi %d ms %.4f\n", key.c_str(), par,
                         bestt[par].block, bestt[par].remap ? 2 : 1, bestt[par].policy + 1, bestt[par].cpi,
                         best[par]);
        if (h->owns_buf) std::fprintf(fp, "%s plane_pad %llu\n", key.c_str(), (unsigned long long)h->su.plane_pad);
        std::fclose(fp);
    }
    return ESBGK_OK;
}

void esbgk_destroy(esbgk_t *h) {
    if (!h) return;
    if (h->owns_buf && h->buf) (void)hipFree(h->buf);
    if (h->d_partials) (void)hipFree(h->d_partials);
    if (h->d_totals) (void)hipFree(h->d_totals);
    delete h;
}

}  // extern "C"
