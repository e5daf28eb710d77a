// gks_api.hip -- host side of the C ABI declared in include/gks.h: validation, workspace carving,
// launch sequencing of one S2O4 step (Section 2) and the body-force update (Section 3.3) on the
// caller's stream, and the FP64 result readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gks.h"
#include "gks_adjoint.h"
#include "gks_body.h"
#include "gks_internal.h"
#include "gks_stats.h"

using namespace gks;

static thread_local std::string g_init_error;

struct Carver {
    char* base;
    size_t off;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
    template <typename T>
    T* ptr(size_t bytes) {
        size_t o = take(bytes);
        return base ? reinterpret_cast<T*>(base + o) : nullptr;
    }
};

struct gks_ctx {
    gks_config cfg;
    GridDesc g;
    size_t es;
    void* q[4];
    void* qs[4];
    void* qa[4];
    char* ws;
    size_t ws_bytes;
    hipStream_t stream;
    DevState* st;
    // residual contributions of the y pass (r0: L, r1: L_t) and of the x pass (rx0, rx1, blocked
    // layout), four variables per cell
    void* r0;
    void* r1;
    void* rx0;
    void* rx1;
    void* qt[4];  // copy of the stage input in the layout [x][z][y], read by the x-direction face pass
    // FP32: low-order parts of Q^n / Q^{n+1}, Q* and S ([cell][4]); the state is field + low part
    void* lo_q;
    void* lo_qs;
    void* lo_qa;
    double* diag_partials;
    int diag_nblk;
    double* umax_part;  // per-workgroup maxima of |U|^2 for the CFL time step
    // per-axis inverse spacings in the stage precision (face spacings [n + 1], widths [n]) and FP64
    // relative widths; stretched: some axis has its own faces
    void* ihf[3];
    void* ihc[3];
    double* wrel[3];
    int stretched;
    std::vector<double> faces[3];  // host copy of the faces of each stretched axis (empty when uniform)
    double lam, c, hmin, eps;
    int chunk[3];      // faces per workgroup of the face kernels, per direction
    int seg_len[3], n_wg[3];  // work split of the order-5 face launches (FaceArgs)
    int flags;
    // actuator line model
    int has_rotor;
    AlmArgs alm;
    double* alm_mem;   // start of the rotor block in the workspace
    // immersed boundary
    int has_ibm;
    IbmArgs ibm;
    char* ibm_mem;
    int ibm_moving;    // rigid motion set: supports rebuilt on the device every step
    IbmMoveArgs ibm_mv;
    // checkpoints
    char* ckpt;
    int ckpt_cap;
    int ckpt_n;
    // running statistics and load history
    double* stats_buf;
    int stats_interval;
    long long stats_n;
    long long host_step;
    double* hist_buf;
    int hist_cap;
    long long hist_n;
    // event timing
    int timing;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_cat;   // category of each recorded pair
    size_t ev_used;            // events in use (2 per pair)
    double t_ms[GKS_TIMER_COUNT];
    long long t_cnt[GKS_TIMER_COUNT];
    std::string err;
    int static_dev;  // device whose static scratch holds the workspace (gks_init_static), else -1
};

// Workspace for callers that cannot allocate device memory (gks_init_static): one array per GPU, held
// until the process ends. Host code never names it in a kernel argument or a copy: it uses the device
// address hipGetSymbolAddress returns, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[GKS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kStaticDevices = 64;
struct StaticSlot {
    void* ptr;             // device address of this GPU's scratch (null until first use)
    const gks_ctx* owner;  // the context whose workspace it is, or null
};
std::mutex g_static_mu;
StaticSlot g_static[kStaticDevices];

}  // namespace

namespace {

const int kPerm[3][4] = {{0, 1, 2, 3}, {0, 2, 1, 3}, {0, 3, 1, 2}};  // local -> global variable
const int kAxes[3][3] = {{0, 1, 2}, {1, 0, 2}, {2, 0, 1}};          // (normal, t1, t2) axes

int fail(gks_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_init_error = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), GKS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(const gks_config* c) { return c->precision == GKS_FP32 ? 4 : 8; }

// t2 extent of the face tile: the high-order kernel's per-precision tile, 16 for the second-order one
template <typename real>
int face_tile_t2(int order) {
    return order == 2 ? TILE2 : FaceTile<real>::T2;
}

// workspace layout; base == nullptr only measures
struct Layout {
    DevState* st;
    void* ihf[3];
    void* ihc[3];
    double* wrel[3];
    void* r0;
    void* r1;
    void* rx0;
    void* rx1;
    void* qt[4];
    void* lo[3];
    double* diag;
    double* umax_part;
    char* alm;
    char* ibm;
    size_t total;
};

size_t alm_block_bytes(int n) {
    if (n <= 0) return 0;
    Carver cv{nullptr, 0};
    for (int i = 0; i < 4; ++i) cv.take(sizeof(double) * n);          // r, chord, twist, width
    cv.take(sizeof(double) * 3 * n);                                   // X
    cv.take(sizeof(double) * 3 * n);                                   // fv
    for (int i = 0; i < 5; ++i) cv.take(sizeof(double) * n);          // alpha, fx, ft, urel, phi
    cv.take(sizeof(double) * 3 * n);                                   // sampled u
    return cv.off;
}

int radix_tiles(long long npairs) { return (int)((npairs + RADIX_TILE - 1) / RADIX_TILE); }

// Lagrangian-point block of the workspace; the carving order here and in gks_set_ibm_points agree
size_t ibm_block_bytes(long long n) {
    if (n <= 0) return 0;
    const long long nc = 64 * n;
    Carver cv{nullptr, 0};
    cv.take(sizeof(double) * 3 * n);
    cv.take(sizeof(double) * n);
    cv.take(sizeof(int) * 3 * nc);
    cv.take(sizeof(int) * (nc + 1));
    cv.take(sizeof(int) * nc);
    cv.take(sizeof(double) * nc);
    cv.take(sizeof(double) * 3 * ((nc + 255) / 256));
    cv.take(sizeof(double) * 3 * n);   // point velocities
    cv.take(sizeof(double) * 3 * nc);  // v-bar
    // rebinning of a moving body
    cv.take(sizeof(double) * 3 * n);   // positions at t0
    cv.take(sizeof(int) * 3 * n);      // lowest support cell
    for (int b = 0; b < 4; ++b) cv.take(sizeof(int) * nc);  // pair keys and values, ping-pong
    cv.take(sizeof(int) * 256 * radix_tiles(nc));
    cv.take(sizeof(int) * 256);
    cv.take(sizeof(int) * radix_tiles(nc));
    cv.take(sizeof(int) * 2);
    return cv.off;
}

bool layout(const gks_config* c, char* base, Layout* L) {
    const size_t es = elem_size(c);
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    Carver cv{base, 0};
    L->st = cv.ptr<DevState>(sizeof(DevState));
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
        L->ihf[a] = cv.ptr<void>((n[a] + 1) * es);
        L->ihc[a] = cv.ptr<void>(n[a] * es);
        L->wrel[a] = cv.ptr<double>(sizeof(double) * n[a]);
    }
    L->r0 = cv.ptr<void>(4 * N * es);
    L->r1 = cv.ptr<void>(4 * N * es);
    const size_t NB = (size_t)c->nx * ((c->ny + 15) / 16) * 16 * c->nz;
    L->rx0 = cv.ptr<void>(4 * NB * es);
    L->rx1 = cv.ptr<void>(4 * NB * es);
    const size_t NP = (size_t)(c->nx + 6) * (c->ny + 6) * (c->nz + 6);
    for (int v = 0; v < 4; ++v) L->qt[v] = cv.ptr<void>(NP * es);
    for (int b = 0; b < 3; ++b) L->lo[b] = c->precision == GKS_FP32 ? cv.ptr<void>(4 * N * es) : nullptr;
    L->diag = cv.ptr<double>(sizeof(double) * 4 * 1024);
    L->umax_part = cv.ptr<double>(sizeof(double) * UMAX_BLOCKS);
    size_t ab = alm_block_bytes(c->max_act);
    L->alm = ab ? cv.ptr<char>(ab) : nullptr;
    size_t ib = ibm_block_bytes(c->max_ibm);
    L->ibm = ib ? cv.ptr<char>(ib) : nullptr;
    L->total = cv.off;
    return true;
}

std::string validate(const gks_config* c) {
    if (!c) return "config is null";
    if (c->nx < 3 || c->ny < 3 || c->nz < 3) return "nx, ny, nz must be >= 3";
    if (c->nx > 65000 || c->ny > 65000 || c->nz > 65000) return "nx, ny, nz must be <= 65000";
    if ((long long)c->nx * c->ny * c->nz > (1LL << 31)) return "grid too large (more than 2^31 cells)";
    if (c->precision != GKS_FP32 && c->precision != GKS_FP64) return "precision must be GKS_FP32 or GKS_FP64";
    if (!(c->lx > 0 && c->ly > 0 && c->lz > 0)) return "domain lengths must be > 0";
    if (!(c->ma > 0 && c->u_ref > 0 && c->rho_ref > 0)) return "ma, u_ref and rho_ref must be > 0";
    if (!(c->mu >= 0)) return "mu must be >= 0";
    if (!(c->cfl > 0) && !(c->dt_fixed > 0)) return "either cfl > 0 or dt_fixed > 0";
    for (int s = 0; s < 6; ++s)
        if (c->bc[s] < GKS_BC_PERIODIC || c->bc[s] > GKS_BC_OUTFLOW) return "unknown boundary kind";
    for (int a = 0; a < 3; ++a)
        if ((c->bc[2 * a] == GKS_BC_PERIODIC) != (c->bc[2 * a + 1] == GKS_BC_PERIODIC))
            return "periodic boundaries must be paired";
    if (c->max_act < 0 || c->max_act > 1024) return "max_act must be in [0, 1024]";
    if (c->max_ibm < 0 || c->max_ibm > (1LL << 24)) return "max_ibm must be in [0, 2^24]";
    if (c->max_ibm > 0 && c->ibm_iters < 1) return "ibm_iters must be >= 1";
    if (c->order != 0 && c->order != 2 && c->order != 5) return "order must be 5 (or 0) or 2";
    const int n[3] = {c->nx, c->ny, c->nz};
    const double org[3] = {c->x0, c->y0, c->z0}, len[3] = {c->lx, c->ly, c->lz};
    for (int a = 0; a < 3; ++a) {
        const double* f = c->faces[a];
        if (!f) continue;
        if (c->bc[2 * a] == GKS_BC_PERIODIC) return "a periodic axis must be uniform (faces NULL)";
        for (int i = 0; i < n[a]; ++i)
            if (!(std::isfinite(f[i]) && std::isfinite(f[i + 1]) && f[i + 1] > f[i]))
                return "faces must be finite and increasing";
        if (!(std::fabs(f[0] - org[a]) <= 1e-12 * len[a] && std::fabs(f[n[a]] - org[a] - len[a]) <= 1e-12 * len[a]))
            return "faces must run from the origin to origin + length of their axis";
    }
    return "";
}

// Inverse spacings of axis a (face spacings [n + 1], widths [n]) and relative widths, from the faces
// of a stretched axis or the uniform size h.
void axis_metrics(const gks_config* c, int a, double h, std::vector<double>* ihf, std::vector<double>* ihc,
                  std::vector<double>* wrel) {
    const int n = a == 0 ? c->nx : (a == 1 ? c->ny : c->nz);
    ihf->assign(n + 1, 1.0 / h);
    ihc->assign(n, 1.0 / h);
    wrel->assign(n, 1.0);
    const double* f = c->faces[a];
    if (!f) return;
    for (int i = 0; i < n; ++i) {
        const double w = f[i + 1] - f[i];
        (*ihc)[i] = 1.0 / w;
        (*wrel)[i] = w / h;
    }
    for (int i = 1; i < n; ++i) (*ihf)[i] = 1.0 / (0.5 * ((f[i] - f[i - 1]) + (f[i + 1] - f[i])));
    (*ihf)[0] = (*ihc)[0];
    (*ihf)[n] = (*ihc)[n - 1];
}

// Grid that a body sees: on a stretched axis the cells from the one holding lo[a] to the one holding
// hi[a], widened by pad cells, must share one width w; the body then works on the uniform grid of that
// block (origin x_{i-1/2} - i w at its first cell i, spacing w). Uniform axes keep the context grid.
// run[a] (optional) receives the widest run of cells of that width around the block, [first, last]
// (all cells of a uniform axis): the cells a moving body may reach without leaving that grid.
bool body_grid(const gks_ctx* c, const double lo[3], const double hi[3], int pad, GridDesc* out,
               int run_lo[3] = nullptr, int run_hi[3] = nullptr) {
    *out = c->g;
    for (int a = 0; a < 3; ++a) {
        const std::vector<double>& f = c->faces[a];
        if (run_lo) {
            run_lo[a] = 0;
            run_hi[a] = c->g.n[a] - 1;
        }
        if (f.empty()) continue;
        const int n = (int)f.size() - 1;
        int i0 = (int)(std::upper_bound(f.begin(), f.end(), lo[a]) - f.begin()) - 1 - pad;
        int i1 = (int)(std::upper_bound(f.begin(), f.end(), hi[a]) - f.begin()) - 1 + pad;
        i0 = std::max(0, i0);
        i1 = std::min(n - 1, i1);
        if (i1 < i0) return false;
        const double w = f[i0 + 1] - f[i0];
        auto same = [&](int i) { return std::fabs((f[i + 1] - f[i]) - w) <= 1e-12 * w; };
        for (int i = i0; i <= i1; ++i)
            if (!same(i)) return false;
        out->x0[a] = f[i0] - i0 * w;
        out->h[a] = w;
        if (run_lo) {
            int r0 = i0, r1 = i1;
            while (r0 > 0 && same(r0 - 1)) --r0;
            while (r1 < n - 1 && same(r1 + 1)) ++r1;
            run_lo[a] = r0;
            run_hi[a] = r1;
        }
    }
    return true;
}

// Copy the per-axis metrics into the workspace; synchronises (the host copies live until then).
template <typename real>
hipError_t upload_metrics(gks_ctx* c, const gks_config* cfg) {
    std::vector<real> hf[3], hw[3];
    std::vector<double> hr[3];
    for (int a = 0; a < 3; ++a) {
        std::vector<double> f, w;
        axis_metrics(cfg, a, c->g.h[a], &f, &w, &hr[a]);
        hf[a].assign(f.begin(), f.end());
        hw[a].assign(w.begin(), w.end());
        hipError_t e = hipMemcpyAsync(c->ihf[a], hf[a].data(), hf[a].size() * sizeof(real), hipMemcpyHostToDevice,
                                      c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ihc[a], hw[a].data(), hw[a].size() * sizeof(real), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->wrel[a], hr[a].data(), hr[a].size() * sizeof(double), hipMemcpyHostToDevice,
                               c->stream);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(c->stream);
}

template <typename real>
Field4<real> field(void* const p[4]) {
    Field4<real> f;
    for (int v = 0; v < 4; ++v) f.v[v] = static_cast<real*>(p[v]);
    return f;
}

template <typename real>
int ghost_all(gks_ctx* c, void* const p[4]) {
    Field4<real> f = field<real>(p);
    for (int a = 0; a < 3; ++a)
        HIPCHK(c, launch_ghost<real>(f, c->g, a, c->cfg.bc[2 * a], c->cfg.bc[2 * a + 1], c->cfg.u_in, c->c,
                                     c->cfg.rho_ref, c->stream));
    return GKS_OK;
}

// Face-kernel arguments for direction d. stage 1: reads src, writes out_a = Q*, out_b = S and reads
// q_c = Q^n in the epilogue; stage 2: reads src = Q*, writes out_a = Q^{n+1} from s_in = S.
template <typename real>
FaceArgs<real> face_args_buf(gks_ctx* c, int d, int stage, void* const src[4], void* const out_a[4],
                             void* const out_b[4], void* const q_c[4], void* const xt[4] = nullptr,
                             void* lo_in = nullptr, void* lo_a = nullptr, void* lo_b = nullptr) {
    FaceArgs<real> a;
    std::memset(&a, 0, sizeof(a));
    const int* pm = kPerm[d];
    const int* ax = kAxes[d];
    const long long ist[3] = {1, c->cfg.nx, (long long)c->cfg.nx * c->cfg.ny};
    for (int v = 0; v < 4; ++v) {
        const int gv = pm[v];
        a.q[v] = static_cast<const real*>(src[gv]);

        a.out_a[v] = static_cast<real*>(out_a[gv]);

        if (stage == 1) {
            a.out_b[v] = static_cast<real*>(out_b[gv]);
            a.q_c[v] = static_cast<const real*>(q_c[gv]);
        } else {
            a.s_in[v] = static_cast<const real*>(out_b[gv]);
        }
    }
    a.r0 = static_cast<real*>(c->r0);
    a.r1 = static_cast<real*>(c->r1);
    a.rx0 = static_cast<real*>(c->rx0);
    a.rx1 = static_cast<real*>(c->rx1);
    a.lo_in = static_cast<const real*>(lo_in);
    a.lo_a = static_cast<real*>(lo_a);
    a.lo_b = static_cast<real*>(lo_b);
    a.n_n = c->g.n[ax[0]];
    a.n_t1 = c->g.n[ax[1]];
    a.n_t2 = c->g.n[ax[2]];
    const int t2 = face_tile_t2<real>(c->cfg.order);
    a.tiles_t1 = (a.n_t1 + TILE1 - 1) / TILE1;
    a.tiles_t2 = (a.n_t2 + t2 - 1) / t2;
    a.chunk = c->chunk[d];
    a.seg_len = c->seg_len[d];
    a.n_wg = c->n_wg[d];
    a.st_n = c->g.st[ax[0]];
    a.st_t1 = c->g.st[ax[1]];
    a.st_t2 = c->g.st[ax[2]];
    a.ist_n = ist[ax[0]];
    a.ist_t1 = ist[ax[1]];
    a.ist_t2 = ist[ax[2]];
    a.pad0 = c->g.pad0;
    if (d == 0 && xt) {
        // the x pass reads the [x][z][y] copy of src: n = x, t1 = y (unit stride), t2 = z
        const long long Y = c->cfg.ny + 6, Z = c->cfg.nz + 6;
        for (int v = 0; v < 4; ++v) a.q[v] = static_cast<const real*>(xt[pm[v]]);
        a.st_n = Y * Z;
        a.st_t1 = 1;
        a.st_t2 = Y;
        a.pad0 = 3 * (Y * Z + 1 + Y);
    }
    a.inv_hn = real(1.0 / c->g.h[ax[0]]);
    a.inv_h1 = real(1.0 / c->g.h[ax[1]]);
    a.inv_h2 = real(1.0 / c->g.h[ax[2]]);
    a.stretched = c->stretched;
    a.ihf = static_cast<const real*>(c->ihf[ax[0]]);
    a.ihc = static_cast<const real*>(c->ihc[ax[0]]);
    a.ih1 = static_cast<const real*>(c->ihc[ax[1]]);
    a.ih2 = static_cast<const real*>(c->ihc[ax[2]]);
    a.eps = real(c->eps);
    a.fc.lam = real(c->lam);
    a.fc.sl = real(std::sqrt(c->lam));
    a.fc.kk = real(1.0 / (2.0 * std::sqrt(M_PI * c->lam)));
    a.fc.c2 = real(1.0 / (2.0 * c->lam));
    a.fc.mu = real(c->cfg.mu);
    a.fc.rho_ref = real(c->cfg.rho_ref);
    for (int j = 0; j < 3; ++j) a.g_global[j] = real(c->cfg.body_force[j]);
    a.dt_ptr = &c->st->dt;
    // x faces write their own arrays in the blocked layout [z][y/16][x][y%16] so that the x pass
    // stores contiguous runs; the y pass writes the main arrays, the z pass accumulates both and
    // applies the S2O4 combination
    a.rx_nx = c->cfg.nx;
    a.rx_nyb = (c->cfg.ny + 15) / 16;
    a.mode = d == 0 ? 3 : (d == 1 ? 0 : 4);
    return a;
}

template <typename real>
FaceArgs<real> face_args(gks_ctx* c, int d, int stage, void* const src[4]) {
    if (stage == 1) return face_args_buf<real>(c, d, 1, src, c->qs, c->qa, c->q, c->qt, c->lo_q, c->lo_qs, c->lo_qa);
    return face_args_buf<real>(c, d, 2, src, c->q, c->qa, nullptr, c->qt, c->lo_qa, c->lo_q, nullptr);
}

AdjFaceArgs adj_args(gks_ctx* c, const AdjBuffers& B, int d, void* const src[4], int exact) {
    AdjFaceArgs a;
    std::memset(&a, 0, sizeof(a));
    const int* pm = kPerm[d];
    const int* ax = kAxes[d];
    const long long ist[3] = {1, c->cfg.nx, (long long)c->cfg.nx * c->cfg.ny};
    for (int v = 0; v < 4; ++v) {
        const int gv = pm[v];
        a.q[v] = static_cast<const double*>(src[gv]);
        a.mu0[v] = B.mu0[gv];
        a.mu1[v] = B.mu1[gv];
        a.acc[v] = B.acc[gv];
    }
    a.gpbar = B.gpbar;
    a.t1v = B.t1v;
    a.fv = B.fv;
    a.fabar = B.fabar;
    a.n_n = c->g.n[ax[0]];
    a.n_t1 = c->g.n[ax[1]];
    a.n_t2 = c->g.n[ax[2]];
    // the forward FP64 face tiles (16 x 8 faces, 256 threads) and march chunks
    a.tiles_t1 = (a.n_t1 + TILE1 - 1) / TILE1;
    a.tiles_t2 = (a.n_t2 + FaceTile<double>::T2 - 1) / FaceTile<double>::T2;
    a.chunk = c->chunk[d];
    a.st_n = c->g.st[ax[0]];
    a.st_t1 = c->g.st[ax[1]];
    a.st_t2 = c->g.st[ax[2]];
    a.ist_n = ist[ax[0]];
    a.ist_t1 = ist[ax[1]];
    a.ist_t2 = ist[ax[2]];
    a.pad0 = c->g.pad0;
    a.nface = (long long)(a.n_n + 1) * a.n_t1 * a.n_t2;
    a.nt1pos = (long long)(a.n_n + 1) * a.n_t1 * (a.n_t2 + 4);
    a.nnpos = (long long)(a.n_n + 1) * (a.n_t1 + 4) * (a.n_t2 + 4);
    a.ihf = static_cast<const double*>(c->ihf[ax[0]]);
    a.ihc = static_cast<const double*>(c->ihc[ax[0]]);
    a.ih1 = static_cast<const double*>(c->ihc[ax[1]]);
    a.ih2 = static_cast<const double*>(c->ihc[ax[2]]);
    a.eps = c->eps;
    a.fc.lam = c->lam;
    a.fc.sl = std::sqrt(c->lam);
    a.fc.kk = 1.0 / (2.0 * std::sqrt(M_PI * c->lam));
    a.fc.c2 = 1.0 / (2.0 * c->lam);
    a.fc.mu = c->cfg.mu;
    a.fc.rho_ref = c->cfg.rho_ref;
    a.exact = exact;
    return a;
}

int timing_flush(gks_ctx* c) {
    if (c->ev_used == 0) return GKS_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t p = 0; p < c->ev_cat.size(); ++p) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[2 * p], c->ev_pool[2 * p + 1]));
        c->t_ms[c->ev_cat[p]] += ms;
        c->t_cnt[c->ev_cat[p]] += 1;
    }
    c->ev_cat.clear();
    c->ev_used = 0;
    return GKS_OK;
}

// open a timed launch group; returns the pair index or -1 when timing is off
int tbeg(gks_ctx* c, int cat) {
    if (!c->timing) return -1;
    if (c->ev_used + 2 > 4096 && timing_flush(c) != GKS_OK) return -1;
    while (c->ev_pool.size() < c->ev_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        c->ev_pool.push_back(e);
    }
    const size_t i = c->ev_used;
    if (hipEventRecord(c->ev_pool[i], c->stream) != hipSuccess) return -1;
    c->ev_used += 2;
    c->ev_cat.push_back(cat);
    return (int)(i / 2);
}

void tend(gks_ctx* c, int pair) {
    if (pair >= 0) (void)hipEventRecord(c->ev_pool[2 * pair + 1], c->stream);
}

// FP32: zero the low-order parts of the compensated state (the state is then the field itself).
hipError_t clear_low_parts(gks_ctx* c) {
    if (c->cfg.precision != GKS_FP32) return hipSuccess;
    const size_t bytes = (size_t)4 * c->cfg.nx * c->cfg.ny * c->cfg.nz * sizeof(float);
    void* const sets[3] = {c->lo_q, c->lo_qs, c->lo_qa};
    for (int b = 0; b < 3; ++b) {
        hipError_t e = launch_zero_words(sets[b], bytes, c->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename real>
int steps(gks_ctx* c, int nsteps) {
    const size_t field_bytes = (size_t)c->g.n_padded * sizeof(real);
    const int cat1[3] = {GKS_TIMER_S1X, GKS_TIMER_S1Y, GKS_TIMER_S1Z};
    const int cat2[3] = {GKS_TIMER_S2X, GKS_TIMER_S2Y, GKS_TIMER_S2Z};
    const size_t fb = (field_bytes + 255) & ~size_t(255);
    for (int s = 0; s < nsteps; ++s) {
        int tp;
        // checkpoint slot of this step: Q^n, Q* and the field before the body forces, then t
        char* ck = nullptr;
        if (c->ckpt && c->ckpt_n < c->ckpt_cap) {
            tp = tbeg(c, GKS_TIMER_OTHER);
            const size_t slot = gks_checkpoint_slot_bytes(&c->cfg);
            ck = c->ckpt + (size_t)c->ckpt_n * slot;
            for (int v = 0; v < 4; ++v) HIPCHK(c, launch_copy_field(c->q[v], ck + v * fb, field_bytes, c->stream));
            HIPCHK(c, launch_copy_field(&c->st->t, ck + slot - 256, sizeof(double), c->stream));
            tend(c, tp);
            c->ckpt_n++;
        }
        tp = tbeg(c, GKS_TIMER_GHOST);
        HIPCHK(c, launch_ghost_transpose<real>(field<real>(c->q), field<real>(c->qt), c->g, c->cfg.bc, c->cfg.u_in,
                                               c->c, c->cfg.rho_ref, c->stream));
        tend(c, tp);
        tp = tbeg(c, GKS_TIMER_DT);
        if (c->cfg.cfl > 0) HIPCHK(c, launch_umax<real>(field<real>(c->q), c->g, c->cfg.rho_ref, c->umax_part, c->stream));
        HIPCHK(c, launch_dt(c->st, c->umax_part, umax_blocks(c->g), c->cfg.cfl, c->hmin, c->c, c->cfg.dt_fixed,
                            c->stream));
        tend(c, tp);
        for (int d = 0; d < 3; ++d) {
            tp = tbeg(c, cat1[d]);
            HIPCHK(c, c->cfg.order == 2 ? launch_face2<real>(face_args<real>(c, d, 1, c->q), 1, c->stream)
                                        : launch_face<real>(face_args<real>(c, d, 1, c->q), 1, c->stream));
            tend(c, tp);
        }
        if (ck) {
            tp = tbeg(c, GKS_TIMER_OTHER);
            for (int v = 0; v < 4; ++v) HIPCHK(c, launch_copy_field(c->qs[v], ck + (4 + v) * fb, field_bytes, c->stream));
            tend(c, tp);
        }
        tp = tbeg(c, GKS_TIMER_GHOST);
        HIPCHK(c, launch_ghost_transpose<real>(field<real>(c->qs), field<real>(c->qt), c->g, c->cfg.bc, c->cfg.u_in,
                                               c->c, c->cfg.rho_ref, c->stream));
        tend(c, tp);
        for (int d = 0; d < 3; ++d) {
            tp = tbeg(c, cat2[d]);
            HIPCHK(c, c->cfg.order == 2 ? launch_face2<real>(face_args<real>(c, d, 2, c->qs), 2, c->stream)
                                        : launch_face<real>(face_args<real>(c, d, 2, c->qs), 2, c->stream));
            tend(c, tp);
        }
        if (ck) {
            tp = tbeg(c, GKS_TIMER_OTHER);
            for (int v = 0; v < 4; ++v) HIPCHK(c, launch_copy_field(c->q[v], ck + (8 + v) * fb, field_bytes, c->stream));
            tend(c, tp);
        }
        if (c->has_rotor) {
            tp = tbeg(c, GKS_TIMER_ALM);
            HIPCHK(c, launch_alm<real>(field<real>(c->q), c->alm, c->stream));
            tend(c, tp);
        }
        if (c->has_ibm) {
            tp = tbeg(c, GKS_TIMER_IBM);
            if (c->ibm_moving) HIPCHK(c, launch_ibm_move(c->ibm, c->ibm_mv, c->stream));
            HIPCHK(c, launch_ibm<real>(field<real>(c->q), c->ibm, c->stream));
            tend(c, tp);
        }
        tp = tbeg(c, GKS_TIMER_OTHER);
        double* hist = (c->hist_buf && c->hist_n < c->hist_cap) ? c->hist_buf + 10 * c->hist_n : nullptr;
        HIPCHK(c, launch_finish(c->st, c->has_rotor, hist, c->stream));
        if (hist) c->hist_n++;
        c->host_step++;
        if (c->stats_buf && c->host_step % c->stats_interval == 0) {
            StatsArgs sa;
            sa.g = c->g;
            sa.rho_ref = c->cfg.rho_ref;
            sa.buf = c->stats_buf;
            c->stats_n++;
            HIPCHK(c, launch_stats_accum<real>(field<real>(c->q), sa, 1.0 / (double)c->stats_n, c->stream));
        }
        tend(c, tp);
    }
    return GKS_OK;
}

}  // namespace

// ================================================================================================
// C ABI
// ================================================================================================
extern "C" {

size_t gks_workspace_bytes(const gks_config* cfg) {
    if (!validate(cfg).empty()) return 0;
    Layout L;
    layout(cfg, nullptr, &L);
    return L.total;
}

size_t gks_checkpoint_slot_bytes(const gks_config* cfg) {
    if (!validate(cfg).empty()) return 0;
    const size_t np = (size_t)(cfg->nx + 6) * (cfg->ny + 6) * (cfg->nz + 6);
    const size_t fb = ((np * elem_size(cfg)) + 255) & ~size_t(255);
    return 12 * fb + 256;  // Q^n, Q* and the field before the body forces; t
}

int gks_init(const gks_config* cfg, gks_field q, gks_field q_stage, gks_field q_acc, void* workspace,
             size_t workspace_bytes, void* hip_stream, gks_ctx** out) {
    if (!out) return fail(nullptr, GKS_E_INVALID_ARG, "out is null");
    *out = nullptr;
    std::string why = validate(cfg);
    if (!why.empty()) return fail(nullptr, GKS_E_INVALID_ARG, why);
    void* qp[4] = {q.rho, q.mx, q.my, q.mz};
    void* sp[4] = {q_stage.rho, q_stage.mx, q_stage.my, q_stage.mz};
    void* ap[4] = {q_acc.rho, q_acc.mx, q_acc.my, q_acc.mz};
    for (int v = 0; v < 4; ++v)
        if (!qp[v] || !sp[v] || !ap[v]) return fail(nullptr, GKS_E_INVALID_ARG, "a field pointer is null");
    if (!workspace) return fail(nullptr, GKS_E_INVALID_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(nullptr, GKS_E_INVALID_ARG, "workspace must be 256-byte aligned");
    Layout L;
    layout(cfg, nullptr, &L);
    if (workspace_bytes < L.total)
        return fail(nullptr, GKS_E_INVALID_ARG,
                    "workspace too small: need " + std::to_string(L.total) + " bytes (gks_workspace_bytes)");
    gks_ctx* c = new (std::nothrow) gks_ctx();
    if (!c) return fail(nullptr, GKS_E_INVALID_ARG, "out of host memory");
    c->static_dev = -1;
    c->cfg = *cfg;
    if (!(c->cfg.weno_eps > 0)) c->cfg.weno_eps = 1e-6;
    c->es = elem_size(cfg);
    for (int v = 0; v < 4; ++v) {
        c->q[v] = qp[v];
        c->qs[v] = sp[v];
        c->qa[v] = ap[v];
    }
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = workspace_bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    layout(cfg, c->ws, &L);
    c->st = L.st;
    for (int v = 0; v < 4; ++v) c->qt[v] = L.qt[v];
    c->r0 = L.r0;
    c->r1 = L.r1;
    c->rx0 = L.rx0;
    c->rx1 = L.rx1;
    c->lo_q = L.lo[0];
    c->lo_qs = L.lo[1];
    c->lo_qa = L.lo[2];
    c->diag_partials = L.diag;
    c->umax_part = L.umax_part;
    c->alm_mem = reinterpret_cast<double*>(L.alm);
    c->ibm_mem = L.ibm;
    const int n[3] = {cfg->nx, cfg->ny, cfg->nz};
    const double len[3] = {cfg->lx, cfg->ly, cfg->lz};
    const double org[3] = {cfg->x0, cfg->y0, cfg->z0};
    for (int a = 0; a < 3; ++a) {
        c->g.n[a] = n[a];
        c->g.h[a] = len[a] / n[a];
        c->g.x0[a] = org[a];
    }
    c->g.st[0] = 1;
    c->g.st[1] = n[0] + 6;
    c->g.st[2] = (long long)(n[0] + 6) * (n[1] + 6);
    c->g.pad0 = 3 * (c->g.st[0] + c->g.st[1] + c->g.st[2]);
    c->g.n_padded = (long long)(n[0] + 6) * (n[1] + 6) * (n[2] + 6);
    c->lam = cfg->ma * cfg->ma / (2.0 * cfg->u_ref * cfg->u_ref);
    c->c = std::sqrt(1.0 / (2.0 * c->lam));
    c->hmin = std::min(c->g.h[0], std::min(c->g.h[1], c->g.h[2]));
    c->stretched = 0;
    for (int a = 0; a < 3; ++a) {
        c->ihf[a] = L.ihf[a];
        c->ihc[a] = L.ihc[a];
        c->wrel[a] = L.wrel[a];
        c->g.wrel[a] = nullptr;
        if (cfg->faces[a]) {
            c->stretched = 1;
            c->g.wrel[a] = L.wrel[a];
            c->faces[a].assign(cfg->faces[a], cfg->faces[a] + n[a] + 1);
            for (int i = 0; i < n[a]; ++i) c->hmin = std::min(c->hmin, cfg->faces[a][i + 1] - cfg->faces[a][i]);
        }
        c->cfg.faces[a] = nullptr;  // the caller's arrays are read here only
    }
    c->eps = c->cfg.weno_eps;
    c->diag_nblk = diag_blocks(c->g);
    c->flags = cfg->ma > 0.3 ? GKS_WARN_MACH : 0;
    const int slots = cfg->order == 2 ? (cfg->precision == GKS_FP32 ? face2_slots<float>() : face2_slots<double>())
                                      : (cfg->precision == GKS_FP32 ? face_slots<float>() : face_slots<double>());
    const int t2 = cfg->precision == GKS_FP32 ? face_tile_t2<float>(cfg->order) : face_tile_t2<double>(cfg->order);
    for (int d = 0; d < 3; ++d) {
        const int* ax = kAxes[d];
        const int tiles = ((n[ax[1]] + TILE1 - 1) / TILE1) * ((n[ax[2]] + t2 - 1) / t2);
        c->chunk[d] = cfg->precision == GKS_FP32 ? face_chunk<float>(n[ax[0]], tiles, slots)
                                                 : face_chunk<double>(n[ax[0]], tiles, slots);
        face_plan(n[ax[0]], tiles, slots, c->chunk[d], &c->seg_len[d], &c->n_wg[d]);
    }
    hipError_t e = cfg->precision == GKS_FP32 ? upload_metrics<float>(c, cfg) : upload_metrics<double>(c, cfg);
    if (e == hipSuccess) e = hipMemsetAsync(c->st, 0, sizeof(DevState), c->stream);
    if (e == hipSuccess) e = clear_low_parts(c);
    if (e != hipSuccess) {
        g_init_error = std::string("clearing the device state: ") + hipGetErrorString(e);
        delete c;
        return GKS_E_HIP;
    }
    int rc = cfg->precision == GKS_FP32 ? ghost_all<float>(c, c->q) : ghost_all<double>(c, c->q);
    if (rc) {
        g_init_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return GKS_OK;
}

int gks_set_actuators(gks_ctx* c, const gks_rotor* r) {
    if (!c) return GKS_E_INVALID_ARG;
    if (!r) return fail(c, GKS_E_INVALID_ARG, "rotor is null");
    const int n = r->n_blades * r->n_per_blade;
    if (r->n_blades < 1 || r->n_per_blade < 1) return fail(c, GKS_E_INVALID_ARG, "n_blades and n_per_blade must be >= 1");
    if (n > c->cfg.max_act) return fail(c, GKS_E_INVALID_ARG, "more actuator points than config.max_act");
    if (!r->r || !r->chord || !r->twist || !r->width) return fail(c, GKS_E_INVALID_ARG, "rotor arrays are null");
    if (!(r->eps > 0) || !(r->radius > 0) || !(r->u_inf > 0)) return fail(c, GKS_E_INVALID_ARG, "eps, radius and u_inf must be > 0");
    double rmax = 0.0;
    for (int i = 0; i < r->n_per_blade; ++i) {
        if (!(r->r[i] >= 0) || !(r->chord[i] >= 0) || !(r->width[i] >= 0))
            return fail(c, GKS_E_INVALID_ARG, "negative radius, chord or width");
        rmax = std::max(rmax, r->r[i]);
    }
    if (r->u_inf_correction) {
        for (int i = 0; i < r->n_per_blade; ++i)
            if (r->chord[i] * (r->cd0 + r->cd2 * (M_PI * M_PI)) >= 4.0 * std::sqrt(M_PI) * r->eps)
                return fail(c, GKS_E_INVALID_ARG, "free-stream correction denominator can vanish (chord too large for eps)");
    }
    if (!(r->line_half_length >= 0.0) || !std::isfinite(r->line_half_length))
        return fail(c, GKS_E_INVALID_ARG, "line_half_length must be finite and >= 0");
    const bool line = r->line_points > 1 && r->line_half_length > 0.0;
    // distance from the rotor axis that a sampling position can reach over a revolution (a segment
    // along the direction of motion at radius r reaches sqrt(r^2 + l^2))
    const double reach = line ? std::sqrt(rmax * rmax + r->line_half_length * r->line_half_length) : rmax;
    // box of cells the rotor can touch: projection spheres (3 eps) around the swept disc, plus the
    // trilinear sampling cells; it must lie inside the interior cells (and on a stretched mesh within
    // cells of one width)
    const double ext = 3.0 * r->eps;
    const double lo[3] = {r->hub[0] - ext, r->hub[1] - rmax - ext, r->hub[2] - rmax - ext};
    const double hi[3] = {r->hub[0] + ext, r->hub[1] + rmax + ext, r->hub[2] + rmax + ext};
    const double glo[3] = {lo[0], std::min(lo[1], r->hub[1] - reach), std::min(lo[2], r->hub[2] - reach)};
    const double ghi[3] = {hi[0], std::max(hi[1], r->hub[1] + reach), std::max(hi[2], r->hub[2] + reach)};
    GridDesc gb;
    if (!body_grid(c, glo, ghi, 1, &gb))
        return fail(c, GKS_E_UNSUPPORTED, "a rotor on a stretched mesh needs one cell width on the cells around it");
    AlmArgs& a = c->alm;
    std::memset(&a, 0, sizeof(a));
    for (int d = 0; d < 3; ++d) {
        int i0 = (int)std::ceil((lo[d] - gb.x0[d]) / gb.h[d] - 0.5);
        int i1 = (int)std::floor((hi[d] - gb.x0[d]) / gb.h[d] - 0.5);
        // sampling cells of any sampling position of the swept disc
        const double slo = (d == 0 ? r->hub[0] : r->hub[d] - reach), shi = (d == 0 ? r->hub[0] : r->hub[d] + reach);
        const int s0 = (int)std::floor((slo - gb.x0[d]) / gb.h[d] - 0.5);
        const int s1 = (int)std::floor((shi - gb.x0[d]) / gb.h[d] - 0.5) + 1;
        if (std::min(i0, s0) < 0 || std::max(i1, s1) >= c->g.n[d])
            return fail(c, GKS_E_INVALID_ARG, "rotor (points, sampling cells or 3 eps spheres) leaves the interior cells");
        a.box_lo[d] = i0;
        a.box_n[d] = i1 - i0 + 1;
        a.samp_lo[d] = s0;
        a.samp_n[d] = s1 - s0 + 1;
    }
    a.n_act = n;
    a.line_n = line ? r->line_points : 1;
    a.line_half = line ? r->line_half_length : 0.0;
    a.nb = r->n_blades;
    a.npb = r->n_per_blade;
    a.corr = r->u_inf_correction ? 1 : 0;
    a.tip = r->tip_correction ? 1 : 0;
    {
        const double tsr = r->omega * r->radius / r->u_inf;
        a.g1_axi = std::exp(-0.1219 * (r->n_blades * tsr - 21.52)) + 0.1;   // Section 4.4 constants
        a.g1_tan = std::exp(-0.0984 * (r->n_blades * tsr - 13.026)) + 0.1;
    }
    if (r->tip_correction)
        for (int i = 0; i < r->n_per_blade; ++i)
            if (!(r->r[i] > 0) || !(r->r[i] < r->radius))
                return fail(c, GKS_E_INVALID_ARG, "tip correction needs 0 < r < radius for every point");
    for (int d = 0; d < 3; ++d) a.hub[d] = r->hub[d];
    a.omega = r->omega;
    a.theta0 = r->theta0;
    a.radius = r->radius;
    a.u_inf = r->u_inf;
    a.eps = r->eps;
    a.cl_slope = r->cl_slope;
    a.alpha_clip = r->alpha_clip;
    a.cd0 = r->cd0;
    a.cd2 = r->cd2;
    a.rho_ref = c->cfg.rho_ref;
    a.area = M_PI * r->radius * r->radius;
    const int cap = c->cfg.max_act;
    Carver cv{reinterpret_cast<char*>(c->alm_mem), 0};
    double* tab[4];
    for (int i = 0; i < 4; ++i) tab[i] = cv.ptr<double>(sizeof(double) * cap);
    a.r = tab[0];
    a.chord = tab[1];
    a.twist = tab[2];
    a.width = tab[3];
    a.X = cv.ptr<double>(sizeof(double) * 3 * cap);
    a.fv = cv.ptr<double>(sizeof(double) * 3 * cap);
    a.out_alpha = cv.ptr<double>(sizeof(double) * cap);
    a.out_fx = cv.ptr<double>(sizeof(double) * cap);
    a.out_ft = cv.ptr<double>(sizeof(double) * cap);
    a.out_urel = cv.ptr<double>(sizeof(double) * cap);
    a.out_phi = cv.ptr<double>(sizeof(double) * cap);
    a.out_u = cv.ptr<double>(sizeof(double) * 3 * cap);
    a.scale = r->scale;
    a.g = gb;
    a.st = c->st;
    const double* src[4] = {r->r, r->chord, r->twist, r->width};
    for (int i = 0; i < 4; ++i)
        HIPCHK(c, hipMemcpyAsync(tab[i], src[i], sizeof(double) * r->n_per_blade, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (r->eps < 2.0 * std::min(gb.h[0], std::min(gb.h[1], gb.h[2]))) c->flags |= GKS_WARN_EPS_SMALL;
    else c->flags &= ~GKS_WARN_EPS_SMALL;
    c->has_rotor = 1;
    return GKS_OK;
}

int gks_set_ibm_points(gks_ctx* c, int64_t n, const double* xyz, const double* dS, const double* vel) {
    if (!c) return GKS_E_INVALID_ARG;
    if (n <= 0 || !xyz || !dS) return fail(c, GKS_E_INVALID_ARG, "need n > 0 points with xyz and dS");
    if (n > c->cfg.max_ibm) return fail(c, GKS_E_INVALID_ARG, "more Lagrangian points than config.max_ibm");
    // grid around the body (stretched meshes: the uniform block that holds it)
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long long p = 0; p < n; ++p)
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(xyz[3 * p + d])) return fail(c, GKS_E_INVALID_ARG, "non-finite point coordinate");
            blo[d] = std::min(blo[d], xyz[3 * p + d]);
            bhi[d] = std::max(bhi[d], xyz[3 * p + d]);
        }
    GridDesc gb;
    int run_lo[3], run_hi[3];
    if (!body_grid(c, blo, bhi, 2, &gb, run_lo, run_hi))
        return fail(c, GKS_E_UNSUPPORTED, "a body on a stretched mesh needs one cell width on the cells around it");
    // host-side binning (index work only): every (cell, point) pair of the 4x4x4 supports, sorted by
    // cell and then point, gives the cell list and a CSR of contributing points per cell
    std::vector<long long> keys;
    keys.reserve((size_t)n * 64);
    const long long nx = c->g.n[0], ny = c->g.n[1];
    for (long long p = 0; p < n; ++p) {
        if (!(dS[p] >= 0)) return fail(c, GKS_E_INVALID_ARG, "negative surface element");
        if (vel && !(std::isfinite(vel[3 * p]) && std::isfinite(vel[3 * p + 1]) && std::isfinite(vel[3 * p + 2])))
            return fail(c, GKS_E_INVALID_ARG, "non-finite point velocity");
        int i0[3];
        for (int d = 0; d < 3; ++d) {
            const double f = (xyz[3 * p + d] - gb.x0[d]) / gb.h[d] - 0.5;
            if (!std::isfinite(f)) return fail(c, GKS_E_INVALID_ARG, "non-finite point coordinate");
            i0[d] = (int)std::floor(f);
            if (i0[d] - 1 < 0 || i0[d] + 2 >= c->g.n[d])
                return fail(c, GKS_E_INVALID_ARG, "a Lagrangian point's 4x4x4 support leaves the interior cells");
        }
        for (int dk = -1; dk <= 2; ++dk)
            for (int dj = -1; dj <= 2; ++dj)
                for (int di = -1; di <= 2; ++di) {
                    const long long cell = ((long long)(i0[2] + dk) * ny + (i0[1] + dj)) * nx + (i0[0] + di);
                    keys.push_back(cell * (1LL << 25) + p);
                }
    }
    std::sort(keys.begin(), keys.end());
    std::vector<int> cells, csr, ent;
    csr.push_back(0);
    long long last = -1;
    for (long long kv : keys) {
        const long long cell = kv >> 25;
        const int p = (int)(kv & ((1LL << 25) - 1));
        if (cell != last) {
            if (last >= 0) csr.push_back((int)ent.size());
            cells.push_back((int)(cell % nx));
            cells.push_back((int)((cell / nx) % ny));
            cells.push_back((int)(cell / (nx * ny)));
            last = cell;
        }
        ent.push_back(p);
    }
    csr.push_back((int)ent.size());
    const int ncell = (int)(cells.size() / 3);
    const long long cap = c->cfg.max_ibm, nc = 64 * cap;
    Carver cv{c->ibm_mem, 0};
    IbmArgs& a = c->ibm;
    std::memset(&a, 0, sizeof(a));
    double* dx = cv.ptr<double>(sizeof(double) * 3 * cap);
    double* ds = cv.ptr<double>(sizeof(double) * cap);
    int* dcell = cv.ptr<int>(sizeof(int) * 3 * nc);
    int* dcsr = cv.ptr<int>(sizeof(int) * (nc + 1));
    int* dent = cv.ptr<int>(sizeof(int) * nc);
    a.vbar = cv.ptr<double>(sizeof(double) * nc);
    a.partials = cv.ptr<double>(sizeof(double) * 3 * ((nc + 255) / 256));
    double* dvel = cv.ptr<double>(sizeof(double) * 3 * cap);
    a.vbar_vel = cv.ptr<double>(sizeof(double) * 3 * nc);
    a.vel = vel ? dvel : nullptr;
    a.xyz = dx;
    IbmMoveArgs& m = c->ibm_mv;
    std::memset(&m, 0, sizeof(m));
    double* dx0 = cv.ptr<double>(sizeof(double) * 3 * cap);
    m.base = cv.ptr<int>(sizeof(int) * 3 * cap);
    for (int b = 0; b < 2; ++b) {
        m.key[b] = cv.ptr<unsigned>(sizeof(int) * nc);
        m.val[b] = cv.ptr<int>(sizeof(int) * nc);
    }
    m.hist = cv.ptr<int>(sizeof(int) * 256 * radix_tiles(nc));
    m.dtot = cv.ptr<int>(sizeof(int) * 256);
    m.tcnt = cv.ptr<int>(sizeof(int) * radix_tiles(nc));
    m.counts = cv.ptr<int>(sizeof(int) * 2);
    m.xyz0 = dx0;
    m.xyz = dx;
    for (int d = 0; d < 3; ++d) {
        m.run_lo[d] = run_lo[d];
        m.run_hi[d] = run_hi[d];
    }
    m.pvel = dvel;
    m.cell = dcell;
    m.csr = dcsr;
    m.ent = dent;
    c->ibm_moving = 0;
    a.dS = ds;
    a.cell = dcell;
    a.csr = dcsr;
    a.ent = dent;
    a.npts = (int)n;
    a.ncell = ncell;
    a.iters = c->cfg.ibm_iters;
    a.rho_ref = c->cfg.rho_ref;
    a.g = gb;
    a.st = c->st;
    HIPCHK(c, hipMemcpyAsync(dx, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dx0, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_zero_words(&c->st->ibm_outside, sizeof(int), c->stream));
    HIPCHK(c, hipMemcpyAsync(ds, dS, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    if (vel) HIPCHK(c, hipMemcpyAsync(dvel, vel, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dcell, cells.data(), sizeof(int) * cells.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dcsr, csr.data(), sizeof(int) * csr.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dent, ent.data(), sizeof(int) * ent.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_ibm_vbar(a, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->has_ibm = 1;
    return GKS_OK;
}

int gks_set_ibm_motion(gks_ctx* c, const gks_motion* mo) {
    if (!c) return GKS_E_INVALID_ARG;
    if (!mo) return fail(c, GKS_E_INVALID_ARG, "motion is null");
    if (!c->has_ibm) return fail(c, GKS_E_STATE, "no Lagrangian points: call gks_set_ibm_points first");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(mo->center[d]) || !std::isfinite(mo->velocity[d]) || !std::isfinite(mo->omega[d]))
            return fail(c, GKS_E_INVALID_ARG, "non-finite motion");
    if (!std::isfinite(mo->t0)) return fail(c, GKS_E_INVALID_ARG, "non-finite motion");
    IbmMoveArgs& m = c->ibm_mv;
    for (int d = 0; d < 3; ++d) {
        m.c0[d] = mo->center[d];
        m.vel[d] = mo->velocity[d];
        m.omega[d] = mo->omega[d];
    }
    m.t0 = mo->t0;
    HIPCHK(c, launch_zero_words(&c->st->ibm_outside, sizeof(int), c->stream));
    IbmArgs& a = c->ibm;
    a.vel = m.pvel;
    a.ncell = 64 * a.npts;
    a.ncell_dev = m.counts;
    a.moving = 1;
    c->ibm_moving = 1;
    return GKS_OK;
}

int gks_step(gks_ctx* c, int32_t nsteps) {
    if (!c) return GKS_E_INVALID_ARG;
    if (nsteps < 0) return fail(c, GKS_E_INVALID_ARG, "nsteps must be >= 0");
    return c->cfg.precision == GKS_FP32 ? steps<float>(c, nsteps) : steps<double>(c, nsteps);
}

int gks_forces(gks_ctx* c, gks_forces_out* out) {
    if (!c) return GKS_E_INVALID_ARG;
    if (!out) return fail(c, GKS_E_INVALID_ARG, "out is null");
    if (c->cfg.precision == GKS_FP32)
        HIPCHK(c, launch_diag<float>(field<float>(c->q), static_cast<const float*>(c->lo_q), c->g, c->cfg.rho_ref,
                                     c->diag_partials, c->diag_nblk, c->st, c->stream));
    else
        HIPCHK(c, launch_diag<double>(field<double>(c->q), nullptr, c->g, c->cfg.rho_ref, c->diag_partials,
                                      c->diag_nblk, c->st, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    DevState h;
    HIPCHK(c, hipMemcpy(&h, c->st, sizeof(DevState), hipMemcpyDeviceToHost));
    out->t = h.t;
    out->dt = h.dt;
    out->step = h.step;
    out->thrust = h.thrust;
    out->torque = h.torque;
    out->power = h.power;
    out->cp = h.cp;
    out->ct = h.ct;
    for (int d = 0; d < 3; ++d) out->ibm_force[d] = h.ibm_force[d];
    double rb;
    std::memcpy(&rb, &h.ibm_res_bits, sizeof(double));
    out->ibm_residual = c->has_ibm ? rb : 0.0;
    out->ibm_iters_used = c->has_ibm ? h.ibm_iters_used : 0;
    out->flags = c->flags;
    out->mass = h.mass;
    for (int d = 0; d < 3; ++d) out->mom[d] = h.mom[d];
    double u2;
    std::memcpy(&u2, &h.umax_diag_bits, sizeof(double));
    out->umax = std::sqrt(u2);
    out->window_power = h.win_p;
    out->window_thrust = h.win_t;
    out->window_steps = h.win_n;
    if (c->has_rotor) {
        const int n = c->alm.n_act;
        if (out->alpha) HIPCHK(c, hipMemcpy(out->alpha, c->alm.out_alpha, sizeof(double) * n, hipMemcpyDeviceToHost));
        if (out->fx) HIPCHK(c, hipMemcpy(out->fx, c->alm.out_fx, sizeof(double) * n, hipMemcpyDeviceToHost));
        if (out->ftheta) HIPCHK(c, hipMemcpy(out->ftheta, c->alm.out_ft, sizeof(double) * n, hipMemcpyDeviceToHost));
        if (out->urel) HIPCHK(c, hipMemcpy(out->urel, c->alm.out_urel, sizeof(double) * n, hipMemcpyDeviceToHost));
    }
    if (c->has_ibm && c->ibm_moving && h.ibm_outside)
        return fail(c, GKS_E_BODY_LEFT, "a moving Lagrangian point's support left the interior cells");
    if (h.nonfinite || !std::isfinite(out->mass)) return fail(c, GKS_E_NONFINITE, "non-finite value in the field");
    if (!(out->umax < c->c)) return fail(c, GKS_E_UNSTABLE, "|U|max reached the sound speed");
    return GKS_OK;
}

int gks_reset_window(gks_ctx* c) {
    if (!c) return GKS_E_INVALID_ARG;
    HIPCHK(c, launch_window_reset(c->st, c->stream));
    return GKS_OK;
}

int gks_field_changed(gks_ctx* c) {
    if (!c) return fail(nullptr, GKS_E_INVALID_ARG, "ctx is null");
    HIPCHK(c, clear_low_parts(c));
    return GKS_OK;
}

int gks_set_checkpoints(gks_ctx* c, void* buffer, int32_t capacity) {
    if (!c) return GKS_E_INVALID_ARG;
    if (buffer && capacity < 1) return fail(c, GKS_E_INVALID_ARG, "capacity must be >= 1");
    if (buffer && reinterpret_cast<uintptr_t>(buffer) % 256) return fail(c, GKS_E_INVALID_ARG, "checkpoint buffer must be 256-byte aligned");
    c->ckpt = static_cast<char*>(buffer);
    c->ckpt_cap = buffer ? capacity : 0;
    c->ckpt_n = 0;
    HIPCHK(c, launch_window_reset(c->st, c->stream));
    return GKS_OK;
}

size_t gks_adjoint_workspace_bytes(const gks_config* cfg, int32_t n_act) {
    if (!validate(cfg).empty() || n_act < 0) return 0;
    return adjoint_workspace_bytes(cfg->nx, cfg->ny, cfg->nz, n_act);
}

int gks_adjoint(gks_ctx* c, int32_t nsteps, const double w[2], double* grad_s, double* grad_q0, void* adj_ws,
                size_t adj_ws_bytes, int32_t flags) {
    if (!c) return GKS_E_INVALID_ARG;
    if (!w || !grad_s || !adj_ws) return fail(c, GKS_E_INVALID_ARG, "null argument");
    if (flags & ~GKS_ADJ_EXACT_WENO) return fail(c, GKS_E_INVALID_ARG, "unknown adjoint flags");
    const int exact = (flags & GKS_ADJ_EXACT_WENO) ? 1 : 0;
    if (c->cfg.precision != GKS_FP64) return fail(c, GKS_E_UNSUPPORTED, "the adjoint needs an FP64 context");
    if (c->cfg.order == 2) return fail(c, GKS_E_UNSUPPORTED, "the adjoint covers the high-order scheme only");
    if (c->cfg.cfl > 0) return fail(c, GKS_E_UNSUPPORTED, "the adjoint needs a fixed dt (cfl <= 0)");
    if (!c->has_rotor) return fail(c, GKS_E_STATE, "the adjoint needs a rotor (gks_set_actuators)");
    if (c->has_ibm && c->ibm_moving) return fail(c, GKS_E_UNSUPPORTED, "the adjoint does not cover moving bodies");
    if (!c->ckpt || nsteps < 1 || nsteps > c->ckpt_n)
        return fail(c, GKS_E_STATE, "need at least nsteps checkpointed steps (gks_set_checkpoints, then gks_step)");
    if (reinterpret_cast<uintptr_t>(adj_ws) % 256) return fail(c, GKS_E_INVALID_ARG, "adj_ws must be 256-byte aligned");
    const size_t need = adjoint_workspace_bytes(c->cfg.nx, c->cfg.ny, c->cfg.nz, c->alm.n_act);
    if (adj_ws_bytes < need)
        return fail(c, GKS_E_INVALID_ARG, "adjoint workspace too small: need " + std::to_string(need) + " bytes");
    AdjBuffers B;
    size_t tot = 0;
    adjoint_carve(static_cast<char*>(adj_ws), c->cfg.nx, c->cfg.ny, c->cfg.nz, c->alm.n_act, &B, &tot);
    const long long np = c->g.n_padded;
    const double dt = c->cfg.dt_fixed;
    hipStream_t S = c->stream;
    for (int v = 0; v < 4; ++v) HIPCHK(c, launch_zero(B.lam[v], np, S));
    HIPCHK(c, launch_zero(grad_s, c->alm.n_act, S));
    const size_t slot = gks_checkpoint_slot_bytes(&c->cfg);
    const size_t fb = ((size_t)np * 8 + 255) & ~size_t(255);
    void* qwork[4];
    void* qpre[4];
    for (int v = 0; v < 4; ++v) {
        qwork[v] = B.qwork[v];
        qpre[v] = B.qpre[v];
    }
    for (int n = nsteps - 1; n >= 0; --n) {
        // step n from its checkpoint: Q^n, Q* and the field before the body forces (stored by the
        // forward, bitwise what a recompute gives), and t
        const char* src = c->ckpt + (size_t)n * slot;
        for (int v = 0; v < 4; ++v) {
            HIPCHK(c, launch_copy_field(src + v * fb, B.qwork[v], (size_t)np * 8, S));
            HIPCHK(c, launch_copy_field(src + (4 + v) * fb, c->qs[v], (size_t)np * 8, S));
            HIPCHK(c, launch_copy_field(src + (8 + v) * fb, B.qpre[v], (size_t)np * 8, S));
        }
        HIPCHK(c, launch_copy_field(src + slot - 256, &c->st->t, sizeof(double), S));
        HIPCHK(c, launch_dt(c->st, nullptr, 0, 0.0, c->hmin, c->c, dt, S));
        int rc = ghost_all<double>(c, qwork);
        if (rc) return rc;
        rc = ghost_all<double>(c, c->qs);
        if (rc) return rc;
        HIPCHK(c, launch_alm_points_only(field<double>(qpre), c->alm, S));
        // immersed body (at rest): lam becomes the adjoint of the field before the forcing
        if (c->has_ibm) HIPCHK(c, launch_ibm_adjoint(B.lam, c->ibm, S));
        // actuator line: lam_pre = lam + (sampling path); gradient in s
        for (int v = 0; v < 4; ++v) HIPCHK(c, launch_axpby(B.lam_pre[v], B.lam[v], 1.0, nullptr, 0.0, np, S));
        AlmAdjArgs A;
        std::memset(&A, 0, sizeof(A));
        A.fwd = c->alm;
        for (int v = 0; v < 3; ++v) A.lam_m[v] = B.lam[1 + v];
        for (int v = 0; v < 4; ++v) {
            A.lam_pre[v] = B.lam_pre[v];
            A.qpre[v] = B.qpre[v];
        }
        A.grad_s = grad_s;
        A.pt = B.pt;
        A.w0 = w[0];
        A.w1 = w[1];
        A.inv_n = 1.0 / nsteps;
        HIPCHK(c, launch_alm_adjoint(A, S));
        // stage 2: lam* = (dt^2/3) J_Lt(Q*)^T lam_pre
        for (int v = 0; v < 4; ++v) {
            HIPCHK(c, launch_pad_to_int(B.mu1[v], B.lam_pre[v], dt * dt / 3.0, nullptr, 0.0, c->g, S));
            HIPCHK(c, launch_zero(B.acc[v], np, S));
        }
        for (int d = 0; d < 3; ++d) HIPCHK(c, launch_adj_direction(adj_args(c, B, d, c->qs, exact), 2, S));
        const double* qs_d[4] = {static_cast<const double*>(c->qs[0]), static_cast<const double*>(c->qs[1]),
                                 static_cast<const double*>(c->qs[2]), static_cast<const double*>(c->qs[3])};
        HIPCHK(c, launch_adj_fold(B.acc, c->g, c->cfg.bc, qs_d, c->cfg.u_in, c->c, c->cfg.rho_ref, S));
        for (int v = 0; v < 4; ++v) HIPCHK(c, launch_axpby(B.lam_star[v], B.acc[v], 1.0, nullptr, 0.0, np, S));
        // stage 1: seeds dt lam_pre + dt/2 lam* (of L) and dt^2/6 lam_pre + dt^2/8 lam* (of L_t) at Q^n
        for (int v = 0; v < 4; ++v) {
            HIPCHK(c, launch_pad_to_int(B.mu0[v], B.lam_pre[v], dt, B.lam_star[v], 0.5 * dt, c->g, S));
            HIPCHK(c, launch_pad_to_int(B.mu1[v], B.lam_pre[v], dt * dt / 6.0, B.lam_star[v], dt * dt / 8.0, c->g, S));
            HIPCHK(c, launch_zero(B.acc[v], np, S));
        }
        for (int d = 0; d < 3; ++d) HIPCHK(c, launch_adj_direction(adj_args(c, B, d, qwork, exact), 1, S));
        const double* qw_d[4] = {B.qwork[0], B.qwork[1], B.qwork[2], B.qwork[3]};
        HIPCHK(c, launch_adj_fold(B.acc, c->g, c->cfg.bc, qw_d, c->cfg.u_in, c->c, c->cfg.rho_ref, S));
        // lam^n = lam_pre + lam* + J^T(...)
        for (int v = 0; v < 4; ++v) {
            HIPCHK(c, launch_axpby(B.lam[v], B.lam_pre[v], 1.0, B.lam_star[v], 1.0, np, S));
            HIPCHK(c, launch_axpby(B.lam[v], B.lam[v], 1.0, B.acc[v], 1.0, np, S));
        }
    }
    if (grad_q0) {
        const long long N = (long long)c->cfg.nx * c->cfg.ny * c->cfg.nz;
        for (int v = 0; v < 4; ++v) HIPCHK(c, launch_pad_to_int(grad_q0 + v * N, B.lam[v], 1.0, nullptr, 0.0, c->g, S));
    }
    HIPCHK(c, hipStreamSynchronize(S));
    return GKS_OK;
}

size_t gks_statistics_bytes(const gks_config* cfg) {
    if (!validate(cfg).empty()) return 0;
    return 9 * sizeof(double) * (size_t)cfg->nx * cfg->ny * cfg->nz;
}

int gks_set_statistics(gks_ctx* c, void* buffer, int32_t interval) {
    if (!c) return GKS_E_INVALID_ARG;
    if (buffer && interval < 1) return fail(c, GKS_E_INVALID_ARG, "interval must be >= 1");
    if (buffer && reinterpret_cast<uintptr_t>(buffer) % 8) return fail(c, GKS_E_INVALID_ARG, "statistics buffer must be 8-byte aligned");
    c->stats_buf = static_cast<double*>(buffer);
    c->stats_interval = buffer ? interval : 0;
    c->stats_n = 0;
    c->host_step = 0;
    if (buffer) {
        StatsArgs sa;
        sa.g = c->g;
        sa.rho_ref = c->cfg.rho_ref;
        sa.buf = c->stats_buf;
        HIPCHK(c, launch_stats_zero(sa, c->stream));
    }
    return GKS_OK;
}

int gks_read_statistics(gks_ctx* c, double u_inf, double* mean, double* rms, double* stress, double* tke,
                        int64_t* nsamples) {
    if (!c) return GKS_E_INVALID_ARG;
    if (!c->stats_buf) return fail(c, GKS_E_STATE, "statistics are not enabled (gks_set_statistics)");
    if (!(u_inf > 0)) return fail(c, GKS_E_INVALID_ARG, "u_inf must be > 0");
    if (nsamples) *nsamples = c->stats_n;
    if (c->stats_n == 0) return fail(c, GKS_E_STATE, "no samples yet");
    StatsArgs sa;
    sa.g = c->g;
    sa.rho_ref = c->cfg.rho_ref;
    sa.buf = c->stats_buf;
    HIPCHK(c, launch_stats_final(sa, 1.0 / (double)c->stats_n, 1.0 / (u_inf * u_inf), mean, rms, stress, tke, c->stream));
    return GKS_OK;
}

int gks_set_history(gks_ctx* c, double* buffer, int32_t capacity) {
    if (!c) return GKS_E_INVALID_ARG;
    if (buffer && capacity < 1) return fail(c, GKS_E_INVALID_ARG, "capacity must be >= 1");
    c->hist_buf = buffer;
    c->hist_cap = buffer ? capacity : 0;
    c->hist_n = 0;
    return GKS_OK;
}

int gks_history_count(gks_ctx* c, int64_t* count) {
    if (!c || !count) return GKS_E_INVALID_ARG;
    *count = c->hist_n;
    return GKS_OK;
}

int gks_set_timing(gks_ctx* c, int32_t enable) {
    if (!c) return GKS_E_INVALID_ARG;
    int rc = timing_flush(c);
    if (rc) return rc;
    c->timing = enable ? 1 : 0;
    for (int i = 0; i < GKS_TIMER_COUNT; ++i) {
        c->t_ms[i] = 0.0;
        c->t_cnt[i] = 0;
    }
    return GKS_OK;
}

int gks_read_timing(gks_ctx* c, double* ms, int64_t* count, int32_t n) {
    if (!c) return GKS_E_INVALID_ARG;
    if (n < 0 || n > GKS_TIMER_COUNT || (n > 0 && (!ms || !count))) return fail(c, GKS_E_INVALID_ARG, "bad timing arrays");
    int rc = timing_flush(c);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        ms[i] = c->t_ms[i];
        count[i] = c->t_cnt[i];
    }
    return GKS_OK;
}

int gks_init_static(const gks_config* cfg, gks_field q, gks_field q_stage, gks_field q_acc, void* hip_stream,
                    gks_ctx** out) {
    if (!out) return fail(nullptr, GKS_E_INVALID_ARG, "out is null");
    *out = nullptr;
    std::string why = validate(cfg);
    if (!why.empty()) return fail(nullptr, GKS_E_INVALID_ARG, why);
    Layout L;
    layout(cfg, nullptr, &L);
    if (L.total > GKS_STATIC_SCRATCH_BYTES)
        return fail(nullptr, GKS_E_INVALID_ARG,
                    "the configuration needs " + std::to_string(L.total) + " bytes of workspace; the static scratch holds " +
                        std::to_string((size_t)GKS_STATIC_SCRATCH_BYTES) + " (use gks_init with a caller workspace)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, GKS_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kStaticDevices) return fail(nullptr, GKS_E_UNSUPPORTED, "device index beyond the static slots");
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticSlot& slot = g_static[dev];
    if (slot.owner)
        return fail(nullptr, GKS_E_STATE, "another context holds this GPU's static scratch (gks_destroy it first)");
    if (!slot.ptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, GKS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        slot.ptr = p;
    }
    gks_ctx* c = nullptr;
    const int rc = gks_init(cfg, q, q_stage, q_acc, slot.ptr, GKS_STATIC_SCRATCH_BYTES, hip_stream, &c);
    if (rc != GKS_OK) return rc;
    c->static_dev = dev;
    slot.owner = c;
    *out = c;
    return GKS_OK;
}

void gks_destroy(gks_ctx* c) {
    if (!c) return;
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static[c->static_dev].owner == c) g_static[c->static_dev].owner = nullptr;
    }
    delete c;
}

const char* gks_last_error(const gks_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
