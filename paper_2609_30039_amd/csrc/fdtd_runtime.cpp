// fdtd_runtime.cpp -- host runtime and C-ABI of libfdtd.
//
// Owns the device memory of a handle (one pooled hipMalloc planned and
// admitted before allocation), the absorber and dispersion coefficient tables,
// the monitor ring buffers, the checkpoint slots, and the step bookkeeping of
// the forward sweep and of the reverse (adjoint) sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "fdtd.h"
#include "fdtd_dev.h"
#include "fdtd_launch.h"

using namespace fdtd;

namespace {

thread_local std::string g_create_error;

struct Err {
    int code;
    std::string msg;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- CPML tables
// Roden-Gedney recursive convolution along one axis (Section 2.2).  Node i is
// at x = i for E-update derivatives and x = i + 1/2 for H-update derivatives;
// depth d in [0,1] from the interface (0) to the outer wall (1);
// sigma = smax d^m, kappa = 1 + (kmax-1) d^m, alpha = amax (1-d);
// b = exp(-(sigma/kappa + alpha) dt), c = sigma (b-1) / (sigma kappa + kappa^2 alpha).
void cpml_tables(int n, int l0, int l1, double S, double m, double kmax, double smax, double amax,
                 std::vector<double>& out /* 6*n: bE cE kiE bH cH kiH */) {
    out.assign(6 * (size_t)n, 0.0);
    for (int half = 0; half < 2; ++half) {
        double* b = out.data() + (size_t)(3 * half + 0) * n;
        double* c = out.data() + (size_t)(3 * half + 1) * n;
        double* ki = out.data() + (size_t)(3 * half + 2) * n;
        for (int i = 0; i < n; ++i) {
            b[i] = 1.0;
            c[i] = 0.0;
            ki[i] = 1.0;
            double x = i + (half ? 0.5 : 0.0);
            double d;
            if (l0 > 0 && i < l0) d = std::max(0.0, (l0 - x) / l0);
            else if (l1 > 0 && i >= n - l1) d = std::max(0.0, (x - (n - l1)) / l1);
            else continue;
            double dm = std::pow(d, m);
            double sig = smax * dm, kap = 1.0 + (kmax - 1.0) * dm, alp = amax * (1.0 - d);
            b[i] = std::exp(-(sig / kap + alp) * S);
            c[i] = sig > 0 ? sig * (b[i] - 1.0) / (sig * kap + kap * kap * alp) : 0.0;
            ki[i] = 1.0 / kap;
        }
    }
}

struct MonHost {
    MonDev dev{};
    int npts = 0;
    size_t acc_elems = 0;   // doubles in acc (and cot)
    int pending = 0, n0 = 0;
    bool cot_set = false;
    std::vector<double> omega;
};

struct DomHost {
    fdtd_domain_desc desc{};
    std::vector<double> eps;                 // host copy
    std::vector<std::vector<double>> waves;
    std::vector<MonHost> mons;
    int ncomp_eps = 1;
    size_t nfield = 0;                       // elements per field array (pitch*ny*nz)
    int gncomp = 0;
    size_t gelems = 0;                       // per component
    size_t rec_step = 0;                     // reversible mode: recorded interface elements per step
};

struct StateArr {
    void* p;                                 // set-0 address
    size_t n;                                // elements
};

struct Slot {
    bool valid = false;
    int step = 0;
    unsigned long long sum = 0;
};

struct Base {
    virtual ~Base() = default;
    std::string err;
    bool poisoned = false;
    virtual int step_forward(int n, unsigned flags) = 0;
    virtual int adjoint_begin(int n) = 0;
    virtual int step_adjoint(int n) = 0;
    virtual int step_reverse(int n) = 0;
    virtual int ckpt_save(int slot) = 0;
    virtual int ckpt_restore(int slot) = 0;
    virtual int monitor(int dom, int mon, int op, void* buf, size_t bytes) = 0;
    virtual int get_field(int dom, int comp, void* buf, size_t bytes, bool set) = 0;
    virtual int get_grad(int dom, double* buf, size_t bytes) = 0;
    virtual int set_eps(int dom, const double* eps, size_t bytes) = 0;
    virtual int reset() = 0;
    virtual void steps(int* n, int* m) = 0;
    virtual double memory() = 0;
    virtual int timing(int op, double* ms, long long* n) = 0;
    virtual int poke_slot(int slot, size_t word, unsigned int value) = 0;
    virtual int energy(int dom, double* out) = 0;
    virtual int probe_trace(int dom, int mon, double* buf, int n) = 0;
};

// Bump allocator over one arena of the pool; with assign=false it only sizes.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    bool assign = false;
    template <typename P>
    void take(P*& p, size_t bytes) {
        off = align256(off);
        if (assign) p = (P*)(base + off);
        off += std::max<size_t>(bytes, 1);
    }
};

// ------------------------------------------------------------ tensor media
// Entries of a symmetric 3x3 tensor in the descriptor's order: xx yy zz xy xz yz.
static inline int sym_idx(int a, int b) {
    if (a == b) return a;
    const int lo = std::min(a, b), hi = std::max(a, b);
    return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

// Eigenvalues (ascending) of a symmetric 3x3 tensor by the trigonometric
// solution of its characteristic cubic (O. K. Smith, Commun. ACM 4(4), 1961).
static void sym3_eigenvalues(const double m[6], double w[3]) {
    const double off = m[3] * m[3] + m[4] * m[4] + m[5] * m[5];
    const double q = (m[0] + m[1] + m[2]) / 3.0;
    if (off == 0.0) {
        w[0] = m[0];
        w[1] = m[1];
        w[2] = m[2];
        std::sort(w, w + 3);
        return;
    }
    const double p2 = (m[0] - q) * (m[0] - q) + (m[1] - q) * (m[1] - q) + (m[2] - q) * (m[2] - q) + 2.0 * off;
    const double p = std::sqrt(p2 / 6.0);
    // B = (A - q I) / p; r = det(B) / 2 in [-1, 1]
    const double b0 = (m[0] - q) / p, b1 = (m[1] - q) / p, b2 = (m[2] - q) / p;
    const double b3 = m[3] / p, b4 = m[4] / p, b5 = m[5] / p;
    double r = 0.5 * (b0 * (b1 * b2 - b5 * b5) - b3 * (b3 * b2 - b5 * b4) + b4 * (b3 * b5 - b1 * b4));
    r = std::min(1.0, std::max(-1.0, r));
    const double phi = std::acos(r) / 3.0;
    const double hi = q + 2.0 * p * std::cos(phi);
    const double lo = q + 2.0 * p * std::cos(phi + 2.0 * std::acos(-1.0) / 3.0);
    w[0] = lo;
    w[2] = hi;
    w[1] = 3.0 * q - lo - hi;
}

// Section 2.3 admission of one node's tensor: finite, every eigenvalue >= 1
// (the vacuum step bound of Eq. 2 holds), and inside the absorbing face of
// normal a the normal is a principal axis whose eigenvalue is the largest or
// the smallest.  Returns nullptr when admitted.
static const char* tensor_node_check(const double m[6], const bool inface[3]) {
    double scale = 0.0;
    for (int q = 0; q < 6; ++q) {
        if (!std::isfinite(m[q])) return "tensor permittivity must be finite";
        scale = std::max(scale, std::fabs(m[q]));
    }
    const double tol = 1e-12 * std::max(1.0, scale);
    double w[3];
    sym3_eigenvalues(m, w);
    if (!(w[0] >= 1.0 - tol)) return "tensor permittivity needs every eigenvalue at least 1";
    for (int a = 0; a < 3; ++a) {
        if (!inface[a]) continue;
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        if (std::fabs(m[sym_idx(a, b)]) > tol || std::fabs(m[sym_idx(a, c)]) > tol)
            return "tensor in an absorbing face with principal axes rotated against the face normal";
        // eigenvalues of the transverse block
        const double p = m[b], r = m[c], o = m[sym_idx(b, c)];
        const double mid = 0.5 * (p + r), rad = std::sqrt(0.25 * (p - r) * (p - r) + o * o);
        if (m[a] > mid - rad + tol && m[a] < mid + rad - tol)
            return "tensor in an absorbing face with intermediate normal eigenvalue";
    }
    return nullptr;
}

// inverse of a symmetric positive-definite 3x3 tensor (cofactors over the determinant)
static void sym3_inverse(const double m[6], double out[6]) {
    const double xx = m[0], yy = m[1], zz = m[2], xy = m[3], xz = m[4], yz = m[5];
    const double cxx = yy * zz - yz * yz, cyy = xx * zz - xz * xz, czz = xx * yy - xy * xy;
    const double cxy = xz * yz - xy * zz, cxz = xy * yz - xz * yy, cyz = xy * xz - xx * yz;
    const double det = xx * cxx + xy * cxy + xz * cxz;
    out[0] = cxx / det;
    out[1] = cyy / det;
    out[2] = czz / det;
    out[3] = cxy / det;
    out[4] = cxz / det;
    out[5] = cyz / det;
}

template <typename T>
struct Handle : Base {
    hipStream_t st = nullptr;
    fdtd_options opt{};
    int ndom = 0;
    std::vector<DomHost> dh;
    std::vector<DomDev<T>> dd;
    DomDev<T>* d_doms = nullptr;
    int* d_bs = nullptr;
    LaunchCfg cfg{};
    std::vector<int> bs_host;   // [0, ndom]: split blocks; [ndom+1, 2 ndom+1]: Lorentz-box blocks
    std::vector<int4> tiles_gen, tiles_bulk, tiles_fgen, tiles_fcp, tiles_fplain;
    int4* d_tiles = nullptr;
    // tile tables of the split adjoint: E-node pass 6 classes, H-node pass 5
    // classes (LaunchCfg::ta1, ta2)
    std::vector<int4> atiles[kAdjClasses1 + kAdjClasses2];
    std::vector<int4> atab1, atab2;   // the tables uploaded: E-node pass, H-node pass
    int4* d_atiles = nullptr;
    // pool: [misc][forward sets x nsets][adjoint sets x 2][split scratch][bf16 slots]
    char* pool = nullptr;
    size_t pool_bytes = 0, misc_bytes = 0, fstride = 0, astride = 0, et_bytes = 0, bfslot = 0;
    int nsets = 2;
    char *fbase = nullptr, *abase = nullptr, *etbase = nullptr, *bfbase = nullptr;
    std::vector<Slot> slots;
    unsigned int* d_scales = nullptr;         // [n_ckpt][n_state] BF16 scales
    std::vector<BfArr> bfarr;                 // BF16 table: one entry per forward state array
    BfArr* d_bfarr = nullptr;
    float* d_bfpart = nullptr;                // per-chunk maxima of a save
    int bfblocks = 0;
    unsigned long long* d_sum = nullptr;      // checksum scratch
    double* d_energy = nullptr;               // watchdog: kEnergyBlocks partial sums, then the sum
    std::vector<StateArr> fwd, adj;           // state arrays (set-0 addresses)
    std::vector<std::pair<void*, size_t>> adj_flat;   // gradient accumulators, for zeroing
    // physical forward sets: two working sets and one per full-precision slot
    int wset[2] = {0, 1};
    std::vector<int> slotset;
    int cur = 0;                               // set holding the current forward state
    int ap = 0, t = 0, m = -1;
    int dft_block = 32;
    bool bf16 = false;
    // captured step chunks (graph_chunk > 0): the kernels read the step index
    // from d_tstep, which the replay advances; keyed by (record, current set)
    int* d_tstep = nullptr;
    int tstep_val = -1;                        // value d_tstep holds after the queued work (-1: unknown)
    hipStream_t cst = nullptr;                 // capture stream
    struct GraphEx {
        int key;
        hipGraph_t g;
        hipGraphExec_t ex;
    };
    std::vector<GraphEx> graphs;
    // reversible mode: record slots [rec_lo, rec_hi] hold the interface of the
    // current trajectory (-1: none)
    int rec_lo = -1, rec_hi = -1, rev_maxcnt = 0;
    long long rev_maxcells = 0;
    // kernel timing
    bool timing_on = false;
    std::vector<hipEvent_t> evs;
    size_t nev = 0;
    // use by the streamed executor: size_only stops create() once the pool
    // size is known; ext_pool (ext_cap bytes) replaces the allocation and is
    // not freed; external_eps: the caller uploads eps^-1 itself (a slab cut
    // from an admitted domain), so create() neither checks nor keeps eps
    bool size_only = false, external_eps = false;
    char* ext_pool = nullptr;
    size_t ext_cap = 0;

    ~Handle() override {
        if (!pool) return;   // nothing was allocated (e.g. refused at admission)
        if (st) (void)hipStreamSynchronize(st);
        else (void)hipDeviceSynchronize();
        for (auto e : evs) (void)hipEventDestroy(e);
        for (auto& g : graphs) {
            (void)hipGraphExecDestroy(g.ex);
            (void)hipGraphDestroy(g.g);
        }
        if (cst) (void)hipStreamDestroy(cst);
        if (ext_pool) return;
        if (opt.alloc) opt.release(opt.alloc_ctx, pool);
        else (void)hipFree(pool);
    }

    int fail(int code, const std::string& msg) {
        err = msg;
        if (code == FDTD_E_DEVICE) poisoned = true;
        return code;
    }

    int check(const char* what) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(FDTD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return FDTD_OK;
    }

    int sync(const char* what) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(FDTD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return check(what);
    }

    char* set_ptr(int q) { return fbase + (size_t)q * fstride; }

    // ------------------------------------------------------------ tiles
    // Split kernels: prefix sums of 64 x 4 column blocks per domain.  Fused
    // kernels: tiles of 64 x-columns (62 owned) by 4R rows (4R - 2 owned) by
    // kz planes, listed as bulk when they lie inside the domain away from
    // PEC nodes, absorbers, the Lorentz box and sources, general otherwise.
    void build_tiles() {
        bs_host.assign(2 * (ndom + 1) + 16, 0);   // [bs][lbs][per-XCD run starts, lengths]
        int* lbs = bs_host.data() + ndom + 1;
        tiles_gen.clear();
        tiles_bulk.clear();
        tiles_fgen.clear();
        tiles_fcp.clear();
        tiles_fplain.clear();
        const int R = cfg.rows, NR = kFusedWaves * R, TYo = NR - 2, kz = cfg.kz;
        for (int q = 0; q < ndom; ++q) {
            const fdtd_domain_desc& s = dh[q].desc;
            const int nx = s.n[0], ny = s.n[1], nz = s.n[2];
            bs_host[q + 1] = bs_host[q] + split_blocks(nx, ny, nz, kz, cfg.sw);
            long long nl = 0;
            if (s.n_lorentz) {
                const fdtd_lorentz_desc& L = s.lorentz;
                nl = (long long)(L.hi[0] - L.lo[0]) * (L.hi[1] - L.lo[1]) * (L.hi[2] - L.lo[2]);
            }
            lbs[q + 1] = lbs[q] + (int)((nl + 255) / 256);
            if (cfg.kernel == 1) continue;
            for (int bz = 0; bz * kz < nz; ++bz)
                for (int by = 0; by * TYo < ny; ++by)
                    for (int bx = 0; bx * 62 < nx; ++bx) {
                        int X0 = bx * 62 - 1, Y0 = by * TYo - 1, k0 = bz * kz, k1 = std::min(k0 + kz, nz);
                        int lo[3] = {X0, Y0, k0 - 1}, hi[3] = {X0 + 63, Y0 + NR - 1, k1};
                        bool lor = false;
                        if (s.n_lorentz) {
                            const fdtd_lorentz_desc& L = s.lorentz;
                            lor = true;
                            for (int a = 0; a < 3; ++a)
                                if (hi[a] < L.lo[a] || lo[a] >= L.hi[a]) lor = false;
                        }
                        bool cp = false;
                        for (int a = 0; a < 3; ++a)
                            if ((s.pml[2 * a] > 0 && lo[a] < s.pml[2 * a]) ||
                                (s.pml[2 * a + 1] > 0 && hi[a] >= s.n[a] - s.pml[2 * a + 1]))
                                cp = true;
                        (lor ? tiles_fgen : (cp ? tiles_fcp : tiles_fplain)).push_back(make_int4(q, X0, Y0, k0));
                        bool bulk = X0 >= 1 && hi[0] <= nx - 1 && Y0 >= 1 && hi[1] <= ny - 1 && k0 >= 1 &&
                                    k1 <= nz - 1;
                        for (int a = 0; a < 3 && bulk; ++a)
                            if (lo[a] < s.pml[2 * a] || hi[a] >= s.n[a] - s.pml[2 * a + 1]) bulk = false;
                        if (bulk && s.n_lorentz) {
                            const fdtd_lorentz_desc& L = s.lorentz;
                            bool meet = true;
                            for (int a = 0; a < 3; ++a)
                                if (hi[a] < L.lo[a] || lo[a] >= L.hi[a]) meet = false;
                            if (meet) bulk = false;
                        }
                        for (int k = 0; k < s.n_sources && bulk; ++k) {
                            const fdtd_source_desc& sr = s.sources[k];
                            bool zin = sr.pos[2] >= lo[2] && sr.pos[2] <= hi[2];
                            bool xyin = sr.kind == FDTD_SRC_PLANE_Z ||
                                        (sr.pos[0] >= lo[0] && sr.pos[0] <= hi[0] && sr.pos[1] >= lo[1] &&
                                         sr.pos[1] <= hi[1]);
                            if (zin && xyin) bulk = false;
                        }
                        (bulk ? tiles_bulk : tiles_gen).push_back(make_int4(q, X0, Y0, k0));
                    }
        }
        cfg.nblk = bs_host[ndom];
        cfg.nlor = lbs[ndom];
        cfg.ntens = cfg.ntper = 0;
        for (int q = 0; q < ndom; ++q) {
            cfg.ntens += dd[q].tens;
            cfg.ntper += dd[q].tens && (dd[q].per[0] || dd[q].per[1]);
        }
        if (cfg.kernel == 1) split_runs();
        build_adjoint_tiles();
        cfg.ngen = (int)tiles_gen.size();
        cfg.nbulk = (int)tiles_bulk.size();
        cfg.nfgen = (int)tiles_fgen.size();
        cfg.nfcp = (int)tiles_fcp.size();
        cfg.nfplain = (int)tiles_fplain.size();
    }

    // Tiles of the split adjoint.  Along x each domain is cut into a low slab
    // zone, an interior zone and a high slab zone; the E-node pass (which reads
    // the memory one step back) widens the low zone by one column, the H-node
    // pass (one step forward) the high zone.  Slab zones take narrow tiles (16
    // columns by 16 rows), the interior zone wide ones (32 by 8) from its first
    // 32-column boundary on (narrow tiles cover the columns before it).  Per axis a,
    // a tile needs the a-slab memory cotangents if a node it updates, or the
    // neighbour it reads along a, lies in an a-slab; it goes to the narrowest
    // class whose mask covers that.  E-node tiles holding Lorentz cells or
    // gradient cells inside a slab take the general class.  The kernels rely
    // on this: a class only handles the slabs its mask names.
    void build_adjoint_tiles() {
        for (auto& l : atiles) l.clear();
        const int kz = cfg.kz;
        for (int q = 0; q < ndom; ++q) {
            const fdtd_domain_desc& s = dh[q].desc;
            if (!s.grad) continue;
            // a periodic domain's adjoint has launches of its own (launch_per_adj)
            if (s.periodic[0] || s.periodic[1] || s.periodic[2]) continue;
            const int n[3] = {s.n[0], s.n[1], s.n[2]};
            for (int pass = 0; pass < 2; ++pass) {
                // a tensor domain's E-node work has launches of its own (launch_tens_adj)
                if (pass == 0 && s.eps_kind == FDTD_EPS_TENSOR) continue;
                const int L0 = s.pml[0], L1 = s.pml[1];
                const int xa = L0 > 0 ? std::min(L0 + (pass == 0 ? 1 : 0), n[0]) : 0;
                const int xb = L1 > 0 ? std::max(n[0] - L1 - (pass == 1 ? 1 : 0), xa) : n[0];
                // wide tiles start on a 32-column (128 B) boundary: a wave's row
                // then spans two cache lines; narrow tiles take the columns before
                const int wa = std::min((xa + 31) / 32 * 32, xb);
                const int zlo[3] = {0, wa, xb}, zhi[3] = {wa, xb, n[0]};
                for (int zone = 0; zone < 3; ++zone) {
                    const bool wide = zone == 1;
                    const int W = wide ? 32 : 16, rows = 256 / W;
                    for (int x0 = zlo[zone]; x0 < zhi[zone]; x0 += W)
                        for (int y0 = 0; y0 < n[1]; y0 += rows)
                            for (int k0 = 0; k0 < n[2]; k0 += kz) {
                                const int xlen = std::min(W, zhi[zone] - x0);
                                const int lo[3] = {x0, y0, k0};
                                const int hi[3] = {x0 + xlen - 1, std::min(y0 + rows, n[1]) - 1,
                                                   std::min(k0 + kz, n[2]) - 1};
                                int mask = 0;
                                for (int a = 0; a < 3; ++a) {
                                    const int A0 = s.pml[2 * a], A1 = s.pml[2 * a + 1];
                                    bool need = lo[a] < A0 || hi[a] >= n[a] - A1;
                                    if (pass == 0 && lo[a] > 0 && lo[a] - 1 < A0) need = true;
                                    if (pass == 1 && A1 > 0 && hi[a] + 1 < n[a] && hi[a] + 1 >= n[a] - A1) need = true;
                                    if (need) mask |= 1 << a;
                                }
                                bool general = false;
                                if (pass == 0) {
                                    if (s.n_lorentz) {
                                        bool meet = true;
                                        for (int a = 0; a < 3; ++a)
                                            if (hi[a] < s.lorentz.lo[a] || lo[a] >= s.lorentz.hi[a]) meet = false;
                                        general = meet;
                                    }
                                    int glo[3], ghi[3];
                                    bool meet = true;
                                    for (int a = 0; a < 3; ++a) {
                                        glo[a] = std::max(lo[a], s.grad_lo[a]);
                                        ghi[a] = std::min(hi[a], s.grad_hi[a] - 1);
                                        if (glo[a] > ghi[a]) meet = false;
                                    }
                                    for (int a = 0; a < 3 && meet; ++a)
                                        if (glo[a] < s.pml[2 * a] || ghi[a] >= n[a] - s.pml[2 * a + 1]) general = true;
                                }
                                int cls;
                                if (pass == 0) {
                                    if (wide) cls = general || (mask & 1) ? 2 : mask ? 1 : 0;
                                    else cls = general ? 5 : !(mask & 1) ? 6 : (mask & ~1) ? 4 : 3;
                                } else {
                                    if (wide) cls = (mask & 1) ? 2 : mask ? 1 : 0;
                                    else cls = !(mask & 1) ? 5 : (mask & ~1) ? 4 : 3;
                                    cls += kAdjClasses1;
                                }
                                const int c = pass == 0 ? cls : cls - kAdjClasses1;
                                atiles[cls].push_back(make_int4(q | (c << 24), x0 | (xlen << 24), y0, k0));
                            }
                }
            }
        }
        // One table per pass.  The general classes of the E-node pass lead (a
        // launch of their own).  Every other tile goes, in spatial order
        // (domain, z chunk, 16-row band, x, y), to one of the 8 XCDs: the
        // order is cut into 8 contiguous runs of equal estimated cost (slab
        // tiles count 1.75 times an interior tile), and the runs are
        // interleaved so that workgroup b, which the dispatcher sends to XCD
        // b % 8, takes the next tile of run b % 8 (short runs are padded with
        // empty tiles).  Tiles that share cache lines (a narrow tile and its x
        // neighbour cover the two halves of a 128 B line) and halo rows and
        // planes then run on one XCD, close in time, sharing its L2, and no
        // XCD is left with the slab-heavy ends of the domain alone.
        auto xcd_runs = [&](std::vector<int4>& v) {
            std::stable_sort(v.begin(), v.end(), [](const int4& a, const int4& b) {
                const long long ka[5] = {a.x & 0xFFFFFF, a.w, a.z >> 4, a.y & 0xFFFFFF, a.z};
                const long long kb[5] = {b.x & 0xFFFFFF, b.w, b.z >> 4, b.y & 0xFFFFFF, b.z};
                return std::lexicographical_compare(ka, ka + 5, kb, kb + 5);
            });
            constexpr int X = 8;
            std::vector<double> cost(v.size());
            double total = 0;
            for (size_t t = 0; t < v.size(); ++t) {
                const int4 e = v[t];
                const fdtd_domain_desc& s = dh[e.x & 0xFFFFFF].desc;
                const int cls = e.x >> 24, rows = cls < 3 ? 8 : 16;   // classes 0-2: 32 x 8 tiles, others 16 x 16
                const double cells = (double)(e.y >> 24) * std::min(rows, s.n[1] - e.z) * std::min(kz, s.n[2] - e.w);
                cost[t] = cells * (cls == 0 ? 1.0 : 1.75);
                total += cost[t];
            }
            std::vector<int4> run[X];
            double acc = 0;
            for (size_t t = 0; t < v.size(); ++t) {
                const int x = std::min(X - 1, (int)((acc + 0.5 * cost[t]) / std::max(total, 1e-30) * X));
                run[x].push_back(v[t]);
                acc += cost[t];
            }
            size_t len = 0;
            for (auto& r : run) len = std::max(len, r.size());
            std::vector<int4> out(len * X);
            for (size_t m = 0; m < len; ++m)
                for (int x = 0; x < X; ++x)
                    out[m * X + x] = m < run[x].size() ? run[x][m]
                                                       : make_int4(v.empty() ? 0 : (v[0].x & 0xFFFFFF), 0, 0, 0);
            v.swap(out);
        };
        atab1.clear();
        atab2.clear();
        for (int c : {5, 2}) atab1.insert(atab1.end(), atiles[c].begin(), atiles[c].end());
        std::vector<int4> rest;
        for (int c : {0, 1, 3, 4, 6}) rest.insert(rest.end(), atiles[c].begin(), atiles[c].end());
        xcd_runs(rest);
        atab1.insert(atab1.end(), rest.begin(), rest.end());
        for (int c = 0; c < kAdjClasses2; ++c)
            atab2.insert(atab2.end(), atiles[kAdjClasses1 + c].begin(), atiles[kAdjClasses1 + c].end());
        xcd_runs(atab2);
        static_assert(kAdjClasses1 == 7, "the general classes 2 and 5 lead the E-node table");
        cfg.na1 = (int)atab1.size();
        cfg.na1g = (int)(atiles[5].size() + atiles[2].size());   // order1 starts with the general classes
        cfg.na2 = (int)atab2.size();
    }

    // Split column blocks in their numbering (domain by domain, x fastest, then
    // rows, then z chunks) cut into 8 contiguous runs of equal estimated cost,
    // one per XCD: a block meeting an absorbing slab counts twice its cells
    // (it also moves the memories).  Contiguous runs keep neighbouring
    // columns and planes on one L2; equal cost keeps the XCDs holding the
    // slab-heavy ends of the domain from finishing last.
    void split_runs() {
        const int W = cfg.sw, NR = 256 / W, kz = cfg.kz, nb = cfg.nblk;
        std::vector<double> cost(nb);
        double total = 0;
        int b = 0;
        for (int q = 0; q < ndom; ++q) {
            const fdtd_domain_desc& s = dh[q].desc;
            const int nbx = (s.n[0] + W - 1) / W, nby = (s.n[1] + NR - 1) / NR, nbz = (s.n[2] + kz - 1) / kz;
            for (int bz = 0; bz < nbz; ++bz)
                for (int by = 0; by < nby; ++by)
                    for (int bx = 0; bx < nbx; ++bx, ++b) {
                        const int lo[3] = {bx * W, by * NR, bz * kz};
                        const int hi[3] = {std::min(lo[0] + W, s.n[0]) - 1, std::min(lo[1] + NR, s.n[1]) - 1,
                                           std::min(lo[2] + kz, s.n[2]) - 1};
                        bool cp = false;
                        for (int a = 0; a < 3; ++a)
                            if (lo[a] < s.pml[2 * a] || hi[a] >= s.n[a] - s.pml[2 * a + 1]) cp = true;
                        const double cells = (double)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
                        cost[b] = cells * (cp ? 2.0 : 1.0);
                        total += cost[b];
                    }
        }
        int* xs = bs_host.data() + 2 * (ndom + 1);
        int* xl = xs + 8;
        for (int x = 0; x < 8; ++x) xs[x] = xl[x] = 0;
        double acc = 0;
        int prev = -1;
        for (int t = 0; t < nb; ++t) {
            const int x = std::min(7, (int)((acc + 0.5 * cost[t]) / std::max(total, 1e-30) * 8));
            if (x != prev) {
                xs[x] = t;
                prev = x;
            }
            xl[x]++;
            acc += cost[t];
        }
        int len = 0;
        for (int x = 0; x < 8; ++x) len = std::max(len, xl[x]);
        cfg.ngrid = 8 * len;
    }

    // ------------------------------------------------------------ layout
    // Places every array in its arena.  Forward state arrays of all domains form
    // one set (stride fstride), adjoint arrays one adjoint set (astride).
    void layout(Arena& M, Arena& F, Arena& A, Arena& X) {
        const bool asg = M.assign;
        if (asg) {
            fwd.clear();
            adj.clear();
            adj_flat.clear();
        }
        bfslot = 0;
        bfblocks = 0;
        if (asg) bfarr.clear();
        size_t nstate = 0;
        const size_t ts = sizeof(T);
        for (int q = 0; q < ndom; ++q) {
            DomHost& h = dh[q];
            DomDev<T>& d = dd[q];
            const fdtd_domain_desc& s = h.desc;
            const int nx = s.n[0], ny = s.n[1], nz = s.n[2];
            const bool g = s.grad != 0;
            auto fst = [&](T*& p, size_t n) {
                F.take(p, n * ts);
                const int nb = (int)((n + kBfChunk - 1) / kBfChunk);
                if (asg) {
                    fwd.push_back(StateArr{p, n});
                    bfarr.push_back(BfArr{p, (long long)n, (long long)bfslot, bfblocks, nb});
                }
                bfslot += align256(n * 2);
                bfblocks += nb;
                nstate++;
            };
            auto ast = [&](T*& p, size_t n) {
                A.take(p, n * ts);
                if (asg) adj.push_back(StateArr{p, n});
            };
            for (int c = 0; c < 3; ++c) {
                fst(d.E[c], h.nfield);
                fst(d.H[c], h.nfield);
            }
            for (int a = 0; a < 3; ++a) M.take(d.tab[a], 6 * (size_t)s.n[a] * ts);
            for (int a = 0; a < 3; ++a)
                for (int side = 0; side < 2; ++side) {
                    size_t L = (size_t)s.pml[2 * a + side];
                    size_t ne = a == 0 ? L * ny * nz : (a == 1 ? L * nx * nz : L * nx * ny);
                    for (int r = 0; r < 2; ++r) {
                        if (!ne) continue;
                        fst(d.psiE[a][side][r], ne);
                        fst(d.psiH[a][side][r], ne);
                        if (g) {
                            ast(d.psiEa[a][side][r], ne);
                            ast(d.psiHa[a][side][r], ne);
                        }
                    }
                }
            size_t ebox = 1;
            for (int a = 0; a < 3; ++a) ebox *= (size_t)(d.ehi[a] - d.elo[a]);
            const size_t erows = ebox ? ebox / (size_t)(d.ehi[0] - d.elo[0]) * d.exs : 0;   // stored elements
            if (d.tens) {
                if (ebox && s.eps)
                    for (int q6 = 0; q6 < 6; ++q6) M.take(d.tinv[q6], erows * ts);
                for (int c = 0; c < 3; ++c) X.take(d.curl[c], h.nfield * ts);
            } else if (ebox && s.eps) {
                for (int c = 0; c < h.ncomp_eps; ++c) M.take(d.epsinv[c], erows * ts);
                if (asg)
                    for (int c = h.ncomp_eps; c < 3; ++c) d.epsinv[c] = d.epsinv[0];
            }
            if (d.has_lor) {
                size_t lbox = 1;
                for (int a = 0; a < 3; ++a) lbox *= (size_t)(d.lhi[a] - d.llo[a]);
                // [0] E^{n-1}; [1] W^n and [2] W^{n-1} of every pole, pole p at + p * lbox
                for (int w = 0; w < 3; ++w)
                    for (int c = 0; c < 3; ++c) {
                        const size_t n = lbox * (w == 0 ? 1 : (size_t)d.npole);
                        fst(d.lor[w][c], n);
                        if (g) ast(d.lora[w][c], n);
                    }
            }
            for (int k = 0; k < s.n_sources; ++k)
                M.take(d.src[k].wave, (size_t)std::max(1, s.sources[k].n_waveform) * ts);
            if (d.rev) M.take(d.rec, h.rec_step * ((size_t)opt.max_steps + 1) * ts);
            if (g) {
                for (int c = 0; c < 3; ++c) {
                    ast(d.Ea[c], h.nfield);
                    ast(d.Ha[c], h.nfield);
                }
                if (cfg.kernel == 1)
                    for (int c = 0; c < 3; ++c) X.take(d.Et[c], h.nfield * ts);
                for (int c = 0; c < h.gncomp; ++c) {
                    size_t nb = std::max<size_t>(h.gelems, 1) * 8;
                    M.take(d.gacc[c], nb);
                    if (asg) adj_flat.push_back({d.gacc[c], nb});
                }
            }
            for (auto& mh : h.mons) {
                MonDev& md = mh.dev;
                M.take(md.omega, std::max(1, md.nf) * 8);
                if (md.kind == 0) {
                    M.take(md.trace, std::max(1, opt.max_steps) * 8);
                    md.ntrace = std::max(1, opt.max_steps);
                    M.take(md.cot, std::max(1, opt.max_steps) * 8);
                } else {
                    M.take(md.samples, (size_t)dft_block * md.rcomp * mh.npts * ts);
                    M.take(md.acc, mh.acc_elems * 8);
                    M.take(md.cot, mh.acc_elems * 8);
                    if (md.kind == 1) {
                        M.take(md.fpart, (size_t)md.nf * flux_blocks(mh.npts) * 8);
                        M.take(md.fout, (size_t)md.nf * 8);
                    }
                }
            }
            if (asg) {   // plane monitors as the split H kernel samples them
                d.nsmp = 0;
                for (auto& mh : h.mons) {
                    const MonDev& md = mh.dev;
                    if (md.kind == 0) continue;
                    SmpDev& sm = d.smp[d.nsmp++];
                    sm.kind = md.kind;
                    sm.comp = md.comp;
                    sm.i0 = md.i0;
                    sm.i1 = md.i1;
                    sm.j0 = md.j0;
                    sm.j1 = md.j1;
                    sm.k = md.k;
                    sm.npts = mh.npts;
                    sm.rcomp = md.rcomp;
                    sm.ring = md.samples;
                }
            }
        }
        M.take(d_doms, sizeof(DomDev<T>) * ndom);
        M.take(d_bs, sizeof(int) * (2 * (ndom + 1) + 16));
        M.take(d_tstep, sizeof(int));
        M.take(d_atiles, sizeof(int4) * std::max<size_t>(1, atab1.size() + atab2.size()));
        M.take(d_tiles, sizeof(int4) * std::max<size_t>(1, tiles_gen.size() + tiles_bulk.size() + tiles_fgen.size() +
                                                               tiles_fcp.size() + tiles_fplain.size()));
        M.take(d_scales, std::max<size_t>(1, (size_t)opt.n_ckpt * nstate) * 4);
        M.take(d_bfarr, std::max<size_t>(1, nstate) * sizeof(BfArr));
        M.take(d_bfpart, std::max<size_t>(1, (size_t)bfblocks) * 4);
        M.take(d_sum, 8);
        M.take(d_energy, (kEnergyBlocks + 1) * 8);
    }

    // ------------------------------------------------------------ create
    int create(const fdtd_domain_desc* doms, int n, const fdtd_options* o) {
        opt = *o;
        st = (hipStream_t)o->stream;
        ndom = n;
        dft_block = o->dft_block > 0 ? std::min(o->dft_block, kMaxDftBlock) : 32;
        if (o->graph_chunk < 0 || o->graph_chunk > kMaxDftBlock)
            return fail(FDTD_E_INVALID, "graph_chunk must be in [0, 64]");
        // a captured chunk ends with the spectrum update of its samples
        if (o->graph_chunk > 0) dft_block = o->graph_chunk;
        bf16 = o->ckpt_storage == FDTD_BF16;
        if (bf16 && sizeof(T) != 4) return fail(FDTD_E_INVALID, "BF16 checkpoints need FP32 fields");
        if (o->n_ckpt < 0 || o->max_steps < 0) return fail(FDTD_E_INVALID, "negative n_ckpt or max_steps");
        if (o->kernel < 0 || o->kernel > 3) return fail(FDTD_E_INVALID, "kernel selector");
        if (o->kernel == FDTD_KERNEL_ONEPASS && o->reversible)
            return fail(FDTD_E_INVALID, "the single-pass family takes no reversible mode");
        if (o->tile_rows != 0 && o->tile_rows != 2 && o->tile_rows != 4 && o->tile_rows != 8)
            return fail(FDTD_E_INVALID, "tile_rows must be 2, 4 or 8");
        if (o->tile_kz < 0) return fail(FDTD_E_INVALID, "tile_kz");
        cfg.kernel = o->kernel == FDTD_KERNEL_FUSED ? 2 : 1;
        cfg.onepass = o->kernel == FDTD_KERNEL_ONEPASS ? 1 : 0;
        cfg.rows = o->tile_rows ? o->tile_rows : 2;
        // split family: tile_rows = rows per block, 4 (64 columns) or 8 (32 columns)
        if (cfg.kernel == 1 && o->tile_rows != 0 && o->tile_rows != 4 && o->tile_rows != 8)
            return fail(FDTD_E_INVALID, "split kernels take tile_rows 4 or 8");
        cfg.sw = (cfg.kernel == 1 && o->tile_rows == 8) ? 32 : 64;
        cfg.kz = o->tile_kz ? o->tile_kz : (cfg.kernel == 1 ? 8 : 16);
        cfg.ndom = n;
        dh.resize(n);
        dd.assign(n, DomDev<T>{});
        for (int q = 0; q < n; ++q) {
            int rc = validate(doms[q], dh[q], q);
            if (rc) return rc;
            init_scalars(q);
        }
        if (o->reversible) {
            // Section 3.2: the reversible mode needs a lossless, nondispersive box
            // between the absorbing slabs that holds the gradient box with the H
            // neighbours its curl reads
            if (o->max_steps < 1) return fail(FDTD_E_INVALID, "reversible mode needs max_steps >= 1");
            bool any = false;
            for (int q = 0; q < n; ++q) {
                const fdtd_domain_desc& s = dh[q].desc;
                if (!s.grad) continue;
                any = true;
                if (s.n_lorentz) return fail(FDTD_E_INVALID, "reversible mode: a dispersive box is not lossless");
                for (int a = 0; a < 3; ++a) {
                    const int lo = s.pml[2 * a], hi = s.n[a] - s.pml[2 * a + 1];
                    if (s.grad_lo[a] < lo + (lo > 0 ? 1 : 0) || s.grad_hi[a] > hi)
                        return fail(FDTD_E_INVALID, "reversible mode: the gradient box reaches an absorbing slab");
                }
            }
            if (!any) return fail(FDTD_E_INVALID, "reversible mode needs a domain with a gradient");
            for (int q = 0; q < n; ++q) {
                rev_maxcnt = std::max(rev_maxcnt, std::max(dd[q].rfcnt[0], std::max(dd[q].rfcnt[1], dd[q].rfcnt[2])));
                if (dd[q].rev)
                    rev_maxcells = std::max(rev_maxcells, (long long)(dd[q].rhi[0] - dd[q].rlo[0]) *
                                                              (dd[q].rhi[1] - dd[q].rlo[1]) * (dd[q].rhi[2] - dd[q].rlo[2]));
            }
        }
        nsets = 2 + (bf16 ? 0 : o->n_ckpt);
        build_tiles();
        // ---- size the arenas
        Arena M, F, A, X;
        layout(M, F, A, X);
        misc_bytes = align256(M.off);
        fstride = align256(F.off);
        astride = align256(A.off);
        et_bytes = align256(X.off);
        size_t bf_total = bf16 ? align256(bfslot) * o->n_ckpt : 0;
        pool_bytes = misc_bytes + fstride * nsets + astride * 2 + et_bytes + bf_total;
        if (size_only) return FDTD_OK;
        if (ext_pool) {
            if (pool_bytes > ext_cap) return fail(FDTD_E_NOMEM, "slab workspace larger than its pool");
            pool = ext_pool;
        }
        if (!ext_pool && o->alloc) {
            if (!o->release) return fail(FDTD_E_INVALID, "an allocator needs its release function");
            pool = (char*)o->alloc(o->alloc_ctx, pool_bytes);
            if (!pool) return fail(FDTD_E_NOMEM, "the caller's allocator returned no memory for the pool");
        } else if (!ext_pool) {
            double budget = o->mem_budget_bytes;
            if (budget <= 0) {
                size_t fr = 0, tot = 0;
                if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(FDTD_E_DEVICE, "hipMemGetInfo failed");
                budget = (double)fr - 256.0 * 1024 * 1024;
            }
            if ((double)pool_bytes > budget) {
                char b[160];
                snprintf(b, sizeof b, "device memory request %.3e B exceeds budget %.3e B", (double)pool_bytes,
                         budget);
                return fail(FDTD_E_NOMEM, b);
            }
            if (hipMalloc((void**)&pool, pool_bytes) != hipSuccess) {
                (void)hipGetLastError();
                pool = nullptr;
                return fail(FDTD_E_NOMEM, "hipMalloc of the device pool failed");
            }
        }
        fbase = pool + misc_bytes;
        abase = fbase + fstride * nsets;
        etbase = abase + astride * 2;
        bfbase = etbase + et_bytes;
        Arena M2, F2, A2, X2;
        M2.base = pool;
        F2.base = fbase;
        A2.base = abase;
        X2.base = etbase;
        M2.assign = F2.assign = A2.assign = X2.assign = true;
        layout(M2, F2, A2, X2);
        for (int q = 0; q < n; ++q) {
            dd[q].fs = (long long)(fstride / sizeof(T));
            dd[q].as = (long long)(astride / sizeof(T));
        }
        slots.assign(o->n_ckpt, Slot{});
        slotset.resize(o->n_ckpt);
        for (int k = 0; k < o->n_ckpt; ++k) slotset[k] = bf16 ? -1 : 2 + k;
        wset[0] = 0;
        wset[1] = 1;
        cur = 0;
        cfg.bs = d_bs;
        cfg.lbs = d_bs + ndom + 1;
        cfg.xr = d_bs + 2 * (ndom + 1);
        cfg.tgen = d_tiles;
        cfg.tbulk = cfg.tgen + tiles_gen.size();
        cfg.tfgen = cfg.tbulk + tiles_bulk.size();
        cfg.tfcp = cfg.tfgen + tiles_fgen.size();
        cfg.tfplain = cfg.tfcp + tiles_fcp.size();
        cfg.ta1 = d_atiles;
        cfg.ta2 = d_atiles + atab1.size();
        // ---- initialise: zero everything, upload tables and inputs
        launch_zero(pool, pool_bytes, st);
        int rc = check("zero pool");
        if (rc) return rc;
        std::vector<T> tmp;
        auto up = [&](const void* dst, const std::vector<double>& src) -> int {
            tmp.assign(src.begin(), src.end());
            if (hipMemcpyAsync((void*)dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, st) !=
                hipSuccess)
                return fail(FDTD_E_DEVICE, "upload failed");
            return hipStreamSynchronize(st) == hipSuccess ? 0 : fail(FDTD_E_DEVICE, "upload sync failed");
        };
        for (int q = 0; q < n; ++q) {
            DomHost& h = dh[q];
            DomDev<T>& d = dd[q];
            const fdtd_domain_desc& s = h.desc;
            std::vector<double> tb;
            for (int a = 0; a < 3; ++a) {
                cpml_tables(s.n[a], s.pml[2 * a], s.pml[2 * a + 1], s.courant, s.pml_m, s.pml_kappa_max,
                            s.pml_sigma_max, s.pml_alpha_max, tb);
                if ((rc = up(d.tab[a], tb))) return rc;
            }
            if ((rc = upload_eps(q))) return rc;
            for (int k = 0; k < s.n_sources; ++k)
                if (s.sources[k].n_waveform > 0 && (rc = up(d.src[k].wave, h.waves[k]))) return rc;
            for (auto& mh : h.mons) {
                if (hipMemcpyAsync((void*)mh.dev.omega, mh.omega.data(), mh.omega.size() * 8, hipMemcpyHostToDevice,
                                   st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "upload omega failed");
            }
        }
        if (hipMemcpyAsync(d_doms, dd.data(), sizeof(DomDev<T>) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(d_bs, bs_host.data(), sizeof(int) * (2 * (n + 1) + 16), hipMemcpyHostToDevice, st) !=
                hipSuccess)
            return fail(FDTD_E_DEVICE, "upload descriptors failed");
        {
            std::vector<int4> all(tiles_gen);
            all.insert(all.end(), tiles_bulk.begin(), tiles_bulk.end());
            all.insert(all.end(), tiles_fgen.begin(), tiles_fgen.end());
            all.insert(all.end(), tiles_fcp.begin(), tiles_fcp.end());
            all.insert(all.end(), tiles_fplain.begin(), tiles_fplain.end());
            if (!all.empty() && hipMemcpyAsync(d_tiles, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice,
                                               st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "upload tile tables failed");
            std::vector<int4> at(atab1);
            at.insert(at.end(), atab2.begin(), atab2.end());
            if (!at.empty() && hipMemcpyAsync(d_atiles, at.data(), sizeof(int4) * at.size(), hipMemcpyHostToDevice,
                                              st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "upload adjoint tiles failed");
            if (!bfarr.empty() && hipMemcpyAsync(d_bfarr, bfarr.data(), sizeof(BfArr) * bfarr.size(),
                                                 hipMemcpyHostToDevice, st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "upload checkpoint table failed");
        }
        return sync("create");
    }

    // scalar (non-pointer) fields of the device descriptor
    void init_scalars(int q) {
        DomHost& h = dh[q];
        DomDev<T>& d = dd[q];
        const fdtd_domain_desc& s = h.desc;
        const int align = 128 / (int)sizeof(T);
        for (int a = 0; a < 3; ++a) d.n[a] = s.n[a];
        d.pitch = (s.n[0] + align - 1) / align * align;
        d.plane = (long long)d.pitch * s.n[1];
        h.nfield = (size_t)d.plane * s.n[2];
        d.S = (T)s.courant;
        for (int a = 0; a < 3; ++a) {
            d.L[a][0] = s.pml[2 * a];
            d.L[a][1] = s.pml[2 * a + 1];
        }
        d.eps_diag = s.eps_kind == FDTD_EPS_DIAG;
        d.tens = s.eps_kind == FDTD_EPS_TENSOR;
        // interior blocks take the single pass unless the domain has tensor media or a periodic axis
        d.onep = opt.kernel == FDTD_KERNEL_ONEPASS && !d.tens && !s.periodic[0] && !s.periodic[1] && !s.periodic[2];
        size_t ebox = 1;
        for (int a = 0; a < 3; ++a) {
            d.elo[a] = s.eps_lo[a];
            d.ehi[a] = s.eps_hi[a];
            ebox *= (size_t)(s.eps_hi[a] - s.eps_lo[a]);
        }
        if (!(ebox && s.eps))
            for (int a = 0; a < 3; ++a) d.elo[a] = d.ehi[a] = 0;
        d.exa = d.elo[0] / align * align;
        d.exs = (d.ehi[0] - d.exa + align - 1) / align * align;
        d.epsinv_bg = (T)(1.0 / s.eps_bg);
        d.has_lor = s.n_lorentz > 0;
        if (d.has_lor) {
            const fdtd_lorentz_desc& L = s.lorentz;
            for (int a = 0; a < 3; ++a) {
                d.llo[a] = L.lo[a];
                d.lhi[a] = L.hi[a];
            }
            // trapezoidal ADE per pole with W = dt J:
            // W^{n+1} = al W^n + xi W^{n-1} + g/2 (E^{n+1} - E^{n-1}), q = 1 + gamma dt/2,
            // Lorentz: al = (2 - (w0 dt)^2)/q, g = deps (w0 dt)^2/q; Drude: al = 2/q, g = (wp dt)^2/q;
            // xi = (gamma dt/2 - 1)/q
            d.npole = L.n_poles;
            double gsum = 0.0;
            for (int p = 0; p < L.n_poles; ++p) {
                const fdtd_pole_desc& pd = L.poles[p];
                const double qq = 1.0 + 0.5 * pd.gamma_dt, w2 = pd.omega_dt * pd.omega_dt;
                const bool drude = pd.kind == FDTD_POLE_DRUDE;
                const double g = drude ? w2 / qq : pd.delta_eps * w2 / qq;
                d.lal[p] = (T)(drude ? 2.0 / qq : (2.0 - w2) / qq);
                d.lxi[p] = (T)((0.5 * pd.gamma_dt - 1.0) / qq);
                d.lg[p] = (T)g;
                gsum += g;
            }
            d.lgs = (T)gsum;
            d.lbox = 1;
            for (int a = 0; a < 3; ++a) d.lbox *= (long long)(L.hi[a] - L.lo[a]);
        }
        d.nsrc = s.n_sources;
        for (int k = 0; k < s.n_sources; ++k) {
            const fdtd_source_desc& sr = s.sources[k];
            SrcDev<T>& sd = d.src[k];
            sd.kind = sr.kind;
            sd.comp = sr.comp;
            sd.i = sr.pos[0];
            sd.j = sr.pos[1];
            sd.k = sr.pos[2];
            sd.nwave = sr.n_waveform;
        }
        for (int a = 0; a < 3; ++a) {
            d.per[a] = s.periodic[a] ? 1 : 0;
            d.bsign[a] = (T)(s.periodic[a] ? s.bloch_sign[a] : 1);
        }
        d.grad = s.grad ? 1 : 0;
        if (s.grad) {
            h.gelems = 1;
            for (int a = 0; a < 3; ++a) {
                d.glo[a] = s.grad_lo[a];
                d.ghi[a] = s.grad_hi[a];
                h.gelems *= (size_t)(s.grad_hi[a] - s.grad_lo[a]);
            }
            h.gncomp = d.tens ? 6 : (d.eps_diag ? 3 : 1);
        }
        d.rev = opt.reversible && s.grad ? 1 : 0;
        h.rec_step = 0;
        for (int f = 0; f < 6; ++f) d.rface[f] = -1;
        if (d.rev) {
            for (int a = 0; a < 3; ++a) {
                d.rlo[a] = s.pml[2 * a];
                d.rhi[a] = s.n[a] - s.pml[2 * a + 1];
            }
            for (int a = 0; a < 3; ++a)
                d.rfcnt[a] = (d.rhi[(a + 1) % 3] - d.rlo[(a + 1) % 3]) * (d.rhi[(a + 2) % 3] - d.rlo[(a + 2) % 3]);
            long long off = 0;
            for (int f = 0; f < 6; ++f) {
                const int a = f % 3;
                const bool present = f < 3 ? d.rlo[a] > 0 : d.rhi[a] < s.n[a];
                if (!present) continue;
                d.rface[f] = off;
                off += 2LL * d.rfcnt[a];
            }
            d.rec_stride = off;
            h.rec_step = (size_t)off;
        }
        for (auto& mh : h.mons) {
            if (mh.dev.kind != 0) mh.acc_elems = (size_t)mh.dev.nf * mh.dev.ncomp * mh.npts * 2;
        }
    }

    // eps^-1 of a domain's eps box in the stored row layout (rows of exs
    // elements from x = exa; the row padding holds the background): ncomp
    // arrays of (box rows) x exs, component c at c * (box rows) * exs.
    // h_eps: [ncomp][bz][by][bx] as the descriptor gives it.
    static void einv_rows(const DomDev<T>& d, int ncomp, const double* h_eps, double bg, std::vector<T>& v) {
        const int bx = d.ehi[0] - d.elo[0], by = d.ehi[1] - d.elo[1], bz = d.ehi[2] - d.elo[2];
        const size_t rows = (size_t)by * bz, ebox = rows * bx, nst = rows * d.exs;
        v.assign(ncomp * nst, T(0));
        const int ncm = ncomp == 6 ? 3 : ncomp;
        for (int c = 0; c < ncm; ++c)
            for (size_t r = 0; r < rows; ++r)
                for (int x = 0; x < d.exs; ++x) v[c * nst + r * d.exs + x] = (T)(1.0 / bg);   // padding: the background
        for (size_t r = 0; r < rows; ++r)
            for (int x = 0; x < bx; ++x) {
                const size_t e = r * bx + x, o = r * d.exs + (d.elo[0] - d.exa) + x;
                if (ncomp == 6) {   // each node's tensor inverted
                    double m[6], w[6];
                    for (int c = 0; c < 6; ++c) m[c] = h_eps[c * ebox + e];
                    sym3_inverse(m, w);
                    for (int c = 0; c < 6; ++c) v[c * nst + o] = (T)w[c];
                } else {
                    for (int c = 0; c < ncomp; ++c) v[c * nst + o] = (T)(1.0 / h_eps[c * ebox + e]);
                }
            }
    }

    int upload_eps(int q) {
        if (external_eps) return FDTD_OK;
        DomHost& h = dh[q];
        DomDev<T>& d = dd[q];
        const int nc = d.tens ? 6 : h.ncomp_eps;
        if (d.tens ? !d.tinv[0] : !d.epsinv[0]) return FDTD_OK;
        std::vector<T> v;
        einv_rows(d, nc, h.eps.data(), h.desc.eps_bg, v);
        const size_t nst = v.size() / nc;
        for (int c = 0; c < nc; ++c) {
            T* dst = d.tens ? const_cast<T*>(d.tinv[c]) : const_cast<T*>(d.epsinv[c]);
            if (hipMemcpyAsync(dst, v.data() + c * nst, nst * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "upload eps failed");
        }
        if (hipStreamSynchronize(st) != hipSuccess) return fail(FDTD_E_DEVICE, "upload eps sync failed");
        return FDTD_OK;
    }

    // ------------------------------------------------------------ validation
    int validate(const fdtd_domain_desc& s, DomHost& h, int dom_index) {
        h.desc = s;
        for (int a = 0; a < 3; ++a)
            if (s.n[a] < 1 || s.n[a] > (1 << 20)) return fail(FDTD_E_INVALID, "grid size out of range");
        if (!(s.courant > 0) || !std::isfinite(s.courant))
            return fail(FDTD_E_UNSTABLE, "Courant number must be positive and finite");
        if (s.courant * std::sqrt(3.0) > 0.99 + 1e-12)
            return fail(FDTD_E_UNSTABLE, "CFL: S*sqrt(3) exceeds 0.99 (Eq. 2)");
        for (int a = 0; a < 3; ++a) {
            int l0 = s.pml[2 * a], l1 = s.pml[2 * a + 1];
            if (l0 < 0 || l1 < 0 || l0 + l1 > s.n[a]) return fail(FDTD_E_INVALID, "absorbing depth out of range");
        }
        // Eq. 2 bounds the step by the vacuum speed, so a permittivity below 1
        // (a faster medium) breaks it; Section 2.3 admits eigenvalues >= 1 only
        if (!(s.eps_bg >= 1.0) || !std::isfinite(s.eps_bg))
            return fail(FDTD_E_UNSTABLE, "background permittivity must be finite and at least 1");
        if (s.eps_kind != FDTD_EPS_ISO && s.eps_kind != FDTD_EPS_DIAG && s.eps_kind != FDTD_EPS_TENSOR)
            return fail(FDTD_E_INVALID, "eps_kind");
        h.ncomp_eps = s.eps_kind == FDTD_EPS_DIAG ? 3 : (s.eps_kind == FDTD_EPS_TENSOR ? 6 : 1);
        size_t ebox = 1;
        for (int a = 0; a < 3; ++a) {
            if (s.eps_lo[a] < 0 || s.eps_hi[a] > s.n[a] || s.eps_lo[a] > s.eps_hi[a])
                return fail(FDTD_E_INVALID, "eps box out of range");
            ebox *= (size_t)(s.eps_hi[a] - s.eps_lo[a]);
        }
        if (ebox && !s.eps && !external_eps) return fail(FDTD_E_INVALID, "eps array missing");
        if (external_eps) {
            h.eps.clear();
        } else {
            h.eps.assign(ebox * h.ncomp_eps, 1.0);
            if (ebox) {
                int rc = validate_eps_only(s, h, s.eps);
                if (rc) return rc;
            }
        }
        if (s.eps_kind == FDTD_EPS_TENSOR) {
            // the tensor path is nondispersive
            if (s.n_lorentz) return fail(FDTD_E_INVALID, "tensor media take no dispersive box");
            if (opt.kernel == FDTD_KERNEL_FUSED) return fail(FDTD_E_INVALID, "tensor media need the split kernels");
            if (opt.reversible) return fail(FDTD_E_INVALID, "tensor media take no reversible mode");
        }
        for (int a = 0; a < 3; ++a) {
            if (s.periodic[a] != 0 && s.periodic[a] != 1) return fail(FDTD_E_INVALID, "periodic flag must be 0 or 1");
            if (!s.periodic[a]) continue;
            if (a == 2) return fail(FDTD_E_INVALID, "periodic z is not supported (x and y only)");
            if (s.pml[2 * a] || s.pml[2 * a + 1])
                return fail(FDTD_E_INVALID, "a periodic axis takes no absorbing cells");
            if (s.bloch_sign[a] != 1 && s.bloch_sign[a] != -1)
                return fail(FDTD_E_INVALID, "bloch_sign of a periodic axis must be +1 or -1");
            if (opt.reversible && s.grad)
                return fail(FDTD_E_INVALID, "periodic domains with a gradient take no reversible mode");
            if (opt.kernel == FDTD_KERNEL_FUSED) return fail(FDTD_E_INVALID, "periodic domains need the split kernels");
        }
        if (s.n_lorentz < 0 || s.n_lorentz > 1) return fail(FDTD_E_INVALID, "at most one Lorentz box per domain");
        if (s.n_lorentz) {
            const fdtd_lorentz_desc& L = s.lorentz;
            for (int a = 0; a < 3; ++a)
                if (L.lo[a] < 0 || L.hi[a] > s.n[a] || L.lo[a] >= L.hi[a]) return fail(FDTD_E_INVALID, "Lorentz box");
            if (L.n_poles < 1 || L.n_poles > FDTD_MAX_POLES) return fail(FDTD_E_INVALID, "1 to 16 poles per box");
            for (int p = 0; p < L.n_poles; ++p) {
                const fdtd_pole_desc& pd = L.poles[p];
                if (pd.kind != FDTD_POLE_LORENTZ && pd.kind != FDTD_POLE_DRUDE)
                    return fail(FDTD_E_INVALID, "pole kind");
                if (!(pd.omega_dt > 0) || !(pd.gamma_dt >= 0) || !std::isfinite(pd.omega_dt) ||
                    !std::isfinite(pd.gamma_dt) ||
                    (pd.kind == FDTD_POLE_LORENTZ && (!(pd.delta_eps >= 0) || !std::isfinite(pd.delta_eps))))
                    return fail(FDTD_E_UNSTABLE, "pole parameters must be finite with omega > 0, gamma >= 0, "
                                                 "delta_eps >= 0");
                // a Lorentz pole's recursion z^2 - alpha z - xi keeps its roots in the unit
                // disc only for (omega_0 dt)^2 < 4, at any damping
                if (pd.kind == FDTD_POLE_LORENTZ && !(pd.omega_dt < 2.0))
                    return fail(FDTD_E_UNSTABLE, "Lorentz omega_0 dt must be below 2");
            }
        }
        if (s.n_sources < 0 || s.n_sources > FDTD_MAX_SOURCES) return fail(FDTD_E_INVALID, "too many sources");
        h.waves.resize(s.n_sources);
        for (int k = 0; k < s.n_sources; ++k) {
            const fdtd_source_desc& sr = s.sources[k];
            if (sr.comp < 0 || sr.comp > 2) return fail(FDTD_E_RANGE, "source component must be Ex, Ey or Ez");
            if (sr.kind == FDTD_SRC_POINT) {
                for (int a = 0; a < 3; ++a)
                    if (sr.pos[a] < 0 || sr.pos[a] >= s.n[a]) return fail(FDTD_E_RANGE, "source position");
            } else if (sr.kind == FDTD_SRC_PLANE_Z) {
                if (sr.pos[2] < 0 || sr.pos[2] >= s.n[2]) return fail(FDTD_E_RANGE, "source plane");
            } else {
                return fail(FDTD_E_INVALID, "source kind");
            }
            if (sr.n_waveform < 0 || (sr.n_waveform > 0 && !sr.waveform)) return fail(FDTD_E_INVALID, "waveform");
            h.waves[k].assign(sr.waveform, sr.waveform + sr.n_waveform);
            for (double w : h.waves[k])
                if (!std::isfinite(w)) return fail(FDTD_E_UNSTABLE, "non-finite waveform sample");
        }
        if (s.n_monitors < 0 || s.n_monitors > FDTD_MAX_MONITORS) return fail(FDTD_E_INVALID, "too many monitors");
        h.mons.resize(s.n_monitors);
        for (int k = 0; k < s.n_monitors; ++k) {
            const fdtd_monitor_desc& md = s.monitors[k];
            MonHost& mh = h.mons[k];
            MonDev& m = mh.dev;
            m.dom = dom_index;
            m.kind = md.kind == FDTD_MON_PROBE ? 0 : (md.kind == FDTD_MON_FLUX_Z ? 1 : 2);
            if (md.kind < 0 || md.kind > 2) return fail(FDTD_E_INVALID, "monitor kind");
            m.comp = md.comp;
            m.k = md.pos[2];
            if (m.k < 0 || m.k >= s.n[2]) return fail(FDTD_E_RANGE, "monitor plane");
            if (md.kind == FDTD_MON_PROBE) {
                if (md.comp < 0 || md.comp > 5) return fail(FDTD_E_RANGE, "probe component");
                m.pi = md.pos[0];
                m.pj = md.pos[1];
                if (m.pi < 0 || m.pi >= s.n[0] || m.pj < 0 || m.pj >= s.n[1]) return fail(FDTD_E_RANGE, "probe position");
                m.ncomp = 1;
                m.nf = 0;
                continue;
            }
            m.i0 = md.rect[0];
            m.i1 = md.rect[1];
            m.j0 = md.rect[2];
            m.j1 = md.rect[3];
            if (m.i0 < 0 || m.i1 > s.n[0] || m.i0 >= m.i1 || m.j0 < 0 || m.j1 > s.n[1] || m.j0 >= m.j1)
                return fail(FDTD_E_RANGE, "monitor rectangle");
            if (md.kind == FDTD_MON_PATCH_Z && (md.comp < 0 || md.comp > 5))
                return fail(FDTD_E_RANGE, "patch component");
            if (md.n_freq < 1 || md.n_freq > 4096 || !md.omega_dt) return fail(FDTD_E_INVALID, "monitor frequencies");
            m.nf = md.n_freq;
            m.ncomp = md.kind == FDTD_MON_FLUX_Z ? 4 : 1;
            m.rcomp = md.kind == FDTD_MON_FLUX_Z ? 6 : 1;
            mh.npts = (m.i1 - m.i0) * (m.j1 - m.j0);
            mh.omega.assign(md.omega_dt, md.omega_dt + md.n_freq);
        }
        if (s.grad) {
            for (int a = 0; a < 3; ++a)
                if (s.grad_lo[a] < 0 || s.grad_hi[a] > s.n[a] || s.grad_lo[a] > s.grad_hi[a])
                    return fail(FDTD_E_INVALID, "gradient box out of range");
        }
        return FDTD_OK;
    }

    // ------------------------------------------------------------ stepping
    void flush(MonHost& mh) {
        if (mh.dev.kind == 0 || mh.pending == 0) return;
        launch_dft<T>(mh.dev, mh.n0, mh.pending, st);
        mh.pending = 0;
    }

    // Ring slot in which the split H kernel can sample every plane monitor
    // during the next step: all plane monitors must be at the same slot (a
    // monitor reset puts one back to 0).  -1: sample with k_sample.
    int insample_slot() const {
        if (cfg.kernel != 1) return -1;
        int slot = -1;
        for (auto& h : dh)
            for (auto& mh : h.mons) {
                if (mh.dev.kind == 0) continue;
                if (slot >= 0 && mh.pending != slot) return -1;
                slot = mh.pending;
            }
        return slot;
    }

    // After a recorded step: probes, and the plane monitors' slot bookkeeping
    // (their samples were written by the H kernel when sampled is set).
    void record(bool sampled) {
        int n = t;   // the current set holds E^n, H^{n+1/2}
        for (auto& h : dh)
            for (auto& mh : h.mons) {
                if (mh.dev.kind == 0) {
                    if (n - 1 < opt.max_steps) launch_probe<T>(d_doms, mh.dev, cur, n - 1, st);
                    continue;
                }
                if (mh.pending == 0) mh.n0 = n;
                if (!sampled) launch_sample<T>(d_doms, mh.dev, cur, mh.pending, st);
                if (++mh.pending == dft_block) flush(mh);
            }
    }

    void ev_mark() {
        if (nev == evs.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                return;
            }
            evs.push_back(e);
        }
        (void)hipEventRecord(evs[nev++], st);
    }

    int write_set() const { return wset[0] != cur ? wset[0] : wset[1]; }

    bool monitors_flushed() const {
        for (auto& h : dh)
            for (auto& mh : h.mons)
                if (mh.dev.kind != 0 && mh.pending != 0) return false;
        return true;
    }

    // Capture graph_chunk in-place split steps (with or without monitor
    // work) into a graph: the step index comes from d_tstep, which the last
    // node advances, so one executable serves every chunk.
    int graph_for(bool rec, GraphEx*& out) {
        const int key = (rec ? 1 : 0) | (cur << 1), G = opt.graph_chunk;
        for (auto& g : graphs)
            if (g.key == key) {
                out = &g;
                return FDTD_OK;
            }
        if (!cst && hipStreamCreateWithFlags(&cst, hipStreamNonBlocking) != hipSuccess)
            return fail(FDTD_E_DEVICE, "capture stream");
        if (hipStreamBeginCapture(cst, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(FDTD_E_DEVICE, "hipStreamBeginCapture failed");
        // recording chunks start with every ring empty: step s samples into slot s.
        // In place (split), or ping-pong between the two working sets (single pass)
        int rset = cur;
        for (int s = 0; s < G; ++s) {
            const int wset_ = cfg.onepass ? (wset[0] != rset ? wset[0] : wset[1]) : rset;
            launch_fwd<T>(cfg, d_doms, rset, wset_, s, cst, d_tstep, rec ? s : -1);
            rset = wset_;
            if (!rec) continue;
            for (auto& h : dh)
                for (auto& mh : h.mons)
                    if (mh.dev.kind == 0) launch_probe<T>(d_doms, mh.dev, rset, s, cst, d_tstep);
        }
        if (rec)
            for (auto& h : dh)
                for (auto& mh : h.mons)
                    if (mh.dev.kind != 0) launch_dft<T>(mh.dev, 1, G, cst, d_tstep);
        launch_step_counter(d_tstep, G, true, cst);
        GraphEx ge{key, nullptr, nullptr};
        if (hipStreamEndCapture(cst, &ge.g) != hipSuccess || !ge.g)
            return fail(FDTD_E_DEVICE, "hipStreamEndCapture failed");
        if (hipGraphInstantiate(&ge.ex, ge.g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(ge.g);
            return fail(FDTD_E_DEVICE, "hipGraphInstantiate failed");
        }
        graphs.push_back(ge);
        out = &graphs.back();
        return FDTD_OK;
    }

    // reversible mode: interface of the current state into record slot t
    void rev_record() {
        if (!opt.reversible || t > opt.max_steps) return;
        launch_rev_record<T>(d_doms, ndom, cur, t, rev_maxcnt, st);
        if (rec_hi < 0 || t < rec_lo || t > rec_hi + 1) rec_lo = rec_hi = t;
        else if (t == rec_hi + 1) rec_hi = t;
    }

    int step_forward(int n, unsigned flags) override {
        if (n < 0) return fail(FDTD_E_INVALID, "negative step count");
        if (opt.reversible) {   // eager steps, the interface recorded before each and after the last
            for (int s = 0; s < n; ++s) {
                int rc = step_forward_eager(1, flags);
                if (rc) return rc;
            }
            rev_record();
            return check("step_forward");
        }
        return step_forward_eager(n, flags);
    }

    int step_reverse(int n) override {
        if (!opt.reversible) return fail(FDTD_E_STATE, "the handle was not created in reversible mode");
        if (n < 0) return fail(FDTD_E_INVALID, "negative step count");
        for (int s = 0; s < n; ++s) {
            if (t < 1 || rec_hi < 0 || t - 1 < rec_lo || t > rec_hi) {
                char b[160];
                snprintf(b, sizeof b, "no recorded interface for the backward step from %d (recorded %d..%d)", t,
                         rec_lo, rec_hi);
                return fail(FDTD_E_STATE, b);
            }
            const bool working = cur == wset[0] || cur == wset[1];
            const int ws = working ? cur : write_set();
            if (timing_on) ev_mark();
            launch_rev_step<T>(d_doms, ndom, cur, ws, t, rev_maxcells, st);
            if (timing_on) ev_mark();
            cur = ws;
            --t;
        }
        return check("step_reverse");
    }

    int step_forward_eager(int n, unsigned flags) {
        if (opt.reversible) rev_record();
        bool rec = (flags & FDTD_RECORD) && !(flags & FDTD_REPLAY);
        // The split kernels update a working set in place; the fused pass
        // reads neighbours' old values after they are overwritten, so it
        // writes the other set.  A restored slot is never written.
        // (the single-pass family reads neighbours' old values across blocks:
        // it and the split kernels beside it write the other working set)
        const bool inplace = cfg.kernel == 1 && !cfg.onepass;
        const int G = opt.graph_chunk;
        for (int s = 0; s < n;) {
            const bool working = cur == wset[0] || cur == wset[1];
            if (G > 0 && cfg.kernel == 1 && (inplace || G % 2 == 0) && working && !timing_on && !opt.reversible &&
                n - s >= G && (!rec || monitors_flushed())) {
                GraphEx* g = nullptr;
                int rc = graph_for(rec, g);
                if (rc) return rc;
                if (tstep_val != t) launch_step_counter(d_tstep, t, false, st);
                if (hipGraphLaunch(g->ex, st) != hipSuccess) return fail(FDTD_E_DEVICE, "hipGraphLaunch failed");
                t += G;
                tstep_val = t;
                s += G;
                continue;   // an even chunk of ping-pong steps ends in the set it started from
            }
            int ws = inplace && working ? cur : write_set();
            const int slot = rec ? insample_slot() : -1;
            if (timing_on) ev_mark();
            launch_fwd<T>(cfg, d_doms, cur, ws, t, st, nullptr, slot);
            if (timing_on) ev_mark();
            cur = ws;
            ++t;
            if (rec) record(slot >= 0);
            ++s;
        }
        return check("step_forward");
    }

    int seed(int n) {
        for (auto& h : dh) {
            if (!h.desc.grad) continue;
            for (auto& mh : h.mons) {
                if (!mh.cot_set) continue;
                if (mh.dev.kind == 0 && (n - 1 >= opt.max_steps || n < 1)) continue;
                launch_seed<T>(d_doms, mh.dev, ap, n, st);
            }
        }
        return check("seed");
    }

    int adjoint_begin(int n) override {
        if (n < 0) return fail(FDTD_E_INVALID, "negative n_total");
        if (astride) launch_zero(abase, astride * 2, st);
        for (auto& a : adj_flat) launch_zero(a.first, a.second, st);
        ap = 0;
        m = n;
        if (n >= 1) return seed(n);
        return check("adjoint_begin");
    }

    // Both passes on the caller's stream.  (Forking the classes of a pass onto
    // further streams and joining them back cost more in event waits than
    // the overlap won.)
    int launch_adjoint_passes() {
        hipStream_t cs[kAdjClasses1];
        for (int q = 0; q < kAdjClasses1; ++q) cs[q] = st;
        launch_adj<T>(cfg, d_doms, ap, ap ^ 1, cur, st, 0, cs);
        for (int q = 0; q < ndom; ++q) {
            if (!dd[q].grad) continue;
            const bool per = dd[q].per[0] || dd[q].per[1];
            if (dd[q].tens) {
                launch_tens_adj<T>(d_doms, q, dd[q].n, ap, ap ^ 1, cur, per, st);
                if (per) launch_per_adj_h<T>(d_doms, q, dd[q].n, ap, ap ^ 1, st);
            } else if (per) {
                launch_per_adj<T>(d_doms, q, dd[q].n, ap, ap ^ 1, cur, st);
            }
        }
        if (cfg.kernel == 1) launch_adj<T>(cfg, d_doms, ap, ap ^ 1, cur, st, 1, cs);
        return FDTD_OK;
    }

    int step_adjoint(int n) override {
        if (m < 0) return fail(FDTD_E_STATE, "fdtd_adjoint_begin has not been called");
        for (int s = 0; s < n; ++s) {
            if (m < 1) return fail(FDTD_E_STATE, "adjoint sweep already at step 0");
            if (t != m - 1) {
                char b[128];
                snprintf(b, sizeof b, "adjoint step %d needs forward state u^%d, forward is at %d", m, m - 1, t);
                return fail(FDTD_E_STATE, b);
            }
            if (timing_on) ev_mark();
            int rc = launch_adjoint_passes();
            if (rc) return rc;
            if (timing_on) ev_mark();
            ap ^= 1;
            --m;
            if (m >= 1) {
                int rc = seed(m);
                if (rc) return rc;
            }
        }
        return check("step_adjoint");
    }

    int timing(int op, double* ms, long long* cnt) override {
        if (op == 1 || op == 0) {
            if (sync("timing")) return FDTD_E_DEVICE;
            timing_on = op == 1;
            nev = 0;
            return FDTD_OK;
        }
        if (op != 2) return fail(FDTD_E_INVALID, "timing op");
        int rc = sync("timing");
        if (rc) return rc;
        double tot = 0;
        for (size_t q = 0; q + 1 < nev; q += 2) {
            float e = 0;
            if (hipEventElapsedTime(&e, evs[q], evs[q + 1]) != hipSuccess) {
                (void)hipGetLastError();
                return fail(FDTD_E_DEVICE, "hipEventElapsedTime failed");
            }
            tot += e;
        }
        if (ms) *ms = tot;
        if (cnt) *cnt = (long long)(nev / 2);
        return FDTD_OK;
    }

    // ------------------------------------------------------------ checkpoints
    // Full-precision slots are forward state sets.  Saving hands the current
    // working set to the slot and takes the slot's old set as the new working
    // set (no copy); restoring points the next step at the slot's set (no copy).
    int ckpt_save(int slot) override {
        if (slot < 0 || slot >= (int)slots.size()) return fail(FDTD_E_RANGE, "checkpoint slot");
        if (bf16) {
            launch_bf16_save(d_bfarr, (int)bfarr.size(), bfblocks, (long long)cur * (long long)fstride, d_bfpart,
                             d_scales + (size_t)slot * bfarr.size(), bfbase + (size_t)slot * align256(bfslot), st);
        } else if (cur == wset[0] || cur == wset[1]) {
            int wi = cur == wset[0] ? 0 : 1;
            int old = slotset[slot];
            slotset[slot] = cur;
            wset[wi] = old;
        } else if (cur != slotset[slot]) {
            launch_copy(set_ptr(cur), set_ptr(slotset[slot]), fstride, st);
        }
        slots[slot].valid = true;
        slots[slot].step = t;
        if (opt.ckpt_checksum) {
            int rc = slot_sum(slot, &slots[slot].sum);
            if (rc) return rc;
        }
        return check("checkpoint_save");
    }

    int slot_sum(int slot, unsigned long long* out) {
        launch_zero(d_sum, 8, st);
        if (bf16) launch_checksum(bfbase + (size_t)slot * align256(bfslot), bfslot, d_sum, st);
        else launch_checksum(set_ptr(slotset[slot]), fstride, d_sum, st);
        if (hipMemcpyAsync(out, d_sum, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
            return fail(FDTD_E_DEVICE, "checksum copy failed");
        return sync("checksum");
    }

    int ckpt_restore(int slot) override {
        if (slot < 0 || slot >= (int)slots.size()) return fail(FDTD_E_RANGE, "checkpoint slot");
        if (!slots[slot].valid) return fail(FDTD_E_STATE, "checkpoint slot is empty");
        if (opt.ckpt_checksum) {
            unsigned long long s2 = 0;
            int rc = slot_sum(slot, &s2);
            if (rc) return rc;
            if (s2 != slots[slot].sum) return fail(FDTD_E_STATE, "checkpoint checksum mismatch");
        }
        if (bf16) {
            int ws = write_set();
            launch_bf16_restore(d_bfarr, (int)bfarr.size(), bfblocks, (long long)ws * (long long)fstride,
                                d_scales + (size_t)slot * bfarr.size(), bfbase + (size_t)slot * align256(bfslot), st);
            cur = ws;
        } else {
            cur = slotset[slot];
        }
        t = slots[slot].step;
        return check("checkpoint_restore");
    }

    int probe_trace(int dom, int mon, double* buf, int n) override {
        if (dom < 0 || dom >= ndom) return fail(FDTD_E_RANGE, "domain index");
        if (mon < 0 || mon >= (int)dh[dom].mons.size()) return fail(FDTD_E_RANGE, "monitor index");
        if (dh[dom].mons[mon].dev.kind != 0) return fail(FDTD_E_INVALID, "not a probe monitor");
        if (n > std::max(1, opt.max_steps)) return fail(FDTD_E_RANGE, "more samples than max_steps");
        if (n == 0) return FDTD_OK;
        return monitor(dom, mon, FDTD_MON_GET, buf, (size_t)n * 8);
    }

    // Watchdog: the fields' sum of squares, reduced on the device; a
    // non-finite sum means a NaN or an infinity somewhere in the state.
    int energy(int dom, double* out) override {
        if (dom < 0 || dom >= ndom) return fail(FDTD_E_RANGE, "domain index");
        launch_energy<T>(d_doms, dom, cur, d_energy, d_energy + kEnergyBlocks, st);
        if (hipMemcpyAsync(out, d_energy + kEnergyBlocks, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
            return fail(FDTD_E_DEVICE, "energy copy failed");
        int rc = sync("energy");
        if (rc) return rc;
        if (!std::isfinite(*out)) return fail(FDTD_E_UNSTABLE, "non-finite field energy: the state holds a NaN or an "
                                                                "infinity (diverged run or non-finite input)");
        return FDTD_OK;
    }

    // Corrupt one word of a slot (failure-path tests of checksum validation).
    int poke_slot(int slot, size_t word, unsigned int value) override {
        if (slot < 0 || slot >= (int)slots.size()) return fail(FDTD_E_RANGE, "checkpoint slot");
        char* base = bf16 ? bfbase + (size_t)slot * align256(bfslot) : set_ptr(slotset[slot]);
        size_t bytes = bf16 ? bfslot : fstride;
        if ((word + 1) * 4 > bytes) return fail(FDTD_E_RANGE, "word index");
        if (hipMemcpyAsync(base + word * 4, &value, 4, hipMemcpyHostToDevice, st) != hipSuccess)
            return fail(FDTD_E_DEVICE, "poke failed");
        return sync("poke");
    }

    // ------------------------------------------------------------ monitors
    int monitor(int dom, int mon, int op, void* buf, size_t bytes) override {
        if (dom < 0 || dom >= ndom) return fail(FDTD_E_RANGE, "domain index");
        DomHost& h = dh[dom];
        if (mon < 0 || mon >= (int)h.mons.size()) return fail(FDTD_E_RANGE, "monitor index");
        MonHost& mh = h.mons[mon];
        MonDev& m = mh.dev;
        size_t ms = (size_t)std::max(1, opt.max_steps);
        if (op == FDTD_MON_RESET) {
            if (m.kind == 0) launch_zero(m.trace, ms * 8, st);
            else launch_zero(m.acc, mh.acc_elems * 8, st);
            mh.pending = 0;
            return check("monitor reset");
        }
        if (op == FDTD_MON_GET || op == FDTD_MON_FLUX) {
            flush(mh);
            if (m.kind == 0) {
                if (op != FDTD_MON_GET) return fail(FDTD_E_INVALID, "flux of a probe");
                size_t nb = std::min(bytes / 8, ms) * 8;
                if (hipMemcpyAsync(buf, m.trace, nb, hipMemcpyDeviceToHost, st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "probe copy failed");
                return sync("probe get");
            }
            if (op == FDTD_MON_GET) {
                if (bytes < mh.acc_elems * 8) return fail(FDTD_E_RANGE, "buffer too small for spectra");
                if (hipMemcpyAsync(buf, m.acc, mh.acc_elems * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "spectra copy failed");
                return sync("spectra get");
            }
            if (m.kind != 1) return fail(FDTD_E_INVALID, "flux needs a flux monitor");
            if (bytes < (size_t)m.nf * 8) return fail(FDTD_E_RANGE, "buffer too small for flux");
            // F(w) = Re sum (Ex Hy* - Ey Hx*) over the plane, reduced on the device
            launch_flux(m.acc, m.nf, mh.npts, m.fpart, m.fout, st);
            if (hipMemcpyAsync(buf, m.fout, (size_t)m.nf * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "flux copy failed");
            int rc = sync("flux");
            if (rc) return rc;
            for (int f = 0; f < m.nf; ++f)   // watchdog: a diverged run shows in its flux
                if (!std::isfinite(((const double*)buf)[f]))
                    return fail(FDTD_E_UNSTABLE, "non-finite flux: the run diverged or was fed non-finite input");
            return FDTD_OK;
        }
        if (op == FDTD_MON_SET_COTANGENT) {
            if (m.kind == 0) {
                std::vector<double> g(ms, 0.0);
                std::memcpy(g.data(), buf, std::min(bytes / 8, ms) * 8);
                if (hipMemcpyAsync(m.cot, g.data(), ms * 8, hipMemcpyHostToDevice, st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "cotangent copy failed");
            } else {
                if (bytes < mh.acc_elems * 8) return fail(FDTD_E_RANGE, "buffer too small for cotangents");
                if (hipMemcpyAsync(m.cot, buf, mh.acc_elems * 8, hipMemcpyHostToDevice, st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "cotangent copy failed");
            }
            mh.cot_set = true;
            return sync("set cotangent");
        }
        return fail(FDTD_E_INVALID, "monitor op");
    }

    // ------------------------------------------------------------ fields
    int get_field(int dom, int comp, void* buf, size_t bytes, bool set) override {
        if (dom < 0 || dom >= ndom) return fail(FDTD_E_RANGE, "domain index");
        if (comp < 0 || comp > 11) return fail(FDTD_E_RANGE, "component");
        DomDev<T>& d = dd[dom];
        bool adjc = comp >= 6;
        int c = comp % 6;
        if (adjc && !d.grad) return fail(FDTD_E_RANGE, "domain has no adjoint state");
        if (set && !adjc && cur != wset[0] && cur != wset[1]) {
            // never write into a checkpoint slot: continue from a working copy
            int ws = write_set();
            launch_copy(set_ptr(cur), set_ptr(ws), fstride, st);
            cur = ws;
        }
        if (set && !adjc) rec_lo = rec_hi = -1;   // the recorded interface belongs to another trajectory
        T* p = adjc ? (c < 3 ? d.Ea[c] : d.Ha[c - 3]) + (size_t)ap * d.as
                    : (c < 3 ? d.E[c] : d.H[c - 3]) + (size_t)cur * d.fs;
        size_t nx = d.n[0], ny = d.n[1], nz = d.n[2];
        if (bytes < nx * ny * nz * sizeof(T)) return fail(FDTD_E_RANGE, "buffer too small for field");
        hipError_t e;
        if (set)
            e = hipMemcpy2DAsync(p, d.pitch * sizeof(T), buf, nx * sizeof(T), nx * sizeof(T), ny * nz,
                                 hipMemcpyHostToDevice, st);
        else
            e = hipMemcpy2DAsync(buf, nx * sizeof(T), p, d.pitch * sizeof(T), nx * sizeof(T), ny * nz,
                                 hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return fail(FDTD_E_DEVICE, "field copy failed");
        return sync("field copy");
    }

    int get_grad(int dom, double* buf, size_t bytes) override {
        if (dom < 0 || dom >= ndom) return fail(FDTD_E_RANGE, "domain index");
        DomHost& h = dh[dom];
        DomDev<T>& d = dd[dom];
        if (!d.grad) return fail(FDTD_E_RANGE, "domain has no gradient");
        if (bytes < h.gelems * h.gncomp * 8) return fail(FDTD_E_RANGE, "buffer too small for gradient");
        for (int c = 0; c < h.gncomp; ++c)
            if (hipMemcpyAsync(buf + c * h.gelems, d.gacc[c], h.gelems * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "gradient copy failed");
        return sync("gradient copy");
    }

    int set_eps(int dom, const double* eps, size_t bytes) override {
        if (dom < 0 || dom >= ndom) return fail(FDTD_E_RANGE, "domain index");
        DomHost& h = dh[dom];
        if (bytes < h.eps.size() * 8) return fail(FDTD_E_RANGE, "buffer too small for eps");
        int rc = validate_eps_only(h.desc, h, eps);
        if (rc) return rc;
        rec_lo = rec_hi = -1;   // another trajectory
        return upload_eps(dom);
    }

    // Checks a permittivity array of the domain's layout (h.eps.size()
    // values) and keeps it as the host copy.  Every value (every eigenvalue of
    // a tensor) must be finite and at least 1: Eq. 2 bounds the step by the
    // vacuum speed.  Section 2.3: inside an absorbing face (index along the
    // normal in the slab: the E position of a diagonal entry, the node of a
    // tensor) the normal must be a principal axis whose eigenvalue is not the
    // intermediate one.
    int validate_eps_only(const fdtd_domain_desc& s, DomHost& h, const double* eps) {
        std::vector<double> v(eps, eps + h.eps.size());
        const int nc = h.ncomp_eps;
        const size_t ebox = h.eps.size() / nc;
        const int bx = s.eps_hi[0] - s.eps_lo[0], by = s.eps_hi[1] - s.eps_lo[1];
        for (size_t e = 0; e < ebox; ++e) {
            const int x[3] = {s.eps_lo[0] + (int)(e % bx), s.eps_lo[1] + (int)((e / bx) % by),
                              s.eps_lo[2] + (int)(e / ((size_t)bx * by))};
            bool inface[3];
            for (int a = 0; a < 3; ++a) inface[a] = x[a] < s.pml[2 * a] || x[a] >= s.n[a] - s.pml[2 * a + 1];
            if (nc == 6) {
                double m[6];
                for (int q = 0; q < 6; ++q) m[q] = v[q * ebox + e];
                const char* why = tensor_node_check(m, inface);
                if (why) return fail(FDTD_E_UNSTABLE, why);
                continue;
            }
            for (int c = 0; c < nc; ++c)
                if (!(v[c * ebox + e] >= 1.0) || !std::isfinite(v[c * ebox + e]))
                    return fail(FDTD_E_UNSTABLE, "permittivity must be finite and at least 1");
            if (nc == 3) {
                const double w[3] = {v[e], v[ebox + e], v[2 * ebox + e]};
                for (int a = 0; a < 3; ++a) {
                    if (!inface[a]) continue;
                    const double o1 = w[(a + 1) % 3], o2 = w[(a + 2) % 3];
                    if (w[a] > std::min(o1, o2) && w[a] < std::max(o1, o2))
                        return fail(FDTD_E_UNSTABLE, "anisotropic eps with intermediate normal eigenvalue in an absorbing face");
                }
            }
        }
        h.eps = std::move(v);
        return FDTD_OK;
    }

    int reset() override {
        cur = wset[0];
        launch_zero(set_ptr(cur), fstride, st);
        for (auto& sl : slots) sl.valid = false;
        for (auto& h : dh)
            for (auto& mh : h.mons) {
                if (mh.dev.kind == 0) launch_zero(mh.dev.trace, std::max(1, opt.max_steps) * 8, st);
                else launch_zero(mh.dev.acc, mh.acc_elems * 8, st);
                mh.pending = 0;
            }
        t = 0;
        m = -1;
        rec_lo = rec_hi = -1;
        return sync("reset");
    }

    void steps(int* n, int* mm) override {
        if (n) *n = t;
        if (mm) *mm = m;
    }

    double memory() override { return (double)pool_bytes; }
};

int guard(fdtd_t h);

}  // namespace

namespace {
// ------------------------------------------------------------ streamed slabs
// Host-streamed causal slabs (Section 4.2).  The domain is cut along z, the
// slowest axis of the x-fastest layout, so that every transfer between the
// host banks and the device is one contiguous copy per state array.  Each
// slab owns a core of at most W planes; the cores tile [0, nz).  One pass
// advances the whole domain by K steps: every slab in turn is loaded from
// bank A (time t) over its core plus K + 1 halo planes on each cut side, is
// stepped K times in a device workspace, and writes its core to bank B
// (time t + K); then the banks swap.  A cut face acts as a wall with ghost
// zeros, and a wrong value moves at most one plane per step (the E update
// reads H one plane back, the H update E one plane forward), so after K
// steps the wrong planes are the K nearest each cut: the core and the
// halo plane next to it are exact, the latter for the flux planes' H below.
// An absorbing z face is either wholly inside a slab's extent (with its
// memories) or outside it, so every slab's absorber tables are the domain's.
struct StreamBase {
    virtual ~StreamBase() = default;
    std::string err;
    bool poisoned = false;
    virtual int step(int n) = 0;
    virtual int get_field(int comp, void* buf, size_t bytes) = 0;
    virtual int monitor(int mon, int op, double* buf, size_t bytes) = 0;
    virtual int reset() = 0;
    virtual void info(fdtd_stream_info* o) = 0;
    virtual int set_cotangent(int mon, const double* buf, size_t bytes) = 0;
    virtual int reverse() = 0;
    virtual int get_grad(double* buf, size_t bytes) = 0;
};

template <typename T>
struct Streamer : StreamBase {
    fdtd_domain_desc g{};                       // the domain (pointers into the copies below)
    fdtd_stream_options so{};
    std::vector<std::vector<double>> waves, omegas;
    hipStream_t st = nullptr;
    int nx = 0, ny = 0, nz = 0, pitch = 0, K = 0, halo = 0, t = 0, npole = 0, ncomp_eps = 1;
    std::vector<int> core;                      // core start plane of each slab; core[ns] = nz
    // One global state array: planes [z0, z1) of `per` elements each, at
    // element offset `off` of a bank.  kind: 0 field E/H c, 1 psi_E, 2 psi_H
    // (a, side, r), 3 dispersive history (w, c, pole p).
    struct GArr {
        int kind, c, a, side, r, w, p;
        int z0, z1;
        size_t per, off;
    };
    std::vector<GArr> ga;
    size_t bank_elems = 0;
    // Forward banks.  Forward only: two, ping-ponged (cb holds time t).  With
    // a gradient: one per pass boundary, bank j holding time j K, so that the
    // reverse sweep finds every block's starting state; passes are then K
    // steps long except a last, shorter one.  With host_banks = B (bounded):
    // B banks, one holding time t (cur_id), snap[p] the bank holding the
    // state at pass boundary p (time 0 always; the forward keeps the
    // positions `planned` of the binomial descent), the rest free.
    bool adj = false;
    std::vector<T*> bank;
    int cb = 0;
    bool bounded = false;
    int cur_id = 0;
    std::vector<int> snap;                      // pass boundary -> bank, or -1
    std::vector<char> planned;                  // pass boundary kept by the forward
    int replay_passes = 0;
    T* abank[2] = {nullptr, nullptr};           // cotangent state banks of the reverse sweep
    std::vector<double> grad;                   // dJ/deps over the gradient box [ncomp][gz][gy][gx]
    int gncomp = 1;
    size_t gelems = 0;
    std::vector<std::vector<double>> cots;      // monitor cotangents (host copies)
    std::vector<char> cot_set;
    int grad_step = -1;                         // the forward length the gradient was taken over
    // eps^-1 of the domain in the field type over its eps box, per component
    // (tensor: six), pinned, uploaded plane-range by plane-range per slab
    T* einv = nullptr;
    T* d_einv = nullptr;                        // a device copy of einv when the budget holds it
    DomDev<T> egeom{};                          // the domain's eps box geometry (elo, ehi, exa, exs)
    size_t ebox = 0;
    int ez0 = 0, ez1 = 0;
    size_t eplane = 0;
    // workspaces: one, or two (overlap) so that one slab's transfers run
    // beside the other's steps, each with its own stream and slab handle
    int nws = 1;
    char* pool[2] = {nullptr, nullptr};
    size_t pool_cap = 0;
    hipStream_t wst[2] = {nullptr, nullptr};
    std::unique_ptr<Handle<T>> hs[2];
    // monitor accumulators of the domain on the device: spectra or the probe trace
    struct GMon {
        int kind, nf, k, slab;
        long long npts;
        size_t elems;
        double *acc = nullptr, *fpart = nullptr, *fout = nullptr;
    };
    std::vector<GMon> gm;
    char* dmon = nullptr;
    size_t dmon_bytes = 0;
    double resident_bytes = 0;
    static inline double dummy_eps = 1.0;

    ~Streamer() override {
        for (int k = 0; k < 2; ++k) hs[k].reset();
        if (st) (void)hipStreamSynchronize(st);
        for (int k = 0; k < 2; ++k) {
            if (wst[k]) (void)hipStreamDestroy(wst[k]);
            if (pool[k]) (void)hipFree(pool[k]);
        }
        if (dmon) (void)hipFree(dmon);
        if (d_einv) (void)hipFree(d_einv);
        for (T* b : bank)
            if (b) (void)hipHostFree(b);
        for (int b = 0; b < 2; ++b)
            if (abank[b]) (void)hipHostFree(abank[b]);
        if (einv) (void)hipHostFree(einv);
    }

    int fail(int code, const std::string& m) {
        err = m;
        if (code == FDTD_E_DEVICE) poisoned = true;
        return code;
    }

    int ns() const { return (int)core.size() - 1; }
    int ext_lo(int s) const { return std::max(0, core[s] - (s > 0 ? halo : 0)); }
    int ext_hi(int s) const { return std::min(nz, core[s + 1] + (s + 1 < ns() ? halo : 0)); }

    fdtd_options slab_options(int n_ckpt = 0) const {
        fdtd_options o{};
        o.n_ckpt = n_ckpt;
        o.dtype = so.dtype;
        o.max_steps = so.max_steps;
        o.kernel = FDTD_KERNEL_SPLIT;
        o.tile_rows = so.tile_rows;
        o.tile_kz = so.tile_kz;
        o.stream = so.stream;
        o.ckpt_storage = so.dtype;
        return o;
    }

    // The descriptor of slab s: the domain's planes [o, e) with the absorbing
    // z faces it contains, the eps and dispersive boxes clipped to it, the
    // sources in it and the monitors whose plane lies in its core (lmon:
    // their indices in the domain's list).
    fdtd_domain_desc slab_desc(int s, std::vector<int>& lmon, bool reverse = false) const {
        const int o = ext_lo(s), e = ext_hi(s);
        fdtd_domain_desc d = g;
        d.n[2] = e - o;
        d.pml[4] = o == 0 ? g.pml[4] : 0;
        d.pml[5] = e == nz ? g.pml[5] : 0;
        d.eps_lo[2] = std::max(g.eps_lo[2], o) - o;
        d.eps_hi[2] = std::max(std::min(g.eps_hi[2], e) - o, d.eps_lo[2]);
        d.eps = ebox ? &dummy_eps : nullptr;
        if (d.eps_hi[2] == d.eps_lo[2]) {
            for (int a = 0; a < 3; ++a) d.eps_lo[a] = d.eps_hi[a] = 0;
            d.eps = nullptr;
        }
        d.n_lorentz = 0;
        if (g.n_lorentz) {
            const int l0 = std::max(g.lorentz.lo[2], o), l1 = std::min(g.lorentz.hi[2], e);
            if (l1 > l0) {
                d.n_lorentz = 1;
                d.lorentz.lo[2] = l0 - o;
                d.lorentz.hi[2] = l1 - o;
            }
        }
        d.n_sources = 0;
        for (int q = 0; q < g.n_sources; ++q) {
            const fdtd_source_desc& sr = g.sources[q];
            if (sr.pos[2] < o || sr.pos[2] >= e) continue;
            fdtd_source_desc& x = d.sources[d.n_sources++];
            x = sr;
            x.pos[2] = sr.pos[2] - o;
        }
        // forward: the monitors whose plane lies in the core (they record);
        // reverse: every monitor whose plane lies in the extent, since its
        // seeds enter the cotangent state wherever the extent holds its plane
        d.n_monitors = 0;
        lmon.clear();
        for (int q = 0; q < g.n_monitors; ++q) {
            const int k = g.monitors[q].pos[2];
            if (reverse ? (k < o || k >= e) : gm[q].slab != s) continue;
            fdtd_monitor_desc& x = d.monitors[d.n_monitors++];
            x = g.monitors[q];
            x.pos[2] = k - o;
            lmon.push_back(q);
        }
        d.grad = reverse ? 1 : 0;
        if (reverse) {   // the gradient box clipped to the extent (possibly empty)
            d.grad_lo[2] = std::min(std::max(g.grad_lo[2], o), e) - o;
            d.grad_hi[2] = std::max(std::min(g.grad_hi[2], e) - o, d.grad_lo[2]);
        }
        return d;
    }

    // device address of the slab handle's copy of global array q and the
    // first global plane it holds (nullptr: the slab does not hold it)
    // (cot: the cotangent copy, in the handle's adjoint set aset)
    T* slab_array(Handle<T>& hd, const GArr& q, int o, int e, int& sz0, int& sz1, bool cot = false,
                  int aset = 0) const {
        const DomDev<T>& d = hd.dd[0];
        sz0 = std::max(q.z0, o);
        sz1 = std::min(q.z1, e);
        if (sz1 <= sz0) return nullptr;
        const long long so = cot ? (long long)aset * d.as : 0;
        switch (q.kind) {
            case 0:
                return (cot ? (q.c < 3 ? d.Ea[q.c] : d.Ha[q.c - 3]) : (q.c < 3 ? d.E[q.c] : d.H[q.c - 3])) + so;
            case 1:
            case 2: {
                if (q.a == 2 && ((q.side == 0 && o != 0) || (q.side == 1 && e != nz))) return nullptr;
                if (cot) return (q.kind == 1 ? d.psiEa[q.a][q.side][q.r] : d.psiHa[q.a][q.side][q.r]) + so;
                return q.kind == 1 ? d.psiE[q.a][q.side][q.r] : d.psiH[q.a][q.side][q.r];
            }
            default: {
                if (!d.has_lor) return nullptr;
                const long long lbox = d.lbox;
                return (cot ? d.lora[q.w][q.c] + so : d.lor[q.w][q.c]) + (long long)q.p * lbox;
            }
        }
    }

    // copies of the state arrays between a host bank and the slab handle:
    // up: the extent [o, e) into the handle; down: planes [c0, c1) to the bank
    int xfer(Handle<T>& hd, T* hbank, bool up, int o, int e, int c0, int c1, hipStream_t st, bool cot = false,
             int aset = 0) {
        for (const GArr& q : ga) {
            int sz0, sz1;
            T* p = slab_array(hd, q, o, e, sz0, sz1, cot, aset);
            if (!p) continue;
            const int z0 = up ? sz0 : std::max(sz0, c0), z1 = up ? sz1 : std::min(sz1, c1);
            if (z1 <= z0) continue;
            T* dv = p + (size_t)slab_plane(q, z0, o, sz0) * q.per;
            T* hv = hbank + q.off + (size_t)(z0 - q.z0) * q.per;
            const size_t nb = (size_t)(z1 - z0) * q.per * sizeof(T);
            if (hipMemcpyAsync(up ? (void*)dv : (void*)hv, up ? (const void*)hv : (const void*)dv, nb,
                               up ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost, st) != hipSuccess)
                return fail(FDTD_E_DEVICE, up ? "slab state upload failed" : "slab state download failed");
        }
        return FDTD_OK;
    }

    // the plane of the slab array holding global plane z
    static int slab_plane(const GArr& q, int z, int o, int sz0) {
        if (q.kind == 0) return z - o;
        if ((q.kind == 1 || q.kind == 2) && q.a < 2) return z - o;
        return z - sz0;   // z faces and the dispersive box: arrays start at their own first plane
    }

    int create(const fdtd_domain_desc* dom, const fdtd_stream_options* o) {
        so = *o;
        g = *dom;
        st = (hipStream_t)o->stream;
        if (o->slab_planes < 1 || o->steps_per_pass < 1 || o->max_steps < 0)
            return fail(FDTD_E_INVALID, "slab_planes and steps_per_pass must be >= 1, max_steps >= 0");
        adj = g.grad != 0;
        if (adj && o->max_steps < 1) return fail(FDTD_E_INVALID, "a streamed gradient needs max_steps >= 1");
        // admission of the domain itself: validate it as a resident handle would, without allocating
        {
            Handle<T> gh;
            gh.size_only = true;
            fdtd_options go = slab_options();
            int rc = gh.create(dom, 1, &go);
            if (rc) return fail(rc, gh.err);
            resident_bytes = (double)gh.pool_bytes;
            pitch = gh.dd[0].pitch;
            gncomp = gh.dh[0].gncomp;
            gelems = gh.dh[0].gelems;
            ncomp_eps = gh.dh[0].ncomp_eps;
            npole = gh.dd[0].has_lor ? gh.dd[0].npole : 0;
            // keep the waveforms and frequencies: the descriptor's pointers are the caller's
            waves.resize(g.n_sources);
            for (int q = 0; q < g.n_sources; ++q) {
                waves[q] = gh.dh[0].waves[q];
                g.sources[q].waveform = waves[q].data();
            }
            omegas.resize(g.n_monitors);
            for (int q = 0; q < g.n_monitors; ++q) {
                omegas[q] = gh.dh[0].mons[q].omega;
                g.monitors[q].omega_dt = omegas[q].empty() ? nullptr : omegas[q].data();
            }
            ebox = 1;
            for (int a = 0; a < 3; ++a) ebox *= (size_t)(g.eps_hi[a] - g.eps_lo[a]);
            if (!g.eps) ebox = 0;
            if (ebox) {
                ez0 = g.eps_lo[2];
                ez1 = g.eps_hi[2];
                // planes of the stored layout (rows of exs elements), the slabs' layout too
                eplane = (size_t)(g.eps_hi[1] - g.eps_lo[1]) * gh.dd[0].exs;
                egeom = gh.dd[0];
            }
        }
        const double* eps_in = g.eps;   // read once below, after admission; not kept
        g.eps = nullptr;
        nx = g.n[0];
        ny = g.n[1];
        nz = g.n[2];
        K = o->steps_per_pass;
        halo = K + 1;
        // cores: nz split into ceil(nz / W) near-equal parts
        const int nsl = (nz + o->slab_planes - 1) / o->slab_planes;
        core.assign(nsl + 1, 0);
        for (int s = 0; s < nsl; ++s) core[s + 1] = core[s] + nz / nsl + (s < nz % nsl ? 1 : 0);
        const int lz0 = g.pml[4], lz1 = g.pml[5];
        for (int s = 0; s < nsl; ++s) {
            const int lo = ext_lo(s), hi = ext_hi(s);
            if ((lo > 0 && lo < lz0) || (hi < nz && hi > nz - lz1)) {
                char b[200];
                snprintf(b, sizeof b, "slab %d spans planes [%d, %d), cutting an absorbing z face: slab_planes must "
                                      "exceed the face depth plus steps_per_pass + 1", s, lo, hi);
                return fail(FDTD_E_INVALID, b);
            }
        }
        // monitors: each belongs to the slab whose core holds its plane
        gm.assign(g.n_monitors, GMon{});
        size_t moff = 0;
        for (int q = 0; q < g.n_monitors; ++q) {
            const fdtd_monitor_desc& md = g.monitors[q];
            GMon& m = gm[q];
            m.kind = md.kind == FDTD_MON_PROBE ? 0 : (md.kind == FDTD_MON_FLUX_Z ? 1 : 2);
            m.k = md.pos[2];
            m.slab = 0;
            while (m.k >= core[m.slab + 1]) ++m.slab;
            m.nf = m.kind ? md.n_freq : 0;
            m.npts = m.kind ? (long long)(md.rect[1] - md.rect[0]) * (md.rect[3] - md.rect[2]) : 0;
            m.elems = m.kind ? (size_t)m.nf * (m.kind == 1 ? 4 : 1) * m.npts * 2 : (size_t)std::max(1, so.max_steps);
            moff = align256(moff) + m.elems * 8;
            if (m.kind == 1) moff = align256(moff) + (size_t)m.nf * flux_blocks(m.npts) * 8 + 256 + (size_t)m.nf * 8;
        }
        dmon_bytes = align256(moff) + 256;
        // global state arrays, in the slab handles' order
        size_t off = 0;
        auto add = [&](int kind, int c, int a, int side, int r, int w, int p, int z0, int z1, size_t per) {
            GArr q{kind, c, a, side, r, w, p, z0, z1, per, off};
            off += (size_t)(z1 - z0) * per;
            ga.push_back(q);
        };
        for (int c = 0; c < 6; ++c) add(0, c, 0, 0, 0, 0, 0, 0, nz, (size_t)ny * pitch);
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                const int L = g.pml[2 * a + side];
                if (!L) continue;
                for (int r = 0; r < 2; ++r)
                    for (int kind = 1; kind <= 2; ++kind) {
                        if (a == 0) add(kind, 0, a, side, r, 0, 0, 0, nz, (size_t)ny * L);
                        else if (a == 1) add(kind, 0, a, side, r, 0, 0, 0, nz, (size_t)L * nx);
                        else add(kind, 0, a, side, r, 0, 0, side ? nz - L : 0, side ? nz : L, (size_t)ny * nx);
                    }
            }
        if (g.n_lorentz) {
            const fdtd_lorentz_desc& L = g.lorentz;
            const size_t per = (size_t)(L.hi[0] - L.lo[0]) * (L.hi[1] - L.lo[1]);
            for (int w = 0; w < 3; ++w)
                for (int c = 0; c < 3; ++c)
                    for (int p = 0; p < (w == 0 ? 1 : npole); ++p) add(3, c, 0, 0, 0, w, p, L.lo[2], L.hi[2], per);
        }
        bank_elems = off;
        // the workspace: the largest slab's pool, forward or (with a gradient)
        // reverse, where a block's K forward states are kept for its K
        // transposed steps
        for (int rev = 0; rev <= (adj ? 1 : 0); ++rev)
            for (int s = 0; s < nsl; ++s) {
                std::vector<int> lm;
                fdtd_domain_desc d = slab_desc(s, lm, rev != 0);
                Handle<T> sh;
                sh.size_only = true;
                sh.external_eps = true;
                fdtd_options so2 = slab_options(rev ? local_slots() : 0);
                int rc = sh.create(&d, 1, &so2);
                if (rc) return fail(rc, "slab " + std::to_string(s) + ": " + sh.err);
                pool_cap = std::max(pool_cap, sh.pool_bytes);
            }
        const int npass = (so.max_steps + K - 1) / K;
        if (o->host_banks != 0 && o->host_banks < 4)
            return fail(FDTD_E_INVALID, "host_banks must be 0 or at least 4");
        bounded = adj && o->host_banks >= 4 && o->host_banks < npass + 1;
        const int nbank = adj ? (bounded ? o->host_banks : npass + 1) : 2;
        if (bounded) {
            // the forward keeps the binomial descent over [0, npass): with s
            // slots (the one at a included) advance m = max(1, l - beta(s-1, r),
            // beta(s, r-2)) passes, keep that boundary, one slot fewer; B - 4 of
            // them, so that the reverse always has two free banks to advance with
            planned.assign(npass + 1, 0);
            int a = 0, s_ = nbank - 3;
            while (npass - a > 1 && s_ > 1) {
                const int l = npass - a;
                int r = 0;
                while (beta(s_, r) < l) ++r;
                a += (int)std::max<long long>(1, std::max<long long>(l - beta(s_ - 1, r), beta(s_, r - 2)));
                planned[a] = 1;
                --s_;
            }
        }
        // admission: device workspaces + accumulators, host banks
        nws = o->overlap ? 2 : 1;
        const size_t est = ebox ? eplane * (size_t)(ez1 - ez0) : 0;   // stored elements per component
        const double dev = (double)(nws * pool_cap + dmon_bytes),
                     host = (double)(nbank + (adj ? 2 : 0)) * bank_elems * sizeof(T) +
                            (double)est * ncomp_eps * sizeof(T) + (adj ? 8.0 * gncomp * gelems : 0.0);
        double budget = o->mem_budget_bytes;
        if (budget <= 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(FDTD_E_DEVICE, "hipMemGetInfo failed");
            budget = (double)fr - 256.0 * 1024 * 1024;
        }
        char b[240];
        if (dev > budget) {
            snprintf(b, sizeof b, "streamed workspace %.3e B exceeds the device budget %.3e B", dev, budget);
            return fail(FDTD_E_NOMEM, b);
        }
        if (o->host_budget_bytes > 0 && host > o->host_budget_bytes) {
            snprintf(b, sizeof b, "host state banks and eps^-1 %.3e B exceed the host budget %.3e B", host,
                     o->host_budget_bytes);
            return fail(FDTD_E_NOMEM, b);
        }
        if (ebox) {
            // eps^-1 in the field type and the stored row layout, as the resident upload computes it
            std::vector<T> v;
            Handle<T>::einv_rows(egeom, ncomp_eps, eps_in, g.eps_bg, v);
            if (hipHostMalloc((void**)&einv, v.size() * sizeof(T), 0) != hipSuccess) {
                (void)hipGetLastError();
                einv = nullptr;
                return fail(FDTD_E_NOMEM, "pinned host allocation of the material arrays failed");
            }
            std::memcpy(einv, v.data(), v.size() * sizeof(T));
        }
        for (int k = 0; k < nws; ++k)
            if (hipMalloc((void**)&pool[k], pool_cap) != hipSuccess ||
                hipStreamCreateWithFlags(&wst[k], hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                return fail(FDTD_E_NOMEM, "device allocation of the streamed workspace failed");
            }
        if (hipMalloc((void**)&dmon, dmon_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FDTD_E_NOMEM, "device allocation of the monitor accumulators failed");
        }
        // eps^-1 stays on the device when the budget holds it beside the
        // workspaces: each visit then copies its planes device to device
        const size_t ebytes = est * ncomp_eps * sizeof(T);
        if (ebox && dev + (double)ebytes <= budget) {
            if (hipMalloc((void**)&d_einv, ebytes) != hipSuccess) {
                (void)hipGetLastError();
                d_einv = nullptr;
            } else if (hipMemcpy(d_einv, einv, ebytes, hipMemcpyHostToDevice) != hipSuccess) {
                return fail(FDTD_E_DEVICE, "eps^-1 upload failed");
            }
        }
        bank.assign(nbank, nullptr);
        for (int k = 0; k < nbank + (adj ? 2 : 0); ++k) {
            T*& b = k < nbank ? bank[k] : abank[k - nbank];
            if (hipHostMalloc((void**)&b, std::max<size_t>(bank_elems, 1) * sizeof(T), 0) != hipSuccess) {
                (void)hipGetLastError();
                b = nullptr;
                return fail(FDTD_E_NOMEM, "pinned host allocation of the state banks failed");
            }
        }
        if (adj) {
            grad.assign((size_t)gncomp * gelems, 0.0);
            cots.resize(g.n_monitors);
            cot_set.assign(g.n_monitors, 0);
        }
        moff = 0;
        for (auto& m : gm) {
            moff = align256(moff);
            m.acc = (double*)(dmon + moff);
            moff += m.elems * 8;
            if (m.kind == 1) {
                moff = align256(moff);
                m.fpart = (double*)(dmon + moff);
                moff += (size_t)m.nf * flux_blocks(m.npts) * 8;
                moff = align256(moff);
                m.fout = (double*)(dmon + moff);
                moff += (size_t)m.nf * 8;
            }
        }
        return reset();
    }

    int reset() override {
        if (int rc = drain()) return rc;
        std::memset(bank[0], 0, bank_elems * sizeof(T));   // the state at time 0; later banks are written whole
        cb = 0;
        cur_id = 0;
        if (bounded) {
            snap.assign(planned.size(), -1);
            snap[0] = 0;
        }
        t = 0;
        grad_step = -1;
        launch_zero(dmon, dmon_bytes, st);
        if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
            return fail(FDTD_E_DEVICE, "stream reset failed");
        return FDTD_OK;
    }

    // Waits for both workspaces and releases their slab handles.
    int drain() {
        for (int k = 0; k < 2; ++k) hs[k].reset();   // a handle's destructor waits for its stream
        for (int k = 0; k < nws; ++k)
            if (wst[k] && hipStreamSynchronize(wst[k]) != hipSuccess) return fail(FDTD_E_DEVICE, "slab stream failed");
        if (hipGetLastError() != hipSuccess) return fail(FDTD_E_DEVICE, "slab pass failed");
        return FDTD_OK;
    }

    // One slab's visit, queued on its workspace's stream: load its extent at
    // time t from bank cb, step n, store its core to the other bank, fold its
    // monitors into the domain's.  The previous slab of that workspace is
    // waited for (its handle released) first; the other workspace's slab keeps
    // running meanwhile.
    int run_slab(int s, int n, T* src_bank, T* dst_bank, int t_start = -1, bool record = true) {
        const int o = ext_lo(s), e = ext_hi(s), c0 = core[s], c1 = core[s + 1];
        const int w = s % nws;
        hs[w].reset();
        std::vector<int> lm;
        fdtd_domain_desc d = slab_desc(s, lm);
        hs[w].reset(new Handle<T>());
        Handle<T>& hd = *hs[w];
        hd.external_eps = true;
        hd.ext_pool = pool[w];
        hd.ext_cap = pool_cap;
        fdtd_options so2 = slab_options();
        so2.stream = wst[w];
        hipStream_t st = wst[w];
        int rc = hd.create(&d, 1, &so2);
        if (rc) return fail(rc, "slab " + std::to_string(s) + ": " + hd.err);
        hd.t = t_start < 0 ? t : t_start;
        const DomDev<T>& dv = hd.dd[0];
        // eps^-1 of the slab's share of the eps box
        if (ebox && dv.elo[2] < dv.ehi[2]) {
            const int z0 = dv.elo[2] + o, z1 = dv.ehi[2] + o;
            for (int c = 0; c < ncomp_eps; ++c) {
                T* dst = ncomp_eps == 6 ? const_cast<T*>(dv.tinv[c]) : const_cast<T*>(dv.epsinv[c]);
                const size_t q0 = c * eplane * (size_t)(ez1 - ez0) + (size_t)(z0 - ez0) * eplane;
                if (hipMemcpyAsync(dst, d_einv ? d_einv + q0 : einv + q0, (size_t)(z1 - z0) * eplane * sizeof(T),
                                   d_einv ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "slab eps upload failed");
            }
        }
        // state at time t over the extent, n steps, the core at time t + n
        if ((rc = xfer(hd, src_bank, true, o, e, c0, c1, st))) return rc;
        if ((rc = hd.step_forward(n, record ? FDTD_RECORD : FDTD_REPLAY))) return fail(rc, hd.err);
        if ((rc = xfer(hd, dst_bank, false, o, e, c0, c1, st))) return rc;
        for (size_t li = 0; record && li < lm.size(); ++li) {
            MonHost& mh = hd.dh[0].mons[li];
            hd.flush(mh);
            GMon& m = gm[lm[li]];
            launch_add_f64(m.acc, m.kind ? mh.dev.acc : mh.dev.trace, m.elems, st);
        }
        if (hipGetLastError() != hipSuccess) return fail(FDTD_E_DEVICE, "slab launch failed");
        return FDTD_OK;
    }

    // bank holding the state at time t
    int cur_bank() const { return bounded ? cur_id : (adj ? (t + K - 1) / K : cb); }

    // banks holding neither the state at time t nor a snapshot (bounded mode)
    std::vector<int> free_banks() const {
        std::vector<char> used(bank.size(), 0);
        used[cur_id] = 1;
        for (int b : snap)
            if (b >= 0) used[b] = 1;
        std::vector<int> f;
        for (int q = 0; q < (int)bank.size(); ++q)
            if (!used[q]) f.push_back(q);
        return f;
    }

    // checkpoint slots a slab keeps while it reverses a block
    int local_slots() const { return so.local_slots > 0 ? std::min(so.local_slots, K) : K; }

    // Binomial checkpointing of one block (Griewank's rule, as in the
    // package's revolve.py): beta(s, r) = C(s + r, s); to reverse [a, b)
    // holding u^a in slot sa, advance m = max(1, l - beta(s-1, r),
    // beta(s, r-2)) steps (r the fewest repetitions with beta(s, r) >= l),
    // keep u^{a+m}, reverse [a+m, b) with one slot fewer, then [a, a+m).
    static long long beta(int s_, int r) {
        if (r < 0 || s_ < 0) return 0;
        long long c = 1;
        for (int q = 1; q <= s_; ++q) c = c * (r + q) / q;
        return c;
    }

    int rev_block(Handle<T>& hd, int a, int b, int sa, std::vector<int>& free_slots, int& at) {
        int rc;
        auto go = [&](int pos) -> int {
            if (at == pos) return FDTD_OK;
            if ((rc = hd.ckpt_restore(sa))) return fail(rc, hd.err);
            at = pos;
            return FDTD_OK;
        };
        auto adv = [&](int k) -> int {
            if (k <= 0) return FDTD_OK;
            if ((rc = hd.step_forward(k, FDTD_REPLAY))) return fail(rc, hd.err);
            at += k;
            return FDTD_OK;
        };
        const int l = b - a;
        if ((rc = go(a))) return rc;
        if (l == 1) return (rc = hd.step_adjoint(1)) ? fail(rc, hd.err) : FDTD_OK;
        const int s_ = (int)free_slots.size() + 1;
        if (s_ == 1) {
            for (int k = b - 1; k >= a; --k) {
                if ((rc = go(a)) || (rc = adv(k - a))) return rc;
                if ((rc = hd.step_adjoint(1))) return fail(rc, hd.err);
            }
            return FDTD_OK;
        }
        int r = 0;
        while (beta(s_, r) < l) ++r;
        const int m = (int)std::max<long long>(1, std::max<long long>(l - beta(s_ - 1, r), beta(s_, r - 2)));
        if ((rc = adv(m))) return rc;
        const int slot = free_slots.back();
        free_slots.pop_back();
        if ((rc = hd.ckpt_save(slot))) return fail(rc, hd.err);
        if ((rc = rev_block(hd, a + m, b, slot, free_slots, at))) return rc;
        free_slots.push_back(slot);
        return rev_block(hd, a, a + m, sa, free_slots, at);
    }

    int step(int n) override {
        if (n < 0) return fail(FDTD_E_INVALID, "negative step count");
        if (adj && n > 0 && (t % K != 0 || t + n > so.max_steps))
            return fail(FDTD_E_STATE, "with a gradient, passes are K steps long except the last one, within "
                                      "max_steps");
        while (n > 0) {
            const int kp = std::min(n, K);
            int did = -1;
            if (bounded) {
                const std::vector<int> f = free_banks();
                did = f.front();   // two or more are free: B - 4 planned snapshots, time 0, time t
            }
            T* src = bank[cur_bank()];
            T* dst = bank[bounded ? did : (adj ? t / K + 1 : cb ^ 1)];
            for (int s = 0; s < ns(); ++s) {
                int rc = run_slab(s, kp, src, dst);
                if (rc) {
                    drain();
                    return rc;
                }
            }
            if (int rc = drain()) return rc;   // the next bank complete before it is read
            cb ^= 1;
            t += kp;
            n -= kp;
            if (bounded) {
                cur_id = did;
                if (t % K == 0 && planned[t / K]) snap[t / K] = did;   // kept for the reverse sweep
            }
        }
        grad_step = -1;
        return FDTD_OK;
    }

    // ---------------------------------------------------------- reverse sweep
    // The transposed steps are local like the forward ones (each reads its
    // neighbours one plane away, in the other direction), so the same slabs
    // and halos serve the reverse sweep, block by block from the last: for
    // each slab, the block's starting state (bank j) is replayed forward K
    // steps in the workspace with every state kept, the cotangent state at
    // the block's end is loaded over the extent, and K transposed steps run
    // with the monitor seeds of every monitor plane in the extent; the core's
    // cotangent state goes to the other cotangent bank and the core's dJ/deps
    // is added to the domain's.  The forward states and cotangents of the
    // core are exact, so its gradient terms are those of the resident sweep.
    int set_cotangent(int mon, const double* buf, size_t bytes) override {
        if (!adj) return fail(FDTD_E_STATE, "the domain takes no gradient");
        if (mon < 0 || mon >= (int)gm.size()) return fail(FDTD_E_RANGE, "monitor index");
        const size_t ne = gm[mon].elems;
        if (gm[mon].kind && bytes < ne * 8) return fail(FDTD_E_RANGE, "buffer too small for cotangents");
        cots[mon].assign(ne, 0.0);
        std::memcpy(cots[mon].data(), buf, std::min(bytes / 8, ne) * 8);
        cot_set[mon] = 1;
        return FDTD_OK;
    }

    int run_slab_reverse(int s, int t0, int kb, int N, T* fstart, T* cot_in, T* cot_out) {
        const int o = ext_lo(s), e = ext_hi(s), c0 = core[s], c1 = core[s + 1];
        const int w = s % nws;
        hs[w].reset();
        std::vector<int> lm;
        fdtd_domain_desc d = slab_desc(s, lm, true);
        hs[w].reset(new Handle<T>());
        Handle<T>& hd = *hs[w];
        hd.external_eps = true;
        hd.ext_pool = pool[w];
        hd.ext_cap = pool_cap;
        const int L = std::min(local_slots(), kb);
        fdtd_options so2 = slab_options(local_slots());
        so2.stream = wst[w];
        hipStream_t st = wst[w];
        int rc = hd.create(&d, 1, &so2);
        if (rc) return fail(rc, "slab " + std::to_string(s) + ": " + hd.err);
        hd.t = t0;
        const DomDev<T>& dv = hd.dd[0];
        if (ebox && dv.elo[2] < dv.ehi[2]) {
            const int z0 = dv.elo[2] + o, z1 = dv.ehi[2] + o;
            for (int c = 0; c < ncomp_eps; ++c) {
                T* dst = ncomp_eps == 6 ? const_cast<T*>(dv.tinv[c]) : const_cast<T*>(dv.epsinv[c]);
                const size_t q0 = c * eplane * (size_t)(ez1 - ez0) + (size_t)(z0 - ez0) * eplane;
                if (hipMemcpyAsync(dst, d_einv ? d_einv + q0 : einv + q0, (size_t)(z1 - z0) * eplane * sizeof(T),
                                   d_einv ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "slab eps upload failed");
            }
        }
        // the block's starting state u^t0 in slot 0
        if ((rc = xfer(hd, fstart, true, o, e, c0, c1, st))) return rc;
        if ((rc = hd.ckpt_save(0))) return fail(rc, hd.err);
        // cotangent state at t0 + kb (its seeds included), then kb transposed
        // steps, the forward states regenerated from the block's slots
        hd.ap = 0;
        hd.m = t0 + kb;
        if ((rc = xfer(hd, cot_in, true, o, e, c0, c1, st, true, 0))) return rc;
        for (size_t li = 0; li < lm.size(); ++li) {
            if (!cot_set[lm[li]]) continue;
            std::vector<double>& cv = cots[lm[li]];
            if ((rc = hd.monitor(0, (int)li, FDTD_MON_SET_COTANGENT, cv.data(), cv.size() * 8)))
                return fail(rc, hd.err);
        }
        if (t0 + kb == N && (rc = hd.seed(N))) return fail(rc, hd.err);
        {
            std::vector<int> free_slots;
            for (int q = L - 1; q >= 1; --q) free_slots.push_back(q);
            int at = t0;
            if ((rc = rev_block(hd, t0, t0 + kb, 0, free_slots, at))) return rc;
        }
        if ((rc = xfer(hd, cot_out, false, o, e, c0, c1, st, true, hd.ap))) return rc;
        // dJ/deps of the core's gradient planes, added to the domain's on the host
        const int gz0 = std::max(g.grad_lo[2], c0), gz1 = std::min(g.grad_hi[2], c1);
        if (gz1 > gz0 && gelems) {
            const size_t gpl = (size_t)(g.grad_hi[0] - g.grad_lo[0]) * (g.grad_hi[1] - g.grad_lo[1]);
            std::vector<double> tmp((size_t)(gz1 - gz0) * gpl);
            const int lz0 = dv.glo[2] + o;   // the slab's gradient box starts at this plane
            for (int c = 0; c < gncomp; ++c) {
                if (hipMemcpyAsync(tmp.data(), dv.gacc[c] + (size_t)(gz0 - lz0) * gpl, tmp.size() * 8,
                                   hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    return fail(FDTD_E_DEVICE, "gradient download failed");
                double* gg = grad.data() + c * gelems + (size_t)(gz0 - g.grad_lo[2]) * gpl;
                for (size_t q = 0; q < tmp.size(); ++q) gg[q] += tmp[q];
            }
        }
        if (hipGetLastError() != hipSuccess) return fail(FDTD_E_DEVICE, "slab launch failed");
        return FDTD_OK;
    }

    // Reverse the block of pass p, whose starting state is in bank bid.
    int run_block(int p, int bid, int N, int& ab) {
        const int t0 = p * K, kb = std::min(K, N - t0);
        for (int s = 0; s < ns(); ++s) {
            int rc = run_slab_reverse(s, t0, kb, N, bank[bid], abank[ab], abank[ab ^ 1]);
            if (rc) {
                drain();
                return rc;
            }
        }
        if (int rc = drain()) return rc;
        ab ^= 1;
        return FDTD_OK;
    }

    // Streamed forward passes a -> m (full K-step passes, no monitors) from
    // bank src; the state lands in bank x, y the other of the ping-pong pair.
    int advance(int src, int a, int m, int x, int y) {
        const int q = m - a;
        int from = src, to = (q % 2) ? x : y;
        for (int p = a; p < m; ++p) {
            for (int s = 0; s < ns(); ++s) {
                int rc = run_slab(s, K, bank[from], bank[to], p * K, false);
                if (rc) {
                    drain();
                    return rc;
                }
            }
            if (int rc = drain()) return rc;
            ++replay_passes;
            from = to;
            to = to == x ? y : x;
        }
        return FDTD_OK;
    }

    // Bounded banks: reverse passes [a, b) holding u at boundary a in snap[a].
    // A snapshot inside (a, b) splits the range (the largest first);
    // otherwise, with s = free banks - 1 slots, the binomial rule picks the
    // boundary m to regenerate and keep (s = 1: each block start regenerated
    // from a in turn).
    int rev_passes(int a, int b, int N, int& ab) {
        int rc;
        if (b - a == 1) return run_block(a, snap[a], N, ab);
        int m = -1;
        for (int p = b - 1; p > a; --p)
            if (snap[p] >= 0) {
                m = p;
                break;
            }
        if (m < 0) {
            const std::vector<int> f = free_banks();
            const int s_ = (int)f.size() - 1;
            if (s_ <= 1) {
                for (int c = b - 1; c > a; --c) {
                    if ((rc = advance(snap[a], a, c, f[0], f[1]))) return rc;
                    if ((rc = run_block(c, f[0], N, ab))) return rc;
                }
                return run_block(a, snap[a], N, ab);
            }
            const int l = b - a;
            int r = 0;
            while (beta(s_, r) < l) ++r;
            m = a + (int)std::max<long long>(1, std::max<long long>(l - beta(s_ - 1, r), beta(s_, r - 2)));
            if ((rc = advance(snap[a], a, m, f[0], f[1]))) return rc;
            snap[m] = f[0];
        }
        if ((rc = rev_passes(m, b, N, ab))) return rc;
        snap[m] = -1;
        return rev_passes(a, m, N, ab);
    }

    int reverse() override {
        if (!adj) return fail(FDTD_E_STATE, "the domain takes no gradient");
        const int N = t;
        if (N < 1) return fail(FDTD_E_STATE, "no forward steps to reverse");
        std::fill(grad.begin(), grad.end(), 0.0);
        std::memset(abank[0], 0, bank_elems * sizeof(T));
        int ab = 0;
        replay_passes = 0;
        if (bounded) {
            if (int rc = rev_passes(0, (N + K - 1) / K, N, ab)) return rc;
            grad_step = N;
            return FDTD_OK;
        }
        for (int j = (N - 1) / K; j >= 0; --j) {
            const int t0 = j * K, kb = std::min(K, N - t0);
            for (int s = 0; s < ns(); ++s) {
                int rc = run_slab_reverse(s, t0, kb, N, bank[j], abank[ab], abank[ab ^ 1]);
                if (rc) {
                    drain();
                    return rc;
                }
            }
            if (int rc = drain()) return rc;
            ab ^= 1;
        }
        grad_step = N;
        return FDTD_OK;
    }

    int get_grad(double* buf, size_t bytes) override {
        if (!adj) return fail(FDTD_E_STATE, "the domain takes no gradient");
        if (grad_step < 0) return fail(FDTD_E_STATE, "no reverse sweep since the last forward steps");
        if (bytes < grad.size() * 8) return fail(FDTD_E_RANGE, "buffer too small for the gradient");
        std::memcpy(buf, grad.data(), grad.size() * 8);
        return FDTD_OK;
    }

    int get_field(int comp, void* buf, size_t bytes) override {
        if (comp < 0 || comp > 5) return fail(FDTD_E_RANGE, "component");
        if (bytes < (size_t)nx * ny * nz * sizeof(T)) return fail(FDTD_E_RANGE, "buffer too small for field");
        const T* src = bank[cur_bank()] + ga[comp].off;
        T* out = (T*)buf;
        for (size_t r = 0; r < (size_t)ny * nz; ++r) std::memcpy(out + r * nx, src + r * pitch, nx * sizeof(T));
        return FDTD_OK;
    }

    int monitor(int mon, int op, double* buf, size_t bytes) override {
        if (mon < 0 || mon >= (int)gm.size()) return fail(FDTD_E_RANGE, "monitor index");
        GMon& m = gm[mon];
        if (op == FDTD_MON_GET) {
            if (bytes < m.elems * 8 && m.kind) return fail(FDTD_E_RANGE, "buffer too small for spectra");
            const size_t nb = std::min(bytes / 8, m.elems) * 8;
            if (hipMemcpyAsync(buf, m.acc, nb, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "monitor copy failed");
            return FDTD_OK;
        }
        if (op == FDTD_MON_FLUX) {
            if (m.kind != 1) return fail(FDTD_E_INVALID, "flux needs a flux monitor");
            if (bytes < (size_t)m.nf * 8) return fail(FDTD_E_RANGE, "buffer too small for flux");
            launch_flux(m.acc, m.nf, m.npts, m.fpart, m.fout, st);
            if (hipMemcpyAsync(buf, m.fout, (size_t)m.nf * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return fail(FDTD_E_DEVICE, "flux failed");
            return FDTD_OK;
        }
        return fail(FDTD_E_INVALID, "monitor op (GET or FLUX)");
    }

    void info(fdtd_stream_info* out) override {
        out->n_slabs = ns();
        out->halo = halo;
        int mx = 0;
        for (int s = 0; s < ns(); ++s) mx = std::max(mx, ext_hi(s) - ext_lo(s));
        out->max_extent = mx;
        out->step = t;
        const double est = ebox ? (double)eplane * (ez1 - ez0) : 0.0;   // stored eps^-1 elements per component
        out->device_bytes = (double)(nws * pool_cap + dmon_bytes) + (d_einv ? est * ncomp_eps * sizeof(T) : 0.0);
        out->host_bytes = (double)(bank.size() + (adj ? 2 : 0)) * bank_elems * sizeof(T) +
                          est * ncomp_eps * sizeof(T) + 8.0 * grad.size();
        out->resident_bytes = resident_bytes;
        out->materials_resident = d_einv ? 1 : 0;
        out->replay_passes = replay_passes;
    }
};

}  // namespace

struct fdtd_stream_s {
    std::unique_ptr<StreamBase> impl;
};

struct fdtd_s {
    std::unique_ptr<Base> impl;
};

namespace {
int guard(fdtd_t h) {
    if (!h || !h->impl) return FDTD_E_INVALID;
    if (h->impl->poisoned) return FDTD_E_DEVICE;
    return FDTD_OK;
}
}  // namespace

#define GUARD(h)                \
    do {                        \
        int _g = guard(h);      \
        if (_g) return _g;      \
    } while (0)

extern "C" {

int fdtd_create(const fdtd_domain_desc* domains, int32_t n_domains, const fdtd_options* opt, fdtd_t* out) {
    if (!out) return FDTD_E_INVALID;
    *out = nullptr;
    if (!domains || n_domains < 1 || !opt) {
        g_create_error = "null descriptor or n_domains < 1";
        return FDTD_E_INVALID;
    }
    if (opt->dtype != FDTD_F32 && opt->dtype != FDTD_F64) {
        g_create_error = "dtype must be FDTD_F32 or FDTD_F64";
        return FDTD_E_INVALID;
    }
    std::unique_ptr<fdtd_s> h(new fdtd_s);
    if (opt->dtype == FDTD_F32) h->impl.reset(new Handle<float>());
    else h->impl.reset(new Handle<double>());
    int rc;
    if (opt->dtype == FDTD_F32) rc = static_cast<Handle<float>*>(h->impl.get())->create(domains, n_domains, opt);
    else rc = static_cast<Handle<double>*>(h->impl.get())->create(domains, n_domains, opt);
    if (rc) {
        g_create_error = h->impl->err;
        return rc;
    }
    *out = h.release();
    return FDTD_OK;
}

int fdtd_destroy(fdtd_t h) {
    if (!h) return FDTD_E_INVALID;
    delete h;
    return FDTD_OK;
}

int fdtd_step_forward(fdtd_t h, int32_t n_steps, uint32_t flags) {
    GUARD(h);
    return h->impl->step_forward(n_steps, flags);
}

int fdtd_adjoint_begin(fdtd_t h, int32_t n_total) {
    GUARD(h);
    return h->impl->adjoint_begin(n_total);
}

int fdtd_step_adjoint(fdtd_t h, int32_t n_steps) {
    GUARD(h);
    return h->impl->step_adjoint(n_steps);
}

int fdtd_step_reverse(fdtd_t h, int32_t n_steps) {
    GUARD(h);
    return h->impl->step_reverse(n_steps);
}

int fdtd_checkpoint_save(fdtd_t h, int32_t slot) {
    GUARD(h);
    return h->impl->ckpt_save(slot);
}

int fdtd_checkpoint_restore(fdtd_t h, int32_t slot) {
    GUARD(h);
    return h->impl->ckpt_restore(slot);
}

int fdtd_monitor_dft(fdtd_t h, int32_t domain, int32_t monitor, int32_t op, void* host_buf, size_t bytes) {
    GUARD(h);
    if (!host_buf && op != FDTD_MON_RESET) return FDTD_E_INVALID;
    return h->impl->monitor(domain, monitor, op, host_buf, bytes);
}

int fdtd_get_field(fdtd_t h, int32_t domain, int32_t comp, void* host_buf, size_t bytes) {
    GUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->get_field(domain, comp, host_buf, bytes, false);
}

int fdtd_set_field(fdtd_t h, int32_t domain, int32_t comp, const void* host_buf, size_t bytes) {
    GUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->get_field(domain, comp, (void*)host_buf, bytes, true);
}

int fdtd_get_grad(fdtd_t h, int32_t domain, double* host_buf, size_t bytes) {
    GUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->get_grad(domain, host_buf, bytes);
}

int fdtd_set_eps(fdtd_t h, int32_t domain, const double* eps, size_t bytes) {
    GUARD(h);
    if (!eps) return FDTD_E_INVALID;
    return h->impl->set_eps(domain, eps, bytes);
}

int fdtd_reset(fdtd_t h) {
    GUARD(h);
    return h->impl->reset();
}

int fdtd_get_step(fdtd_t h, int32_t* fwd_n, int32_t* adj_m) {
    GUARD(h);
    int n = 0, m = 0;
    h->impl->steps(&n, &m);
    if (fwd_n) *fwd_n = n;
    if (adj_m) *adj_m = m;
    return FDTD_OK;
}

int fdtd_probe_trace(fdtd_t h, int32_t domain, int32_t probe, double* host_buf, int32_t n) {
    GUARD(h);
    if (!host_buf || n < 0) return FDTD_E_INVALID;
    return h->impl->probe_trace(domain, probe, host_buf, n);
}

int fdtd_field_energy(fdtd_t h, int32_t domain, double* energy) {
    GUARD(h);
    if (!energy) return FDTD_E_INVALID;
    return h->impl->energy(domain, energy);
}

int fdtd_get_memory(fdtd_t h, double* bytes) {
    GUARD(h);
    if (bytes) *bytes = h->impl->memory();
    return FDTD_OK;
}

int fdtd_checkpoint_corrupt(fdtd_t h, int32_t slot, size_t word, uint32_t value) {
    GUARD(h);
    return h->impl->poke_slot(slot, word, value);
}

int fdtd_kernel_timing(fdtd_t h, int32_t op, double* total_ms, int64_t* launches) {
    GUARD(h);
    long long n = 0;
    int rc = h->impl->timing(op, total_ms, &n);
    if (launches) *launches = n;
    return rc;
}

int fdtd_copy_probe(size_t bytes, int32_t reps, double* ms_per_copy) {
    if (bytes == 0 || bytes % 4 || reps < 1 || !ms_per_copy) return FDTD_E_INVALID;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return FDTD_E_NOMEM;
    }
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(a);
        return FDTD_E_NOMEM;
    }
    hipEvent_t e0, e1;
    int rc = FDTD_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = FDTD_E_DEVICE;
    if (!rc) {
        launch_zero(a, bytes, nullptr);
        launch_copy(a, b, bytes, nullptr);   // warm-up
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r) launch_copy(a, b, bytes, nullptr);
        (void)hipEventRecord(e1, nullptr);
        float ms = 0;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = FDTD_E_DEVICE;
        *ms_per_copy = ms / reps;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}

int fdtd_flux_reduce(const double* spectra, int32_t n_freq, int64_t n_pts, double* flux, void* workspace,
                     size_t workspace_bytes, void* stream) {
    if (!spectra || !flux || n_freq < 1 || n_pts < 1) {
        g_create_error = "fdtd_flux_reduce: null pointer, n_freq < 1 or n_pts < 1";
        return FDTD_E_INVALID;
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t need = (size_t)n_freq * flux_blocks(n_pts) * 8;
    void* part = workspace;
    const bool own = !workspace;
    if (own) {
        if (hipMalloc(&part, need) != hipSuccess) {
            (void)hipGetLastError();
            g_create_error = "fdtd_flux_reduce: workspace allocation failed";
            return FDTD_E_NOMEM;
        }
    } else if (workspace_bytes < need) {
        g_create_error = "fdtd_flux_reduce: workspace smaller than FDTD_FLUX_WORKSPACE_BYTES";
        return FDTD_E_RANGE;
    }
    launch_flux(spectra, n_freq, n_pts, (double*)part, flux, st);
    int rc = hipGetLastError() == hipSuccess ? FDTD_OK : FDTD_E_DEVICE;
    if (own) {
        if (hipStreamSynchronize(st) != hipSuccess) rc = FDTD_E_DEVICE;
        (void)hipFree(part);
    }
    if (rc) g_create_error = "fdtd_flux_reduce: HIP launch failed";
    return rc;
}

int fdtd_flux_reduce_noalloc(const double* spectra, int32_t n_freq, int64_t n_pts, double* flux, void* stream) {
    if (!spectra || !flux || n_freq < 1 || n_pts < 1) {
        g_create_error = "fdtd_flux_reduce_noalloc: null pointer, n_freq < 1 or n_pts < 1";
        return FDTD_E_INVALID;
    }
    if ((size_t)n_freq * flux_blocks(n_pts) * 8 > kFluxScratchBytes) {
        g_create_error = "fdtd_flux_reduce_noalloc: n_freq x blocks exceeds FDTD_FLUX_SCRATCH_BYTES";
        return FDTD_E_RANGE;
    }
    double* part = nullptr;
    if (flux_scratch(&part)) {
        g_create_error = "fdtd_flux_reduce_noalloc: no device address for the scratch array";
        return FDTD_E_DEVICE;
    }
    launch_flux(spectra, n_freq, n_pts, part, flux, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) {
        g_create_error = "fdtd_flux_reduce_noalloc: HIP launch failed";
        return FDTD_E_DEVICE;
    }
    return FDTD_OK;
}

// ---------------------------------------------------------------- streamed
namespace {
int sguard(fdtd_stream_t h) {
    if (!h || !h->impl) return FDTD_E_INVALID;
    if (h->impl->poisoned) return FDTD_E_DEVICE;
    return FDTD_OK;
}
}  // namespace

#define SGUARD(h)               \
    do {                        \
        int _g = sguard(h);     \
        if (_g) return _g;      \
    } while (0)

int fdtd_stream_create(const fdtd_domain_desc* domain, const fdtd_stream_options* opt, fdtd_stream_t* out) {
    if (!out) return FDTD_E_INVALID;
    *out = nullptr;
    if (!domain || !opt) {
        g_create_error = "null descriptor or options";
        return FDTD_E_INVALID;
    }
    if (opt->dtype != FDTD_F32 && opt->dtype != FDTD_F64) {
        g_create_error = "dtype must be FDTD_F32 or FDTD_F64";
        return FDTD_E_INVALID;
    }
    std::unique_ptr<fdtd_stream_s> h(new fdtd_stream_s);
    int rc;
    if (opt->dtype == FDTD_F32) {
        auto* p = new Streamer<float>();
        h->impl.reset(p);
        rc = p->create(domain, opt);
    } else {
        auto* p = new Streamer<double>();
        h->impl.reset(p);
        rc = p->create(domain, opt);
    }
    if (rc) {
        g_create_error = h->impl->err;
        return rc;
    }
    *out = h.release();
    return FDTD_OK;
}

int fdtd_stream_destroy(fdtd_stream_t h) {
    if (!h) return FDTD_E_INVALID;
    delete h;
    return FDTD_OK;
}

int fdtd_stream_step(fdtd_stream_t h, int32_t n_steps) {
    SGUARD(h);
    return h->impl->step(n_steps);
}

int fdtd_stream_get_field(fdtd_stream_t h, int32_t comp, void* host_buf, size_t bytes) {
    SGUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->get_field(comp, host_buf, bytes);
}

int fdtd_stream_monitor(fdtd_stream_t h, int32_t monitor, int32_t op, double* host_buf, size_t bytes) {
    SGUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->monitor(monitor, op, host_buf, bytes);
}

int fdtd_stream_set_cotangent(fdtd_stream_t h, int32_t monitor, const double* host_buf, size_t bytes) {
    SGUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->set_cotangent(monitor, host_buf, bytes);
}

int fdtd_stream_reverse(fdtd_stream_t h) {
    SGUARD(h);
    return h->impl->reverse();
}

int fdtd_stream_get_grad(fdtd_stream_t h, double* host_buf, size_t bytes) {
    SGUARD(h);
    if (!host_buf) return FDTD_E_INVALID;
    return h->impl->get_grad(host_buf, bytes);
}

int fdtd_stream_reset(fdtd_stream_t h) {
    SGUARD(h);
    return h->impl->reset();
}

int fdtd_stream_get_info(fdtd_stream_t h, fdtd_stream_info* out) {
    SGUARD(h);
    if (!out) return FDTD_E_INVALID;
    h->impl->info(out);
    return FDTD_OK;
}

const char* fdtd_stream_last_error(fdtd_stream_t h) {
    if (!h || !h->impl) return g_create_error.c_str();
    return h->impl->err.c_str();
}

const char* fdtd_last_error(fdtd_t h) {
    if (!h || !h->impl) return g_create_error.c_str();   // failing create or handle-free call
    return h->impl->err.c_str();
}

}  // extern "C"
