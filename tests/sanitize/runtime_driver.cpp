// Host memory-safety driver for libfdtd's admission paths (test
// infrastructure): built with the address and undefined-behaviour sanitizers
// on the host code only, it calls fdtd_create and fdtd_stream_create through
// the C-ABI with valid descriptors under a tiny budget (admitted, then refused
// with FDTD_E_NOMEM before any allocation) and with invalid ones (refused with
// their codes): the descriptor checks, the node-by-node tensor admission, the
// pole and permittivity bounds, the memory estimates and the streamed slab
// plan all run without a GPU.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fdtd.h"

namespace {

int failures = 0;

void expect(const char* what, int got, int want) {
    std::printf("%-58s %4d (want %4d)%s\n", what, got, want, got == want ? "" : "  MISMATCH");
    if (got != want) ++failures;
}

struct Dom {
    fdtd_domain_desc d;
    std::vector<double> eps, wave, omega;
};

// a small walled domain: absorbing faces, diagonal eps box, a two-pole box,
// two sources, a flux plane, a patch and a probe, a gradient box
void basic(Dom& m, int kind = FDTD_EPS_DIAG) {
    std::memset(&m.d, 0, sizeof m.d);
    fdtd_domain_desc& d = m.d;
    d.n[0] = 20;
    d.n[1] = 18;
    d.n[2] = 40;
    d.courant = 0.99 / std::sqrt(3.0);
    for (int q = 0; q < 6; ++q) d.pml[q] = 4;
    d.pml_m = 3;
    d.pml_kappa_max = 5;
    d.pml_sigma_max = 0.8 * 4 / (0.99);
    d.pml_alpha_max = 0.05;
    d.eps_kind = kind;
    const int lo[3] = {5, 5, 6}, hi[3] = {15, 13, 34};
    size_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        d.eps_lo[a] = lo[a];
        d.eps_hi[a] = hi[a];
        cells *= (size_t)(hi[a] - lo[a]);
    }
    const int nc = kind == FDTD_EPS_ISO ? 1 : (kind == FDTD_EPS_DIAG ? 3 : 6);
    m.eps.assign(nc * cells, 0.0);
    for (size_t p = 0; p < cells; ++p)
        for (int c = 0; c < nc; ++c) m.eps[c * cells + p] = c < 3 ? 1.5 + 0.1 * (double)((p + c) % 7) : 0.05;
    d.eps = m.eps.data();
    d.eps_bg = 1.0;
    if (kind != FDTD_EPS_TENSOR) {
        d.n_lorentz = 1;
        fdtd_lorentz_desc& L = d.lorentz;
        for (int a = 0; a < 3; ++a) {
            L.lo[a] = lo[a] + 1;
            L.hi[a] = lo[a] + 4;
        }
        L.n_poles = 2;
        L.poles[0] = {FDTD_POLE_LORENTZ, 1.2, 0.4, 0.02};
        L.poles[1] = {FDTD_POLE_DRUDE, 0.0, 0.3, 0.05};
    }
    m.wave.assign(50, 0.0);
    for (int t = 0; t < 50; ++t) m.wave[t] = std::sin(0.3 * t) * std::exp(-0.01 * (t - 20) * (t - 20));
    d.n_sources = 2;
    d.sources[0] = {FDTD_SRC_PLANE_Z, 0, {0, 0, 6}, m.wave.data(), 50};
    d.sources[1] = {FDTD_SRC_POINT, 2, {10, 9, 12}, m.wave.data(), 50};
    m.omega = {0.2, 0.3, 0.4};
    d.n_monitors = 3;
    d.monitors[0] = {FDTD_MON_FLUX_Z, 0, {0, 0, 30}, {4, 16, 4, 14}, m.omega.data(), 3};
    d.monitors[1] = {FDTD_MON_PATCH_Z, 2, {0, 0, 25}, {2, 18, 3, 15}, m.omega.data(), 2};
    d.monitors[2] = {FDTD_MON_PROBE, 4, {9, 8, 28}, {0, 0, 0, 0}, nullptr, 0};
    d.grad = 1;
    for (int a = 0; a < 3; ++a) {
        d.grad_lo[a] = 2;
        d.grad_hi[a] = d.n[a] - 2;
    }
}

fdtd_options opts(double budget) {
    fdtd_options o;
    std::memset(&o, 0, sizeof o);
    o.dtype = FDTD_F32;
    o.n_ckpt = 3;
    o.ckpt_storage = FDTD_F32;
    o.max_steps = 50;
    o.kernel = FDTD_KERNEL_SPLIT;
    o.mem_budget_bytes = budget;
    return o;
}

int create(const Dom& m, const fdtd_options& o) {
    fdtd_t h = nullptr;
    int rc = fdtd_create(&m.d, 1, &o, &h);
    if (h) fdtd_destroy(h);
    return rc;
}

int stream(const Dom& m, int slab, int K, int banks, double host_budget) {
    fdtd_stream_options o;
    std::memset(&o, 0, sizeof o);
    o.dtype = FDTD_F32;
    o.slab_planes = slab;
    o.steps_per_pass = K;
    o.max_steps = 50;
    o.mem_budget_bytes = 1.0;
    o.host_budget_bytes = host_budget;
    o.overlap = 1;
    o.local_slots = 2;
    o.host_banks = banks;
    fdtd_stream_t h = nullptr;
    int rc = fdtd_stream_create(&m.d, &o, &h);
    if (h) fdtd_stream_destroy(h);
    return rc;
}

}  // namespace

int main() {
    Dom m;
    basic(m);
    expect("diagonal, two poles, monitors, gradient: admitted", create(m, opts(1.0)), FDTD_E_NOMEM);
    {
        fdtd_options o = opts(1.0);
        o.dtype = FDTD_F64;
        o.ckpt_storage = FDTD_BF16;
        expect("FP64 with BF16 slots refused", create(m, o), FDTD_E_INVALID);
    }
    Dom b = m;
    b.d.courant = 0.995 / std::sqrt(3.0);
    expect("Courant number above the bound", create(b, opts(1.0)), FDTD_E_UNSTABLE);
    b = m;
    b.d.eps = b.eps.data();
    b.eps[3] = 0.9;
    expect("permittivity below one", create(b, opts(1.0)), FDTD_E_UNSTABLE);
    b = m;
    b.d.eps = b.eps.data();
    b.d.lorentz.poles[0].omega_dt = 2.5;
    expect("Lorentz pole at omega_0 dt = 2.5", create(b, opts(1.0)), FDTD_E_UNSTABLE);
    b = m;
    b.d.eps = b.eps.data();
    b.d.lorentz.n_poles = 17;
    expect("seventeen poles", create(b, opts(1.0)), FDTD_E_INVALID);
    b = m;
    b.d.eps = b.eps.data();
    b.d.monitors[1].rect[1] = 40;
    expect("patch rectangle past the grid", create(b, opts(1.0)), FDTD_E_RANGE);
    b = m;
    b.d.eps = b.eps.data();
    b.d.sources[1].pos[2] = 99;
    expect("point source past the grid", create(b, opts(1.0)), FDTD_E_RANGE);
    // periodic x and y: no absorbing cells there
    b = m;
    b.d.eps = b.eps.data();
    b.d.periodic[0] = b.d.periodic[1] = 1;
    b.d.bloch_sign[0] = -1;
    b.d.bloch_sign[1] = 1;
    expect("periodic axes with absorbing cells", create(b, opts(1.0)), FDTD_E_INVALID);
    b.d.pml[0] = b.d.pml[1] = b.d.pml[2] = b.d.pml[3] = 0;
    expect("periodic cell with a dispersive box and a gradient", create(b, opts(1.0)), FDTD_E_NOMEM);
    // tensor media: every node checked
    Dom t;
    basic(t, FDTD_EPS_TENSOR);
    expect("tensor media with a gradient: admitted", create(t, opts(1.0)), FDTD_E_NOMEM);
    Dom tb = t;
    tb.d.eps = tb.eps.data();
    tb.eps[0] = 0.5;   // an xx entry below one: an eigenvalue below one
    expect("tensor with an eigenvalue below one", create(tb, opts(1.0)), FDTD_E_UNSTABLE);
    tb = t;
    tb.d.eps = tb.eps.data();
    for (int a = 0; a < 3; ++a) {
        tb.d.eps_lo[a] = 0;
        tb.d.eps_hi[a] = tb.d.n[a];
    }
    {
        size_t cells = (size_t)tb.d.n[0] * tb.d.n[1] * tb.d.n[2];
        tb.eps.assign(6 * cells, 0.0);
        for (size_t p = 0; p < cells; ++p) {
            tb.eps[p] = 2.0;
            tb.eps[cells + p] = 3.0;
            tb.eps[2 * cells + p] = 2.5;   // the z eigenvalue between the others: refused in the z faces
        }
        tb.d.eps = tb.eps.data();
    }
    expect("tensor with an intermediate normal eigenvalue in a face", create(tb, opts(1.0)), FDTD_E_UNSTABLE);
    // streamed slabs
    expect("streamed: admitted, refused by the device budget", stream(m, 16, 4, 0, 0.0), FDTD_E_NOMEM);
    expect("streamed: three host banks", stream(m, 16, 4, 3, 0.0), FDTD_E_INVALID);
    expect("streamed: four host banks", stream(m, 16, 4, 4, 0.0), FDTD_E_NOMEM);
    expect("streamed: a slab cutting an absorbing z face", stream(m, 3, 4, 0, 0.0), FDTD_E_INVALID);
    expect("streamed tensor media", stream(t, 16, 4, 0, 0.0), FDTD_E_NOMEM);
    std::printf("%s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
