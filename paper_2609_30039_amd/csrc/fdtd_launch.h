// fdtd_launch.h -- host-visible launch interface between the runtime and the
// kernels of libfdtd (internal; not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fdtd {

constexpr int kMaxDftBlock = 64;   // buffered time samples per DFT flush

// One monitor as the kernels see it.
struct MonDev {
    int dom, kind, comp, ncomp, nf;   // kind 0 probe, 1 flux (Ex, Ey, <Hx>, <Hy>), 2 patch
    int rcomp;                        // ring components: flux 6 (Ex, Ey, Hx(k), Hx(k-1), Hy(k), Hy(k-1)), else 1
    int i0, i1, j0, j1, k;            // plane rectangle and plane index
    int pi, pj;                       // probe (pi, pj, k)
    const double* omega;              // [nf] omega * dt
    void* samples;                    // ring buffer [block][rcomp][npts] of the field type
    double* acc;                      // spectra [nf][ncomp][npts] (re, im)
    double* cot;                      // cotangents, same layout (probe: [max_steps])
    double* trace;                    // probe samples [ntrace]
    int ntrace;
    double* fpart;                    // flux: partial sums [nf][flux_blocks(npts)]
    double* fout;                     // flux: F(w) [nf]
};

// One stepping launch over all domains: kernel 1 = split, 2 = fused; rows =
// register-blocked rows per wave of the fused kernels; kz = z chunk.
// Split: bs = device prefix sums of blocks per domain (ndom + 1 entries).
// Fused: tile tables (domain, X0, Y0, k0) of general and bulk tiles.
constexpr int kAdjClasses1 = 7, kAdjClasses2 = 6;

struct LaunchCfg {
    int kernel, rows, kz, nblk, ndom;
    int sw;                    // split forward: block width in columns (64 or 32; 256 / sw rows)
    const int* bs;             // split blocks per domain (prefix sums)
    const int* xr;             // split: per-XCD runs of column blocks, 8 starts then 8 lengths
    int ngrid;                 // split: column workgroups per launch (8 x the longest run)
    const int* lbs;            // blocks over each domain's Lorentz box (prefix sums)
    int nlor;
    int ntens;                 // split: domains with tensor media (two E passes)
    int ntper;                 // split: those of them with a periodic axis
    int onepass;               // split family with the single-pass kernel on interior blocks (ping-pong sets)
    // split adjoint: one tile table per pass, (domain | class << 24,
    // x0 | xlen << 24, y0, k0), domains with a gradient only.  x is cut into
    // the slab zones (narrow tiles, W = 16) and the interior zone (W = 32); a
    // class names the slabs its tiles, or the neighbours they read, meet.
    // E-node pass kAdjClasses1 classes [W32: none, y/z, general; W16: x, all,
    // general, y/z], H-node pass kAdjClasses2 classes [W32: none, y/z, all;
    // W16: x, all, y/z]; general = Lorentz cells or gradient cells in a slab.
    int na1, na2, na1g;        // tiles per pass; general tiles leading the E-node table
    const int4* ta1;
    const int4* ta2;

    int ngen, nbulk;           // adjoint: general tiles, interior (bulk) tiles
    const int4* tgen;
    const int4* tbulk;
    int nfgen, nfcp, nfplain;  // forward: Lorentz tiles, absorber tiles, all other tiles
    const int4* tfgen;
    const int4* tfcp;
    const int4* tfplain;
};

constexpr int kFusedWaves = 4;

template <typename T>
// tdev: when set, kernels add the device-held step index to t (graph replays)
// slot >= 0: the split H kernel also writes every plane monitor's samples of
// the new state into that ring slot (the fused family ignores it)
void launch_fwd(const LaunchCfg& c, const void* doms, int rs, int ws, int t, hipStream_t s, const int* tdev = nullptr,
                int slot = -1);
template <typename T>
// pass 0: the E-node pass (all of the fused adjoint), 1: the H-node pass of
// the split family; cs[q]: stream of split class q of that pass
void launch_adj(const LaunchCfg& c, const void* doms, int rs, int ws, int fsr, hipStream_t s, int pass,
                const hipStream_t* cs);
// the E-node work of the split adjoint for tensor domain dom (n: its cells):
// the H-update transpose into the new Ebar, then u = S M Ebar into the
// scratch Et, the E-side memory cotangents and the node-tensor gradient;
// launch_adj's H-node pass completes the step (launch_per_adj_h in a
// periodic domain: per)
template <typename T>
void launch_tens_adj(const void* doms, int dom, const int n[3], int rs, int ws, int fsr, bool per, hipStream_t s);
// the whole adjoint step of Bloch-periodic domain dom (both passes, the seam
// in their neighbour gathers)
template <typename T>
void launch_per_adj(const void* doms, int dom, const int n[3], int rs, int ws, int fsr, hipStream_t s);
// its H-node pass alone: u of the scratch Et into the new Hbar across the seams
template <typename T>
void launch_per_adj_h(const void* doms, int dom, const int n[3], int rs, int ws, hipStream_t s);
template <typename T>
void launch_sample(const void* doms, const MonDev& m, int cs, int slot, hipStream_t s);
template <typename T>
void launch_dft(const MonDev& m, int n0, int count, hipStream_t s, const int* tdev = nullptr);
template <typename T>
void launch_probe(const void* doms, const MonDev& m, int cs, int n, hipStream_t s, const int* tdev = nullptr);
template <typename T>
void launch_seed(const void* doms, const MonDev& m, int as_, int n, hipStream_t s);

// reversible mode: record the interface of the current set cs into record
// slot `slot` (maxcnt: the largest face of any domain); one backward step
// u^m -> u^{m-1} over every domain's lossless box from set rs into set ws
// (maxcells: the largest box)
template <typename T>
void launch_rev_record(const void* doms, int ndom, int cs, int slot, int maxcnt, hipStream_t s);
template <typename T>
void launch_rev_step(const void* doms, int ndom, int rs, int ws, int m, long long maxcells, hipStream_t s);

// column blocks of the split forward for block width w (64 or 32 columns)
int split_blocks(int nx, int ny, int nz, int kz, int w);

void launch_zero(void* p, size_t bytes, hipStream_t s);
void launch_step_counter(int* c, int value, bool add, hipStream_t s);
void launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// y[0..n) += x[0..n) (monitor accumulators of a slab into the domain's)
void launch_add_f64(double* y, const double* x, size_t n, hipStream_t s);
// BF16 checkpoint slots: one table entry per forward state array (FP32)
constexpr int kBfChunk = 32768;              // elements per block
struct BfArr {
    const void* p;                           // set-0 address of the array
    long long n;                             // elements
    long long boff;                          // byte offset of its bf16 copy in a slot (256-aligned)
    int blk0, nblk;                          // its chunk blocks [blk0, blk0 + nblk)
};
// save: scale[q] = max |array q| over set (shift bytes from set 0); slot gets x / scale[q] in bf16
void launch_bf16_save(const BfArr* arr, int narr, int nblk, long long shift, float* part, unsigned int* scale,
                      char* slot, hipStream_t s);
// restore: array q of the set at shift = slot value * scale[q]
void launch_bf16_restore(const BfArr* arr, int narr, int nblk, long long shift, const unsigned int* scale,
                         const char* slot, hipStream_t s);
void launch_checksum(const void* p, size_t bytes, unsigned long long* out, hipStream_t s);
// sum of squares of domain dom's six fields of set cs into *out (FP64), through
// kEnergyBlocks partial sums in part
constexpr int kEnergyBlocks = 512;
template <typename T>
void launch_energy(const void* doms, int dom, int cs, double* part, double* out, hipStream_t s);
// Poynting flux per frequency of spectra [nf][4][npts] complex128 (device):
// flux_blocks(npts) partial sums per frequency in part (nf * flux_blocks
// doubles), the result in out[nf]
constexpr int kFluxPoints = 4096;      // plane points per block of the first pass
constexpr int kFluxMaxBlocks = 256;
int flux_blocks(long long npts);
void launch_flux(const double* spectra, int nf, long long npts, double* part, double* out, hipStream_t s);
// device address (on the current device) of the file-scope scratch array of
// kFluxScratchBytes that the allocation-free flux entry point uses; 0 on success
constexpr size_t kFluxScratchBytes = 65536;
int flux_scratch(double** out);

}  // namespace fdtd
