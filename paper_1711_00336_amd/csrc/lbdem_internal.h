// Internal declarations shared by the HIP kernels and the host runtime of
// the coupled LBM-DEM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbdem {

// Lattice geometry: cell (i,j,k) centred at (i+1/2, j+1/2, k+1/2),
// flat index i + nx*(j + ny*k). Non-periodic axes have walls at 0 and n.
struct Geo {
    int n[3];
    int per[3];
    int64_t nc;
    // invariant-divisor constants: c / nx and c / (nx*ny) as (umulhi(c,m)+c) >> s
    uint32_t mx, sx, mxy, sxy;
};

// Model parameters in lattice units, resolved on the host.
struct Phys {
    double tau, omega;          // BGK relaxation time and its inverse
    double rho_f, mu;           // closure density, dynamic viscosity (tau-1/2)/3 rho_f
    double g[3], fb[3];         // particle gravity, fluid body-force density
    double e_n, mu_c, T_c, h_c, h_min;
    int lub_stab, use_lub, use_am;
    int lub_contact;            // lubrication also while the spheres overlap (gap clamped)
    int use_lift;               // shear-induced lift with the lattice curl
    int use_eilers, use_les;    // per-cell tau_e: Eilers viscosity, Smagorinsky LES
    int n_int, n_dem;
    double dt_int, dt_dem, c_am;
    double kn_per_m, xi_per_m;  // k_n / m_ij and xi_n / m_ij from T_c and e_n
    double skin;                // allowed displacement within one subcycle
    double vskin;               // Verlet list skin
    int rbin;                   // DEM search radius in cells (list build)
};

// Cell fields, [ncomp][nc] each. R = float (FP32 deviations) or double.
template <typename R>
struct Cells {
    R *df_src, *df_dst;         // [19][nc] f_q - w_q
    R *drho;                    // rho - 1 at step start
    R *j;                       // [3] sum_q c_q f_q at step start
    R *uprev;                   // [3] u_f of the previous step
    R *un;                      // [3] u_f of the current post-stream state
    R *dudt;                    // [nc][4] Du_f/Dt as (x, y, z, 0) per cell
    R *gradp;                   // [3] grad P
    R *epsp;                    // solid fraction 1 - eps_f of the current positions
    R *fam;                     // [3] -sum_p D F_am of the current subcycle
    R *uf;                      // [3] u_f re-evaluated with f_ext = eps_f f_b + fam
    R *facc;                    // [3] subcycle mean of f_ext
    R *curl;                    // [nc][4] curl of u_f at the subcycle start as (x, y, z, 0) (lift only)
};

// 1-cell bins: particles sorted by the cell of their position.
struct Bins {
    int *cnt;                   // [nc] counts (zero between builds)
    int *start;                 // [nc+1] exclusive prefix of cnt = slot ranges after the permutation
    int *list;                  // [np] slot indices, ordered by (cell, id) before the permutation
    int *bsum;                  // scan block sums (exclusive prefix after the top-level scan)
    int *loc;                   // [nc] prefix of cnt within its scan block
};

// Packed copy of what a DEM pair evaluation reads of a neighbour, one 64-byte
// record per slot (FP32-deviation form only): one cache line per neighbour
// instead of eleven scattered SoA loads. Positions and diameters stay FP64;
// mass, velocity and spin are rounded to FP32.
struct alignas(64) DemRec {
    double x[3];
    double d;                   // FP64: the overlap d_i/2 + d_j/2 - |x_j - x_i| cancels
    float m;
    float u[3], w[3];
    float pad;
};
static_assert(sizeof(DemRec) == 64, "one 64-byte record");

// Particles, SoA: vectors [3][cap] (component a of slot i at a*cap+i).
// Slots are kept sorted by (cell, original index) after every rebinning, so
// a bin is a contiguous slot range and neighbouring threads touch
// neighbouring cells. id[i] is the insertion index of the particle in slot i.
struct Parts {
    int64_t np, cap;
    double *x, *u, *w, *a;      // position, velocity, angular velocity, du/dt of last subcycle
    double *d, *rho;            // diameter, density
    int *id;
    double *x2, *u2, *w2, *a2, *d2, *rho2;  // permutation targets
    int *id2;
    int *sb;                    // [3][cap] kernel stencil base cell floor(x) per axis
    double *sw;                 // [9][cap] per-axis kernel weights, (3*axis + o+1)*cap + i (FP64 form)
    float *swf;                 // the same in FP32 (FP32-deviation form; exactly one of sw, swf is set)
    double *Fam, *Fd, *Fpr, *Fc;// current subcycle's fluid forces and F_const (slot order)
    double *Fdem, *Tdem;        // contact + lubrication force and torque of the substep
    double *ustart, *xstart;    // velocity / position at subcycle start
    double *Fam_id, *Fd_id, *Fpr_id, *Fc_id;  // last subcycle's forces by insertion index
    double *Fl, *Fl_id;         // lift (slot order; last subcycle by insertion index), lift only
    // Verlet lists labelled by the slot a particle had when the lists were
    // built (bslot[slot], carried through the reorders): nlist[label*nbr + t]
    // holds neighbour labels in ascending insertion index, nnb[label] entries,
    // build positions xbuild[3][cap] by label; slot_of[label] = current slot;
    // nslot[label*nbr + t] = slot_of[nlist[label*nbr + t]] (t < nnb[label]),
    // refreshed with the lists at the start of every subcycle when n_DEM >= 3
    int *nlist, *nnb, *slot_of, *nslot;
    int *bslot, *bslot2;        // label of the particle in each slot (+ permutation target)
    int nbr;                    // list capacity per particle (sized from the density and reach)
    double *xbuild;
    int *need;                  // 1: rebuild the lists before the next DEM substep
    DemRec *pk, *pk2;           // packed DEM records by slot (+ permutation target), or null
};

// launch choices picked per domain (autotuner); -1 = heuristic default
struct Tune {
    int gather;                 // -1 by density; 0/1/2/4 LDS tiles 16x4x8, 16x4x4, 8x4x4, 16x4x16; 3 per cell
    int dem_order;              // 0: DEM force pass in slot order; 1: in the blocked order of Order
    int cell_waves;             // workgroups per CU of the streaming cell passes (moments, stream-collide):
                                // 0 unlimited, else capped through reserved LDS; -1 default
    int fuse;                   // DEM substep forces and integration in one pass where the form
                                // allows it (FP32 form, n_DEM >= 3): -1 default (off), 0 off, 1 on
};

// Processing order of the DEM force pass. Slots are sorted by cell in
// row-major order, so a run of consecutive slots is a thin slab of rows
// whose neighbours reach two planes up and down. In the blocked order the
// particles are visited block by block (blocks of ob[0] x ob[1] x ob[2]
// cells, each block row by row), so the workgroups in flight on one XCD
// cover a compact region and their neighbours' records stay in its L2.
// Each particle's force is the same whatever the order.
struct Order {
    int *porder;                // [cap] slot of the v-th particle in blocked order
    int *rowoff;                // [nrows] particles per block row, then their block-local exclusive prefix
    int *rowsum;                // [nrows / kScanPerBlock + 2] scan block sums, then their exclusive prefix
    int64_t nrows;              // block rows: blocks per axis (padded) x ob[1] x ob[2]
    int ob[3];                  // block shape in cells
    int nb[3];                  // blocks per axis, ceil(n / ob)
};

struct Desc {
    Geo g;
    Phys p;
    Tune t;
    Bins b;
    Parts pt;
    Order o;
    int *flags;                 // error bits
    long long *stepc;           // device step counter
};

enum : int {
    FLAG_WALL = 1,              // particle centre through a wall
    FLAG_SKIN = 2,              // moved more than the skin within a subcycle
    FLAG_NONFINITE = 4,
    FLAG_EPS = 8,               // eps_f <= 0
    FLAG_NLIST = 16,            // a particle has more list neighbours than the capacity nbr
    FLAG_FLUID_NONFINITE = 32,  // non-finite density or velocity of a cell at the collision
    FLAG_MACH = 64              // |u_bar| > 0.1 in a cell (beyond the low-Mach range of the LBM)
};

constexpr int kTimingClasses = 13;  // kernel classes of lbdem_kernel_time

constexpr int kBlock = 256;
constexpr int kScanItems = 8;   // per thread in the block scan
constexpr int kScanPerBlock = kBlock * kScanItems;

// -- launchers (lbdem_kernels.hip) -----------------------------------------
template <typename R> void launch_moments(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_cellfields(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_curl(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_part_am(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_gather_am(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_part_drag(const Desc &D, const Cells<R> &C, int record, hipStream_t s);
template <typename R> void launch_gather_fd(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_gather_eps(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_gather_eps_am(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_gather_eps_uf(const Desc &D, const Cells<R> &C, hipStream_t s);
constexpr int kGatherVariants = 5;
template <typename R> void launch_stream_collide(const Desc &D, const Cells<R> &C, hipStream_t s);
template <typename R> void launch_zero(R *p, int64_t n, hipStream_t s);
template <typename R> void launch_to_double(const R *src, double *dst, int64_t n, hipStream_t s);
template <typename R> void launch_vec4_to_double(const R *src, double *dst, int64_t nc, hipStream_t s);
template <typename R> void launch_fluid_fraction(const R *src, double *dst, int64_t nc, hipStream_t s);
template <typename R> void launch_from_double(const double *src, R *dst, int64_t n, hipStream_t s);
template <typename R>
void launch_diag(const Desc &D, const Cells<R> &C, const R *df, double *partials, int nblk, double *out,
                 hipStream_t s);
int diag_blocks(const Desc &D);
// the diagnostics reduction: 12 values, at most 1024 blocks of partials
constexpr int kDiagValues = 12;
constexpr int kDiagMaxBlocks = 1024;
constexpr int64_t kDiagScratchDoubles = (int64_t)kDiagValues * kDiagMaxBlocks + 16;
// Device address of the static diagnostics scratch on `device` (looked up
// once per device, with that device current); nullptr if the lookup fails.
double *diag_scratch_on_device(int device);

void launch_dem_force(const Desc &D, hipStream_t s);
// FP32 form with n_DEM >= 3 when asked for (tuning): force, torque and the
// integration of a substep in one pass (records alternate between pk and pk2
// by substep parity)
bool dem_substep_fused(const Desc &D);
void launch_dem_substep_fused(const Desc &D, int sub, int last, hipStream_t s);
void launch_dem_order(const Desc &D, hipStream_t s);   // blocked processing order of the current slots
void launch_nlist(const Desc &D, hipStream_t s);      // rebuild Verlet lists if flagged
void launch_integrate(const Desc &D, int last_substep, hipStream_t s);
void launch_bin_count(const Desc &D, hipStream_t s);
void launch_bin_build(const Desc &D, hipStream_t s);   // scan + place
void launch_sort_permute(const Desc &D, hipStream_t s); // order bins, slots <- bin order, stencils
// the same, with the next subcycle's added-mass force evaluated in the permutation
template <typename R> void launch_sort_permute_am(const Desc &D, const Cells<R> &C, hipStream_t s);
void launch_zero_int(int *p, int64_t n, hipStream_t s);
void launch_set_step(long long *stepc, long long v, hipStream_t s);
void launch_set_int(int *p, int v, hipStream_t s);

}  // namespace lbdem
