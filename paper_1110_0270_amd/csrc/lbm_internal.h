// Parameter blocks and launch entry points shared by the host API
// (lbm_api.hip) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Device-resident state of the Ehrenfest top-k selection (section 4,
// Ehrenfests' regularisation with a budget of k sites per step).
// Floors and histogram frames are kept per step parity: with omega near 2
// the nonequilibrium part changes sign every step, and the steps of one
// parity resemble each other more than consecutive steps do.
struct SelState {
  unsigned long long floor_key[2]; // candidate iff eligible and key >= floor_key[parity]
  unsigned long long base_key[2];  // histogram frame: bucket = (key - base_key) >> shift
  unsigned long long step;         // steps selected so far (parity = step & 1)
  unsigned long long fallbacks;  // steps that needed a full rescan (cumulative)
  unsigned long long overflows;  // steps whose boundary list overflowed (cumulative)
  unsigned long long cand_total; // candidates over all steps (cumulative)
  long long n_sel;               // sites selected in the last completed step
  unsigned int shift[2];         // bucket width is 2^shift keys
  unsigned int ticket;           // last-workgroup ticket
  int fallback;                  // 1: this step's candidates came from a rescan
  int fb_bin;                    // coarse bin chosen by the rescan
  int floor_raised[2];           // floor_key is above the eligibility threshold
  int b_bin;                     // this step's boundary bucket (-1: take every candidate)
  unsigned long long b_nc;       // this step's candidate count
  unsigned long long b_above;    // candidates in buckets above b_bin
  long long tape_t;              // steps selected since the rollout began (tape index)
  int pad[4];
  // Sites selected so far in the running step (high 32 bits) and the length
  // of the boundary-bucket list (low 32 bits): one atomic per region-sweep
  // workgroup reserves both, on a cache line of its own (every workgroup of
  // the sweep adds to it).
  alignas(128) unsigned long long sel_bnd;
  unsigned long long pad_line[15];
};

// Regions (the candidate areas of the step kernel's wavefronts) per
// workgroup of the region sweep, one per thread: 16 wavefronts.  Each
// workgroup reserves its slots in the selected and boundary lists with one
// same-address atomic, so fewer, larger workgroups queue fewer of them
// (1024 against 256 regions: 7 us less per FP32 step).
constexpr int kSweepRegions = 1024;
constexpr int kBuckets = 4096;        // histogram of candidate keys
// Bucket b is counted at hist[hist_pos(b)].  The step kernel's atomics crowd
// into the few buckets just above the floor, and atomics on one cache line
// queue behind each other: consecutive buckets go to 128 different lines
// (bucket 128 q + r at word 32 r + q, r < 128).
constexpr long long kHistWords = kBuckets;
__host__ __device__ inline int hist_pos(int b) { return (b % 128) * 32 + b / 128; }
static_assert(kBuckets == 128 * 32, "hist_pos spreads 4096 buckets over 128 lines of 32");
constexpr int kCoarse = 4096;         // rescan histogram: top 12 bits of the FP32 key
constexpr int kCountSlots = 64;       // candidate counters, 128 bytes apart
constexpr int kCountStride = 16;      // in unsigned long long

// Counters of limiter activity (cumulative since the last reset).
enum Counter : int {
  CNT_POSITIVITY = 0, CNT_MEDIAN = 1, CNT_ELBM_NOROOT = 2, CNT_ELBM_F64 = 3,
  CNT_ELBM_NONPOS = 4, CNT_ELBM_ITERS = 5, CNT_N = 8
};
// The limiter counters are spread over kCntSlots copies, one 64-byte line
// each ([slot][CNT_N]); a workgroup adds to copy blockIdx.x % kCntSlots, so
// one step's atomics do not queue on a single address.
constexpr int kCntSlots = 64;

// Device state of the ensemble limiters (section 4): the step's threshold
// and mean, the radix descent that solves eq. EntThresh over the lattice's
// Delta S values, and the monitor's sums.
enum EnsMode : int { ENS_NONE = 0, ENS_THRESHOLD = 1, ENS_SMOOTH = 2, ENS_DOUBLE_MONOTONE = 3,
                     ENS_POINTWISE = 4 };
constexpr int kEnsBins = 4096;        // radix of the descent: 12 bits per level
struct EnsState {
  double sum_dS;        // sum of the finite Delta S (pre-pass)
  double production;    // sum of [1 - (omega - 1)^2] Delta S (pre-pass)
  double n_finite;      // sites with finite Delta S (pre-pass)
  double threshold;     // Delta S_t of the step (+inf: the limiter rests)
  double mean;          // E(Delta S)
  double rhs;           // delta_0 * production
  double above_n;       // descent: values whose key lies above the resolved range
  double above_s;       //          and their sum
  unsigned long long prefix;  // descent: key bits resolved so far
  int prefix_bits;
  int active;           // descent still running
  int pad[5];
  // the step kernel's monitor sums of the step, spread over kEnsSlots copies
  // (a workgroup adds to copy blockIdx mod kEnsSlots): [slot][0] the LBGK
  // production, [slot][1] sum (1 - phi^2) Delta S, [slot][2] sum Delta S,
  // [slot][3] sites with finite Delta S; cleared before each step
  double step_acc[64][4];
};
constexpr int kEnsSlots = 64;

template <class R> struct KeyOf;
template <> struct KeyOf<float> { using T = uint32_t; };
template <> struct KeyOf<double> { using T = unsigned long long; };

template <class R>
struct StepArgs {
  const void* src;
  void* dst;
  long long qs;          // elements between populations = ny * pitch
  int nx, ny, pitch;     // ny: rows (D3Q27: nz * ny3, row z * ny3 + y)
  int ny3, nz;           // D3Q27: the grid's y and z extents
  int tiles_x, tiles_y;
  int tile_tx;           // sites per tile row (256 or 64); tiles hold 256 sites
  int bc;
  int eq_kind;
  int positivity;
  int ehrenfest;
  int count_events;
  R rho0;
  R omega;
  const R* omega_field;  // [ny][pitch] or nullptr
  R lid[9];              // moving-wall term 6 w_i rho_wall (v_i . u_wall)
  R lid_u;               // lid speed of the diffusive wall
  // MRT (moment space): F = f + Minv (rates .* (M (f* - f)))
  R M[81];
  R Minv[81];
  R rates[9];
  unsigned nu_rows;      // bit mask of rows whose rate is the shear rate
  unsigned q_rows;       // rows whose rate is a function q_mode of the shear rate
  int q_mode;            // 1: 8 (2 - s) / (8 - s); 2: 3 (2 - s) / (3 - s)
  int sel_mrt;           // selected sites get the MRT collision instead of f*
  // ELBM
  R eps, atol, dS_cut;
  int max_iter, norm, fallback;
  double eps64, dS_cut64;
  R f64_below;
  // median
  R med_delta;
  // Ehrenfest
  R ehr_delta;
  SelState* sel;
  // Candidate buffer: wavefront w of tile t owns entries [64 (4t + w), +64);
  // wcount[4t + w] holds how many it filled this step (0 where none).
  typename KeyOf<R>::T* cand_key;
  uint32_t* cand_idx;
  R* cand_mom;           // [3][cap]: rho (or rho - rho0 when shifted), ux, uy
  long long cap;         // 256 * number of tiles
  uint32_t* wcount;
  unsigned long long* ccount;  // kCountSlots partial candidate counts (spread atomics)
  unsigned int* hist;    // kBuckets counts of this step's candidates (stride kHistStride)
  unsigned long long* counters;  // [kCntSlots][CNT_N]
  // ELBM recompute for the adjoint: alpha and branch of every site ([ny][pitch]),
  // or nullptr
  R* alpha_out;
  unsigned char* branch_out;
  // ensemble limiters: mode, parameters, device state; dsb (pre-pass Delta S
  // per site, [ny][pitch]) and the descent histogram
  int ens_mode;
  R ens_alpha, ens_k, ens_delta;
  EnsState* ens;
  R* ens_dsb;
  unsigned int* ens_cnt;      // kEnsBins
  double* ens_sum;            // kEnsBins
  // ELBM with FP32 arithmetic: the step kernels list the sites whose root
  // solve needs FP64 (site index) and k_elbm_f64 finishes them, so that the
  // step kernels do not carry the FP64 solve's registers; [0] count,
  // [1] last-workgroup ticket.  nullptr: no such sites can occur.
  uint32_t* f64_sites;
  unsigned int* f64_count;
  // general nonlocal filter of section 4: the coefficients d(y) in tensor
  // order of the shifts y ([3] D1Q3, [9] D2Q9), or nullptr
  const R* nl_coef;
};

// Launchers (one per translation unit); return hipSuccess or the error.
// storage: 0 f64, 1 f32, 2 f16 shifted, 3 bf16 shifted.
// e0/e1 (optional): events recorded at the step kernel's start and end.
hipError_t launch_step(int storage, int Q, int coll, bool median, const void* args,
                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The step with the general nonlocal filter (periodic D1Q3 / D2Q9).
hipError_t launch_step_nl(int storage, int Q, int coll, const void* args, hipStream_t s,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The D3Q27 step (periodic; LBGK, median filter, positivity rule).
hipError_t launch_step3(int storage, bool median, const void* args, hipStream_t s,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_set_eq(int storage, int Q, const void* rho, const void* ux,
                         const void* uy, const void* uz, int in_f64, void* lat, long long qs, int nx,
                         int ny, int pitch, int eq_kind, double rho0, hipStream_t s);
hipError_t launch_set_pop(int storage, int Q, const void* f, int in_f64, void* lat,
                          long long qs, int nx, int ny, int pitch, double rho0,
                          hipStream_t s);
hipError_t launch_get_pop(int storage, int Q, void* f, int out_f64, const void* lat,
                          long long qs, int nx, int ny, int pitch, double rho0,
                          hipStream_t s);
hipError_t launch_moments(int storage, int Q, const void* lat, long long qs, int nx, int ny,
                          int pitch, double rho0, void* rho, void* ux, void* uy,
                          int out_f64, hipStream_t s);
// Whole-lattice FP64 reduction into out[0..7] = mass, mom_x, mom_y, entropy,
// min_rho, nonfinite, the sum of the squared vorticity and the number of
// sites it covers (four neighbours in the lattice; every site when
// periodic).  partial: workspace of stats_partial_doubles().
long long stats_partial_doubles(int nx, int ny);
hipError_t launch_stats(int storage, int Q, const void* lat, long long qs, int nx, int ny,
                        int pitch, int periodic, double rho0, double* partial, double* out,
                        long long* diverged_step, long long step, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// Ensemble limiters: before the step kernel, the pre-pass (Delta S of every
// site, E(Delta S), the LBGK production) and, with a dissipation budget, the
// descent that solves eq. EntThresh; leaves the step's threshold and mean in
// the EnsState.  delta0 <= 0: fixed threshold delta.
hipError_t launch_ensemble(int storage, int Q, const void* step_args, double delta0,
                           double delta, hipStream_t s);


// Ehrenfest selection after a step (selection kernels).
struct SelectArgs {
  int storage, Q, coll;
  const void* step_args;   // StepArgs<R> of the step (for rescans)
  long long k;
  long long n_sites;
  int32_t* selected;       // out: selected site indices, ascending not guaranteed
  int32_t* segsel;         // per-workgroup staging of selected indices (cap entries)
  uint32_t* blist;         // boundary-bucket candidate positions
  long long bcap;          // capacity of blist
  unsigned int* coarse;    // kCoarse
  long long* n_sel_out;    // optional: the step's selection count is copied here
  // Recording a rollout: the selection goes to tape_sel + t k and its count
  // to tape_cnt[t], t = SelState::tape_t (read on the device, so that the
  // arguments are the same every step and the steps can be replayed from a
  // HIP graph); t >= tape_len writes to `selected` / n_sel_out instead.
  int32_t* tape_sel;
  long long* tape_cnt;
  long long tape_len;
};
hipError_t launch_select(const SelectArgs& a, hipStream_t s);
// Place the first candidate floor of a freshly set lattice at the 3k-th
// largest Delta S of its next step (one rescan).
hipError_t launch_select_calibrate(const SelectArgs& a, hipStream_t s);
void init_select_state(SelState* h, int f64);


}  // namespace lbm
