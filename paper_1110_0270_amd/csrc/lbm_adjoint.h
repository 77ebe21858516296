// Recording of a forward rollout for the adjoint (checkpoints every K steps
// and the per-step Ehrenfest selections) and the backward pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lbm.h"

namespace lbm {

struct AdjointLayout {
  bool on = false;
  int K = 0;                 // checkpoint interval
  long long max_steps = 0;
  long long n_ckpt = 0;      // slots: state after 0, K, 2K, ... steps
  long long k = 0;           // selection budget per step (tape width)
  size_t lat_bytes = 0;
  size_t lam_bytes = 0;      // one adjoint lattice (compute precision)
  size_t off_ckpt = 0;       // n_ckpt lattices
  size_t off_seg = 0;        // K lattices: states of the segment being reversed
  size_t off_lam[2] = {0, 0};
  size_t off_gom = 0;        // per-site omega gradient accumulator
  size_t off_tape_sel = 0;   // max_steps * k site indices
  size_t off_tape_cnt = 0;   // max_steps counts
  size_t off_mask = 0;       // one byte per site: sent to f* in the step being reversed
  bool store_alpha = false;  // ELBM: the recompute keeps alpha and branch per site
  size_t off_alpha = 0;      // K x [ny][pitch] alpha (compute precision)
  size_t off_branch = 0;     // K x [ny][pitch] branch bytes
  bool median = false;       // median filter: per-site records of its adjoint
  size_t off_med_gs = 0;     // [ny][pitch] dL/d Delta S through the site's own homothety
  size_t off_med_h = 0;      // [ny][pitch] dL/d Delta S of the site's median neighbour
  size_t off_med_am = 0;     // [ny][pitch] bytes: that neighbour's offset code (255: none)
  size_t end = 0;
};

// Per-site records of the median filter's adjoint (all nullptr when the
// filter is off): see k_adjoint_med.
struct MedianAdjoint {
  void* gs = nullptr;
  void* h = nullptr;
  unsigned char* am = nullptr;
};

AdjointLayout adjoint_layout(const lbm_config* c, size_t lat_bytes, long long qs, long long k,
                             size_t offset);
hipError_t adjoint_begin_record(const AdjointLayout& L, char* ws, const void* lat,
                                size_t lat_bytes, hipStream_t s);
hipError_t adjoint_after_step(const AdjointLayout& L, char* ws, long long steps_done,
                              const void* lat, size_t lat_bytes, hipStream_t s);
// Where step t writes its selected site indices (the tape when recording).
int32_t* adjoint_selected_slot(const AdjointLayout& L, char* ws, long long t, int32_t* dflt);
long long* adjoint_count_slot(const AdjointLayout& L, char* ws, long long t);

// Adjoint kernels (lbm_adjoint.hip).  step_args points at the StepArgs of
// the compute precision (double for LBM_F64 storage, float otherwise) with
// src = the state the step read; lam_in/lam_out/gom use the same precision
// and the pitched layout of the lattice.
// alpha/branch: the step's ELBM alpha and branch per site, from the
// recompute (required for ELBM, ignored otherwise).  list/count/k: the
// step's Ehrenfest sites when k <= kAdjListMax (read into LDS in place of
// the mask; nullptr otherwise).  med: the median filter's records (the
// step then runs as two kernels).  e0/e1: optional events recorded right
// before and after the kernel(s).
constexpr long long kAdjListMax = 64;
hipError_t launch_adjoint(int storage, int Q, int coll, const void* step_args, const void* lam_in,
                          void* lam_out, void* gom, const unsigned char* mask,
                          const void* alpha, const unsigned char* branch, const int32_t* list,
                          const long long* count, long long k, const MedianAdjoint& med,
                          hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// f* written into step_args->dst at the first *count sites of list (<= k).
hipError_t launch_tape_fix(int storage, int Q, const void* step_args, const int32_t* list,
                           const long long* count, long long k, hipStream_t s);
hipError_t launch_mark(unsigned char* mask, const int32_t* list, const long long* count,
                       long long k, unsigned char val, hipStream_t s);
// Dense [nf][ny][nx] (FP64 or FP32) <-> pitched [nf][ny][pitch] (FP64 or FP32).
hipError_t launch_to_pitch(const void* src, int src_f64, void* dst, int dst_f64, int nf, int nx,
                           int ny, int pitch, long long qs, hipStream_t s);
hipError_t launch_from_pitch(const void* src, int src_f64, void* dst, int dst_f64, int nf, int nx,
                             int ny, int pitch, long long qs, hipStream_t s);

hipError_t launch_convert_field(const void* src, int src_f64, void* dst, int dst_f64, int nx,
                                int ny, int pitch, hipStream_t s);

}  // namespace lbm

