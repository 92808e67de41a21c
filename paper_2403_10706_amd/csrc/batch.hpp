// Batched execution, host side.  The launch sequence of one volume pair is recorded instead of
// enqueued (every launcher checks active_recorder()); the sequences of several pairs are then
// issued launch by launch, each Gauss-Newton kernel (loss_grad, PCG scalars and steps, Armijo
// trials and decisions, the step update) once for all pairs through an argument table in device
// memory, everything else pair by pair.  While recording for a batch, batch_plans() makes the
// launch planners pick shapes that a shared launch can use (256-thread workgroups, every share a
// whole number of XCD rounds, one PCG tile shape).
#pragma once

#include <cstring>
#include <functional>
#include <utility>
#include <vector>

#include "rgp_launch.hpp"

namespace rgp {

enum class RecKind : int {
  kOther = 0,
  kLossGrad,
  kTrial,
  kDecide,
  kApply,
  kPcgScalars,
  kPcgStep
};

struct RecLaunch {
  RecKind kind = RecKind::kOther;
  std::vector<unsigned char> args;  // the kernel's argument block
  MarchGeo geo{};                   // PCG step: the volume's plane march
  unsigned grid = 0, block = 0;
  size_t lds = 0;
  int var[4] = {0, 0, 0, 0};        // template parameters that a shared launch needs equal
  int64_t cells = 0, nodes = 0;     // volume the launch covers (kernel timing of shared launches)
  int tag = 0;                      // kernel timing tag (as the plain launch's)
  std::function<hipError_t(hipStream_t)> replay;  // the plain launch of this one volume
};

struct Recorder {
  std::vector<RecLaunch> launches;
};

Recorder*& active_recorder();
bool& batch_plans();
int& batch_march_min();  // while batch_plans(): minimum PCG march length (0: none)

template <typename A>
inline hipError_t record_launch(RecKind kind, const A& a, unsigned grid, unsigned block,
                                size_t lds, int v0, int v1, int v2,
                                std::function<hipError_t(hipStream_t)> replay,
                                const MarchGeo* geo = nullptr) {
  RecLaunch r;
  r.kind = kind;
  r.args.resize(sizeof(A));
  std::memcpy(r.args.data(), &a, sizeof(A));
  r.grid = grid;
  r.block = block;
  r.lds = lds;
  r.var[0] = v0;
  r.var[1] = v1;
  r.var[2] = v2;
  if (geo) r.geo = *geo;
  r.replay = std::move(replay);
  active_recorder()->launches.push_back(std::move(r));
  return hipSuccess;
}

// Notes the volume and timing tag of the launch just recorded.
inline hipError_t note_volume(int64_t cells, int64_t nodes, int tag) {
  RecLaunch& r = active_recorder()->launches.back();
  r.cells = cells;
  r.nodes = nodes;
  r.tag = tag;
  return hipSuccess;
}

inline hipError_t record_other(std::function<hipError_t(hipStream_t)> replay) {
  RecLaunch r;
  r.replay = std::move(replay);
  active_recorder()->launches.push_back(std::move(r));
  return hipSuccess;
}

// Shared launches: tab points to n argument blocks in device memory, starts to n+1 workgroup
// offsets (one workgroup per volume for the single-block kernels).  cells/nodes/tag: the summed
// volume and the timing tag that a kernel-timing session records for the launch.
hipError_t launch_loss_grad_batch(const void* tab, const uint32_t* starts, int n, unsigned grid,
                                  DType img, DType real, int64_t cells, int64_t nodes, int tag,
                                  hipStream_t s);
hipError_t launch_trial_batch(const void* tab, const uint32_t* starts, int n, unsigned grid,
                              int nc, DType img, DType real, int64_t cells, int64_t nodes,
                              hipStream_t s);
hipError_t launch_decide_batch(const void* tab, int n, int nc, hipStream_t s);
hipError_t launch_apply_step_batch(const void* tab, const uint32_t* starts, int n, unsigned grid,
                                   DType real, hipStream_t s);
hipError_t launch_pcg_scalars_batch(const void* tab, int n, hipStream_t s);
// max_xl: the longest march of the volumes (units of at most 3 planes load them all up front)
hipError_t launch_pcg_step_batch(const void* tab, const MarchGeo* geo, const uint32_t* starts,
                                 int n, unsigned grid, size_t lds, DType real, int max_xl,
                                 int64_t cells, int64_t nodes, int tag, hipStream_t s);

}  // namespace rgp
