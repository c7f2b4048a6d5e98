// Registration engine shared by ls_register_pair and the serving loop.
#pragma once

#include <vector>

#include "kernels.h"

namespace ls {

struct RegPair {
  ls_pair pair;               // device pointers of the caller; c2w pointers unused (copies below)
  ls_reg_params prm;
  std::vector<double> c2wP;   // [vP][12]
  std::vector<double> c2wQ;   // [vQ][12]
  std::vector<int> sel[2];    // keyframes of P / of Q taking part (ascending; empty: all)
};

// One localisation problem: a keyframe of one submap rendering the other.
struct View {
  int pair;
  int index;      // keyframe index within its submap
  bool reverse;   // keyframe of Q localised in P (estimate of T_{Q->P})
  double c2w[12];
};

class RegEngine {
 public:
  ~RegEngine();
  // Host tables of the pairs' views (no device work), then the device state
  // in a caller workspace of workspace_bytes(capacity) bytes.
  ls_status prepare(const std::vector<RegPair>& pairs);
  size_t workspace_bytes(int64_t capacity) const;
  ls_status bind(void* work, size_t work_bytes, int64_t capacity, hipStream_t s);
  ls_status measure(hipStream_t s, int32_t* count4);
  // After measure(): renders every view and returns its co-visibility
  // (fraction of measured pixels the other submap covers, alpha >= 0.5).
  ls_status coverage(hipStream_t s, std::vector<float>& cov);
  ls_status step(hipStream_t s);
  ls_status final_forward(hipStream_t s);
  ls_status view_loss(hipStream_t s);  // the loss the pair's parameters select
  // overflow[2]: {any overflow since bind, instances required at the first one}
  ls_status readback(std::vector<float>& pose_h, std::vector<float>& loss_h, int32_t* overflow, hipStream_t s);
  ls_status fuse_pair(int p, const std::vector<float>& pose_h, const std::vector<float>& loss_h, ls_reg_result* out);
  ls_status read_exposure(int p, ls_reg_result* out, hipStream_t s);
  // joint registration (one T per pair, optimised on the device)
  ls_status step_joint(hipStream_t s);
  ls_status read_joint_T(hipStream_t s);  // device T of every pair -> joint_T
  std::vector<double> joint_T;            // [pairs][7], after read_joint_T
  JointView* jviews = nullptr;            // device, [R]
  JointPair* jpairs = nullptr;            // device, [pairs]
  std::vector<JointView> jviews_h;        // staging of the uploads
  std::vector<JointPair> jpairs_h;
  int joint_step = 0;
  void release();

  std::vector<RegPair> pairs;
  std::vector<View> views;
  std::vector<int> first_view;  // [pairs + 1]
  std::vector<int64_t> pix_off;
  int R = 0, T = 0;
  int64_t M = 0, P = 0, capacity = 0;
  ls_batch* batch = nullptr;
  ls_projected proj{};
  ls_bins bins{};
  ls_image img{};
  float *tgt_rgb = nullptr, *tgt_depth = nullptr, *g_rgb = nullptr, *g_depth = nullptr;
  float *scale = nullptr, *loss = nullptr, *pose = nullptr, *pose_grad = nullptr, *adam_m = nullptr,
        *adam_v = nullptr;
  ViewOpt* opt = nullptr;
  // exposure coefficients (a, b) per view, their gradient, Adam moments and
  // block partials; null unless the pair asks for exposure compensation
  float *expo = nullptr, *expo_grad = nullptr, *expo_m = nullptr, *expo_v = nullptr, *expo_part = nullptr;
  int32_t *range = nullptr, *count = nullptr, *sticky = nullptr;
  // plain L1 without exposure, joint mode or the loss-plateau exit: the
  // pose-only backward forms the loss gradient itself (render_bwd_pose_l1)
  // with 1 / |Omega| computed once at bind, and no loss kernel runs per
  // iteration (the final forward still computes the residuals)
  bool fused_l1 = false;

 private:
  struct Layout {
    size_t tables, rec, rad, til, aux, rgb, dep, alp, Tf, nl, trgb, tdep, grgb, gdep, scale, loss, pose, pg, m, v,
        opt, range, count, sticky, expo, joint, zero_end, tile_of, item, work, total;
  };
  Layout layout(int64_t capacity) const;
  static ls_status hip_ok();
};

void rot_of_quat(const double* q, double* R);
void rigid_inv(const double* A, double* out);
void rigid_mul(const double* A, const double* B, double* out);
void view_estimate(const double* c2w, const float* pose7, double* E);
int fuse_estimates(const double* est, const double* resid, const int32_t* rev, int n, double* out);
ls_status validate_pair(const ls_pair* p, const ls_reg_params* prm);
// Whether the iterations may take the fused L1 backward (LS_FUSED_L1=0 in the
// environment turns it off; for tests and measurements).
bool fused_l1_allowed(const ls_reg_params& pm);
RegPair make_reg_pair(const ls_pair* p, const ls_reg_params* prm);

}  // namespace ls
