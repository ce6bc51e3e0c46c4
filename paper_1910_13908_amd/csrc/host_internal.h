// Host-side internals shared by the library's translation units (not part of the ABI).
#pragma once

#include "../../include/ddcal.h"
#include "common.h"

#include <string>
#include <vector>

namespace ddc {
namespace host {

// Device buffers of one calibration inside a context's workspace.
struct CalBufs {
  void* solve = nullptr;       // normal-equation / factor buffers (owned description)
  void* coh = nullptr;         // [K][8][T][F][B]
  void* Rb = nullptr;          // residual planes
  void* Yb = nullptr;          // per-cluster data planes
  int32_t* doffs = nullptr;    // cluster offsets on the device
  LMState* dinfo = nullptr;    // per-visit LM reports [n_sweeps][K]
  ddc_lm_step* dtrace = nullptr;  // per-iteration records [n_sweeps][K][n_iter]
  int n_info = 0, n_iter = 0, K = 0, prec = 0;
  std::vector<int32_t> offs_host;
};

int64_t calibrate_footprint(const ObsDev& o, int K, int n_sweeps, int n_iter, int prec);
ddc_status prepare_calibrate(ddc_ctx* c, const ObsDev& o, const ddc_sky* sky, int n_sweeps,
                             int n_iter, int prec, CalBufs& cb);
void release_calibrate(CalBufs& cb);
// The SAGE sweeps of one calibration; residual_ready: cb.Rb already holds V - sum_k J_k C_k J_k^H
// (formed by a batched launch), otherwise it is formed first.
ddc_status enqueue_sage(ddc_ctx* c, const ObsDev& o, const void* vis, double* jones,
                        const ddc_cal_opts& opt, CalBufs& cb, bool residual_ready = false);
// Reads every visit's state back; info and trace (HOST, nullable) receive the reports.
ddc_status collect_infos(ddc_ctx* c, CalBufs& cb, ddc_lm_info* info, ddc_lm_step* trace);
ddc_status ctx_obs(ddc_ctx* c, const ddc_obs* obs, ObsDev& o);
hipStream_t ctx_stream(ddc_ctx* c);
void ctx_lend_workspace(ddc_ctx* c, void* ws, size_t bytes);
const char* ctx_error(ddc_ctx* c);

}  // namespace host
}  // namespace ddc
