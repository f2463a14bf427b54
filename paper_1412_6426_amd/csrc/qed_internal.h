// qed_internal.h -- shared declarations between the host entry points and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qed.h"
#include "qed_device.h"

namespace qedk {

// Header of the qed_step workspace; followed by the per-instance arrays laid out by
// WorkLayout.
struct alignas(64) WorkHdr {
  unsigned long long lep_queue;  // next lepton tile to hand out
  unsigned long long pho_queue;  // next photon tile
  long long lep_tiles;           // lepton tiles this step
  long long pho_tiles;           // photon tiles this step
  long long step;                // global step index n
  double tn;                     // field time t0 + n dt
  uint32_t tables_ok;
  uint32_t reserved[3];
};

struct WorkLayout {
  size_t n0;        // long long [n_inst * 3]: live slots at step start (0 when frozen)
  size_t lep_pref;  // long long [2 n_inst + 1]: tile prefix over (instance, e-/e+) segments
  size_t pho_pref;  // long long [n_inst + 1]
  size_t eb;        // double [n_inst * 6]: E, B of space-independent fields at t_n
  size_t total;
  static WorkLayout make(int n_inst) {
    WorkLayout L;
    size_t off = sizeof(WorkHdr);
    auto take = [&off](size_t bytes) {
      size_t o = off;
      off += (bytes + 63) & ~(size_t)63;
      return o;
    };
    L.n0 = take(sizeof(long long) * 3 * (size_t)n_inst);
    L.lep_pref = take(sizeof(long long) * (2 * (size_t)n_inst + 1));
    L.pho_pref = take(sizeof(long long) * ((size_t)n_inst + 1));
    L.eb = take(sizeof(double) * 6 * (size_t)n_inst);
    L.total = off;
    return L;
  }
};

struct StepArgs {
  qed_soa sp[3];
  qed_instance* inst;
  int n_inst;
  const DevTables* tables;
  FieldArgs field;
  double e0[3], b0[3];
  double dt, t0, eps_r;
  double inv_lep_scale;  // 1 / (kappa 28 pi eps_r)
  double inv_pho_scale;  // 1 / (kappa 260 pi eps_r)
  double dtfac_per_h;    // alpha / eps_r
  int adaptive, forced, emission, pairs, push_photons, freeze_on_drop;
  long long tile;
  WorkHdr* hdr;
  long long* n0;
  long long* lep_pref;
  long long* pho_pref;
  double* eb;
  qed_stats* stats;
  long long* d_step;
  hipEvent_t events[4];
};

struct LaunchShape {
  int grid;
  int block;
};

// Kernel launchers (qed_step.hip / qed_tables.hip).
hipError_t launch_step(const StepArgs& a, int precision, LaunchShape lep, LaunchShape pho,
                       bool run_photons, hipStream_t s);
hipError_t launch_build_tables(DevTables* t, const Series64& s, hipStream_t st);
hipError_t launch_append_stats(const qed_stats* src, qed_stats* log, long long cap,
                               long long* cnt, hipStream_t s);
hipError_t launch_spectrum(const qed_soa& ph, qed_instance* inst, int n_inst, double lo,
                           double hi, int bins, double* hist, hipStream_t s);
hipError_t launch_fill_standing(float* const g[6], const int n[3], const double dx[3],
                                const double org[3], double amp, double omega, double phase,
                                double t, hipStream_t s);
// Persistent-grid sizing: resident workgroups per CU for the step kernels.
int step_blocks_per_cu(int precision, bool photon, int block);

}  // namespace qedk
