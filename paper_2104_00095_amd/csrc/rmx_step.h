// Device tables and launchers of one time step of the reference map around the
// extrapolation (Lin, Derr & Rycroft, arXiv 2104.00095, SI "Timestepping algorithm",
// steps 5-7 and 11; SI "Evaluating the advective term").
#pragma once
#include "rmx_internal.h"

namespace rmx {

// The step's own fields of one solid (the extrapolation's DevSolid carries xi^{n+1} as
// xi, the labels at n + 1 as labels, the interior mask and the box).
struct StepDev {
    const double* xi_n;       // [3][ncell] xi^n
    const int8_t* labels_n;   // [ncell] labels at step n
    const double* u;          // [3][ncell] cell-centred velocity u^n
    const double* uf[3];      // face-normal velocities: [n2][n1][n0+1], [n2][n1+1][n0],
                              // [n2+1][n1][n0]
    double* xi_half;          // [3][ncell] xi^{n+1/2}
    double* trans;            // [3 axes][4][ncell] transverse faces (scratch)
    double* faces;            // [3 axes][2 sides][3][ncell] expansions of xi to the cell's
                              // +a face (side 0) and -a face (side 1)
};

struct StepBatch {
    const DevSolid* solids;
    const StepDev* steps;
    int32_t n_solids;
    int32_t pad_;
    int64_t total_words;      // 64-cell row segments of all boxes
    unsigned long long* stats;
    int32_t* bcount;
    BandCtl* band;
    double lam[3];            // dt / Delta_a
    double hl[3];             // dt / (2 Delta_a)
    int32_t* lists;           // [2][kStepLists][list_cap]: row segments with a cell
                              // labelled 0..L at step n (0) and at n + 1 (1), in
                              // kStepLists sub-lists (the scan's blocks b % kStepLists)
    int32_t* counts;          // [2][kStepLists]: their lengths (zero when the call starts)
    int64_t list_cap;         // entries per sub-list
};

// Sub-lists per list: a scan block appends its segments to sub-list (block % kStepLists)
// with one atomic, so the appends spread over that many counters.
constexpr int kStepLists = 8;
// Row segments per scan block (16 per wave).
constexpr int kStepScanWords = 64;
// Entries per sub-list for a batch of `words` row segments.
inline int64_t step_list_cap(int64_t words) {
    const int64_t blocks = (words + kStepScanWords - 1) / kStepScanWords;
    return (blocks + kStepLists - 1) / kStepLists * kStepScanWords;
}

// Lists the row segments labelled at step n (which = 0: also zeroes the call's statistics,
// counters and interior masks, as the classification does in an extrapolation call) or
// at n + 1 (which = 1).
hipError_t launch_step_scan(const StepBatch& b, int which, hipStream_t st);
// Transverse face states and advecting velocities.
hipError_t launch_step_trans(const StepBatch& b, hipStream_t st);
// Expansions of xi from the cells next to predicted cells to their faces.
hipError_t launch_step_faces(const StepBatch& b, hipStream_t st);
// Predictor, the rest of the old band undefined, the interior mask at n + 1.
hipError_t launch_step_predict(const StepBatch& b, hipStream_t st);
// Corrector on the cells labelled at n + 1.
hipError_t launch_step_correct(const StepBatch& b, hipStream_t st);

}  // namespace rmx
