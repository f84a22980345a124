// Operator kernels of advection-diffusion with the BR1 viscous flux.
#include "st_ops_impl.hpp"

namespace stdg {
// the three temporal degrees and the one-time-level operator
#define ST_NT3(EQ, D, N1)                       \
    t.push_back(make_table<EQ, D, N1, 2>());    \
    t.push_back(make_table<EQ, D, N1, 3>());    \
    t.push_back(make_table<EQ, D, N1, 4>());    \
    t.push_back(make_spatial_table<EQ, D, N1>());

void register_ops_advdiff(std::vector<OpTable>& t) {
    ST_NT3(EQ_ADVDIFF, 1, 2) ST_NT3(EQ_ADVDIFF, 1, 3) ST_NT3(EQ_ADVDIFF, 1, 4) ST_NT3(EQ_ADVDIFF, 1, 5) ST_NT3(EQ_ADVDIFF, 1, 6)
    ST_NT3(EQ_ADVDIFF, 2, 2) ST_NT3(EQ_ADVDIFF, 2, 3) ST_NT3(EQ_ADVDIFF, 2, 4) ST_NT3(EQ_ADVDIFF, 2, 5) ST_NT3(EQ_ADVDIFF, 2, 6)
    ST_NT3(EQ_ADVDIFF, 3, 2) ST_NT3(EQ_ADVDIFF, 3, 3) ST_NT3(EQ_ADVDIFF, 3, 4) ST_NT3(EQ_ADVDIFF, 3, 5)
}
}  // namespace stdg
