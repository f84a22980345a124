// Operator kernels of the compressible Euler equations.
#include "st_ops_impl.hpp"

namespace stdg {
// the three temporal degrees and the one-time-level operator
#define ST_NT3(EQ, D, N1)                       \
    t.push_back(make_table<EQ, D, N1, 2>());    \
    t.push_back(make_table<EQ, D, N1, 3>());    \
    t.push_back(make_table<EQ, D, N1, 4>());    \
    t.push_back(make_spatial_table<EQ, D, N1>());

void register_ops_euler(std::vector<OpTable>& t) {
    ST_NT3(EQ_EULER, 1, 2) ST_NT3(EQ_EULER, 1, 3) ST_NT3(EQ_EULER, 1, 4) ST_NT3(EQ_EULER, 1, 5)
    ST_NT3(EQ_EULER, 2, 2) ST_NT3(EQ_EULER, 2, 3) ST_NT3(EQ_EULER, 2, 4) ST_NT3(EQ_EULER, 2, 5)
    ST_NT3(EQ_EULER, 3, 2) ST_NT3(EQ_EULER, 3, 3) ST_NT3(EQ_EULER, 3, 4) ST_NT3(EQ_EULER, 3, 5)
}
}  // namespace stdg
