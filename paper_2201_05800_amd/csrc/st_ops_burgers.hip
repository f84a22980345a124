// Operator kernels of the inviscid Burgers equation (one space dimension).
#include "st_ops_impl.hpp"

namespace stdg {
// the three temporal degrees and the one-time-level operator
#define ST_NT3(EQ, D, N1)                       \
    t.push_back(make_table<EQ, D, N1, 2>());    \
    t.push_back(make_table<EQ, D, N1, 3>());    \
    t.push_back(make_table<EQ, D, N1, 4>());    \
    t.push_back(make_spatial_table<EQ, D, N1>());

void register_ops_burgers(std::vector<OpTable>& t) {
    ST_NT3(EQ_BURGERS, 1, 2) ST_NT3(EQ_BURGERS, 1, 3) ST_NT3(EQ_BURGERS, 1, 4) ST_NT3(EQ_BURGERS, 1, 5) ST_NT3(EQ_BURGERS, 1, 6)
}
}  // namespace stdg
