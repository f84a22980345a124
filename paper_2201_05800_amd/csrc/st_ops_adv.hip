// Operator kernels of linear advection, u_t + a . grad u = 0.
#include "st_ops_impl.hpp"

namespace stdg {
// the three temporal degrees and the one-time-level operator
#define ST_NT3(EQ, D, N1)                       \
    t.push_back(make_table<EQ, D, N1, 2>());    \
    t.push_back(make_table<EQ, D, N1, 3>());    \
    t.push_back(make_table<EQ, D, N1, 4>());    \
    t.push_back(make_spatial_table<EQ, D, N1>());

void register_ops_adv(std::vector<OpTable>& t) {
    ST_NT3(EQ_ADV, 1, 2) ST_NT3(EQ_ADV, 1, 3) ST_NT3(EQ_ADV, 1, 4) ST_NT3(EQ_ADV, 1, 5) ST_NT3(EQ_ADV, 1, 6)
    ST_NT3(EQ_ADV, 2, 2) ST_NT3(EQ_ADV, 2, 3) ST_NT3(EQ_ADV, 2, 4) ST_NT3(EQ_ADV, 2, 5) ST_NT3(EQ_ADV, 2, 6)
    ST_NT3(EQ_ADV, 3, 2) ST_NT3(EQ_ADV, 3, 3) ST_NT3(EQ_ADV, 3, 4) ST_NT3(EQ_ADV, 3, 5)
}
}  // namespace stdg
