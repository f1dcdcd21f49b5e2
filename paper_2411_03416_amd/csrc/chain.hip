// Dispatch of the chain kernels over the supported state dimensions (each
// dimension is compiled in its own translation unit, chain_n<k>.hip).
#include "ctx.h"

namespace pg {

template <int n>
hipError_t launch_chain_n(const DevState& st, int mode, int lo, int hi, hipStream_t s);
template <int n>
hipError_t launch_prior_costs_n(const DevState& st, int plan, int N, hipStream_t s);
template <int n>
hipError_t launch_iteration_n(const DevState& st, int phw, int part, int round, hipStream_t s);

bool chain_supported(int n) { return n == 2 || n == 4 || n == 6 || n == 8 || n == 14; }

hipError_t launch_chain(const DevState& st, int mode, int lo, int hi, hipStream_t s) {
    switch (st.n) {
        case 2: return launch_chain_n<2>(st, mode, lo, hi, s);
        case 4: return launch_chain_n<4>(st, mode, lo, hi, s);
        case 6: return launch_chain_n<6>(st, mode, lo, hi, s);
        case 8: return launch_chain_n<8>(st, mode, lo, hi, s);
        case 14: return launch_chain_n<14>(st, mode, lo, hi, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_iteration(const DevState& st, int phw, int part, int round, hipStream_t s) {
    switch (st.n) {
        case 2: return launch_iteration_n<2>(st, phw, part, round, s);
        case 4: return launch_iteration_n<4>(st, phw, part, round, s);
        case 6: return launch_iteration_n<6>(st, phw, part, round, s);
        case 8: return launch_iteration_n<8>(st, phw, part, round, s);
        case 14: return launch_iteration_n<14>(st, phw, part, round, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_prior_costs(const DevState& st, int plan, int N, hipStream_t s) {
    switch (st.n) {
        case 2: return launch_prior_costs_n<2>(st, plan, N, s);
        case 4: return launch_prior_costs_n<4>(st, plan, N, s);
        case 6: return launch_prior_costs_n<6>(st, plan, N, s);
        case 8: return launch_prior_costs_n<8>(st, plan, N, s);
        case 14: return launch_prior_costs_n<14>(st, plan, N, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pg
