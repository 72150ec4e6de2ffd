// rn_dopri.h -- the Dormand-Prince 5(4) tableau (J. R. Dormand, P. J. Prince,
// J. Comput. Appl. Math. 6 (1980) 19) used by the rate-equation and hybrid
// sweeps: stage coefficients A, fifth-order weights B and the error weights
// E = B - B* of the embedded fourth-order solution (FSAL: the seventh stage is
// f at the new state).  The systems are autonomous, so no stage times.
#pragma once

namespace rn {
namespace dopri {

constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 44.0 / 45.0, A42 = -56.0 / 15.0, A43 = 32.0 / 9.0;
constexpr double A51 = 19372.0 / 6561.0, A52 = -25360.0 / 2187.0, A53 = 64448.0 / 6561.0,
                 A54 = -212.0 / 729.0;
constexpr double A61 = 9017.0 / 3168.0, A62 = -355.0 / 33.0, A63 = 46732.0 / 5247.0,
                 A64 = 49.0 / 176.0, A65 = -5103.0 / 18656.0;
constexpr double B1 = 35.0 / 384.0, B3 = 500.0 / 1113.0, B4 = 125.0 / 192.0,
                 B5 = -2187.0 / 6784.0, B6 = 11.0 / 84.0;
constexpr double E1 = 71.0 / 57600.0, E3 = -71.0 / 16695.0, E4 = 71.0 / 1920.0,
                 E5 = -17253.0 / 339200.0, E6 = 22.0 / 525.0, E7 = -1.0 / 40.0;

}  // namespace dopri
}  // namespace rn
