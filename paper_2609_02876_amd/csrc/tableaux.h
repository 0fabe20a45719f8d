// Coefficients of the explicit Runge-Kutta pairs of the paper (Sections 2.1
// and 3.2), in Butcher form: nodes are implied by the row sums of A, B are
// the propagating weights and EW = b - bhat the weights of the embedded
// error estimate (its sign is immaterial: only |e| enters the RMS test).
// Zero entries are skipped at compile time by the stage loops.
#pragma once

namespace ens {

// Tsitouras (2011): 5(4) pair, 7 stages, the last stage input is the new
// state (first same as last).
struct Tsit5 {
  static constexpr int S = 7;       // stages formed by a trial step
  static constexpr int SU = 6;      // stages that enter the update (b_7 = 0)
  static constexpr bool FSAL = true;
  static constexpr bool ROS = false;
  static constexpr int ORDER = 5;
  static constexpr int QEMB = 4;    // order of the embedded solution
  static constexpr double A[7][7] = {
      {0, 0, 0, 0, 0, 0, 0},
      {0.161, 0, 0, 0, 0, 0, 0},
      {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0, 0},
      {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0, 0},
      {5.325864828439257, -11.748883564062828, 7.4955393428898365,
       -0.09249506636175525, 0, 0, 0},
      {5.86145544294642, -12.92096931784711, 8.159367898576159,
       -0.071584973281401, -0.028269050394068383, 0, 0},
      {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742,
       -3.290069515436081, 2.324710524099774, 0}};
  static constexpr double B[7] = {0.09646076681806523, 0.01,
                                  0.4798896504144996,  1.379008574103742,
                                  -3.290069515436081,  2.324710524099774, 0};
  static constexpr double EW[7] = {
      -0.00178001105222577714, -0.0008164344596567469, 0.007880878010261995,
      -0.1447110071732629,     0.5823571654525552,     -0.45808210592918697,
      0.015151515151515152};
};

// Verner (2010): 7(6) pair, 10 stages; b uses stages 1,4..9 and bhat
// stages 1,4..7,10.
struct Vern7 {
  static constexpr int S = 10;
  static constexpr int SU = 9;
  static constexpr bool FSAL = false;
  static constexpr bool ROS = false;
  static constexpr int ORDER = 7;
  static constexpr int QEMB = 6;
  static constexpr double A[10][10] = {
      {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
      {0.005, 0, 0, 0, 0, 0, 0, 0, 0, 0},
      {-1.07679012345679, 1.185679012345679, 0, 0, 0, 0, 0, 0, 0, 0},
      {0.04083333333333333, 0, 0.1225, 0, 0, 0, 0, 0, 0, 0},
      {0.6389139236255726, 0, -2.455672638223657, 2.272258714598084, 0, 0, 0,
       0, 0, 0},
      {-2.6615773750187572, 0, 10.804513886456137, -8.3539146573962,
       0.820487594956657, 0, 0, 0, 0, 0},
      {6.067741434696772, 0, -24.711273635911088, 20.427517930788895,
       -1.9061579788166472, 1.006172249242068, 0, 0, 0, 0},
      {12.054670076253203, 0, -49.75478495046899, 41.142888638604674,
       -4.461760149974004, 2.042334822239175, -0.09834843665406107, 0, 0, 0},
      {10.138146522881808, 0, -42.6411360317175, 35.76384003992257,
       -4.3480228403929075, 2.0098622683770357, 0.3487490460338272,
       -0.27143900510483127, 0, 0},
      {-45.030072034298676, 0, 187.3272437654589, -154.02882369350186,
       18.56465306347536, -7.141809679295079, 1.3088085781613787, 0, 0, 0}};
  static constexpr double B[10] = {0.04715561848627222, 0, 0,
                                   0.25750564298434153, 0.26216653977412624,
                                   0.15216092656738558, 0.4939969170032485,
                                   -0.29430311714032503, 0.08131747232495111,
                                   0};
  static constexpr double EW[10] = {
      0.0025470118799348416, 0, 0, -0.009658394872807551, 0.04206470975642573,
      -0.06668224374695614, 0.26500974646213266, -0.29430311714032503,
      0.08131747232495111, -0.020295184663355476};
};

// Rodas4 (Hairer & Wanner, Solving ODEs II, Sec. IV.7): stiffly accurate
// Rosenbrock-Wanner method of order 4 with an embedded order-3 solution,
// in the transformed variables u_i = h sum_j gamma_ij k_j (W = I/(gamma h) - J):
//   Y_i = y + sum_{j<i} A_ij u_j,   W u_i = f(Y_i) + (1/h) sum_{j<i} C_ij u_j,
//   y_new = Y_6 + u_6 = y + sum_j M_j u_j,   error estimate u_6.
// Fields shared by the Rosenbrock methods: S stages, the first SU of which
// enter y_new; NEW_AT_INPUT: y_new is the input Y_S of the last stage
// (otherwise Y_S + u_S); the error estimate is sum_j E_j u_j.
struct Rodas4 {
  static constexpr int S = 6;
  static constexpr int SU = 6;
  static constexpr bool FSAL = false;
  static constexpr bool ROS = true;
  static constexpr bool NEW_AT_INPUT = false;
  static constexpr int ORDER = 4;
  static constexpr int QEMB = 3;
  static constexpr double GAMMA = 0.25;
  static constexpr double A[6][6] = {
      {0, 0, 0, 0, 0, 0},
      {1.544, 0, 0, 0, 0, 0},
      {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
      {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
      {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
      {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0}};
  static constexpr double C[6][6] = {
      {0, 0, 0, 0, 0, 0},
      {-5.6688, 0, 0, 0, 0, 0},
      {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
      {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
      {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
      {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
       -6.058818238834054, 0}};
  static constexpr double M[6] = {1.221224509226641, 6.019134481288629, 12.53708332932087,
                                  -0.6878860361058950, 1.0, 1.0};
  static constexpr double E[6] = {0, 0, 0, 0, 0, 1.0};
};

// Rosenbrock23 (Shampine & Reichelt 1997, MATLAB's ode23s) for autonomous
// fields, order 2 with an O(h^3) error estimate.  With d = 1/(2 + sqrt 2) and
// e32 = 6 + sqrt 2 the published slope form is
//   W = I - h d J,  W k1 = f(y),  W (k2 - k1) = f(y + h k1/2) - k1,
//   y_new = y + h k2,  W k3 = f(y_new) - e32 (k2 - f(y + h k1/2)) - 2 (k1 - f(y)),
//   error (h/6)(k1 - 2 k2 + k3).
// Since k1 - f(y) = h d J k1 and k2 - f(y + h k1/2) = h d J (k2 - k1), it is
// the Rosenbrock method with gamma = d, alpha_21 = 1/2, alpha_32 = 1,
// gamma_21 = -d, gamma_31 = (e32 - 2) d, gamma_32 = -e32 d, b = (0, 1, 0);
// in the transformed variables (Gamma^{-1} = [[1,0,0],[1,1,0],[2,e32,1]]/d):
//   A_21 = 1/(2d), A_31 = A_32 = 1/d;  C_21 = -1/d, C_31 = -2/d, C_32 = -e32/d;
//   y_new = Y_3 = y + (u_1 + u_2)/d;  error (u_1 + (e32 - 2) u_2 + u_3)/(6d).
// The third stage serves the error estimate only, so a replay takes two.
struct Ros23 {
  static constexpr int S = 3;
  static constexpr int SU = 2;
  static constexpr bool FSAL = false;
  static constexpr bool ROS = true;
  static constexpr bool NEW_AT_INPUT = true;
  static constexpr int ORDER = 2;
  static constexpr int QEMB = 2;
  static constexpr double GAMMA = 0.2928932188134525;
  static constexpr double A[3][3] = {{0, 0, 0},
                                     {1.7071067811865475, 0, 0},
                                     {3.414213562373095, 3.414213562373095, 0}};
  static constexpr double C[3][3] = {{0, 0, 0},
                                     {-3.414213562373095, 0, 0},
                                     {-6.82842712474619, -25.31370849898476, 0}};
  static constexpr double M[3] = {3.414213562373095, 3.414213562373095, 0};
  static constexpr double E[3] = {0.5690355937288492, 3.080880229039762, 0.5690355937288492};
};

}  // namespace ens
