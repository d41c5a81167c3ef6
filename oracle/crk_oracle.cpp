// CPU oracle for the CRK-SPH pair passes and short-range gravity.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct FP64
// reference that the GPU library is checked against.  Only the tests, the
// smoke check and the benchmark's CPU-baseline leg may load it; the product
// path never does, and this file shares no code, header or table with the GPU
// library.
//
// Everything is FP64 and every neighbour search is brute force: for a particle
// i the candidate set is scanned in full and each candidate is tested with the
// periodic minimum image.  No tree, no cell list, no blocking.
//
// What is computed (the paper names the passes -- Geometry, Corrections,
// Acceleration, Energy, Sec. 5 -- and cites conservative reproducing-kernel
// SPH for the method, Sec. 3.1, without printing its equations; the formulas
// below are linear CRK-SPH written out from its mathematics):
//
//   geometry     x_ij = x_i - x_j, each component wrapped to [-1/2, 1/2)
//   kernel       Wendland C4, support H = 2h:
//                  W = 495/(32 pi H^3) (1-q)^6 (1 + 6q + 35 q^2/3),  q = r/H < 1
//                  grad_i W = F x_ij,  F = -1155/(4 pi H^5) (1+5q)(1-q)^5
//   volume       S_i = sum_{j: r_ij < H_i} W(r_ij, h_i)  (j = i included)
//                V_i = 1/S_i,  rho_i = m_i S_i
//   moments      with W_ij = W(r_ij, h_i), d_c W_ij = F(r_ij, h_i) x_ij^c, over
//                j with r_ij < H_i (j = i included):
//                  m0 = sum V_j W,  m1^a = sum V_j x^a W,  m2^ab = sum V_j x^a x^b W
//                  g0^c = sum V_j d_cW,  g1^ac = sum V_j (delta^ac W + x^a d_cW)
//                  g2^abc = sum V_j (delta^ac x^b W + delta^bc x^a W + x^a x^b d_cW)
//   corrections  B = -m2^-1 m1,  A = 1/(m0 + B.m1)
//                d_cB = -m2^-1 (g1[.,c] + g2[.,.,c] B)
//                d_cA = -A^2 (g0^c + B.g1[.,c] + m1.d_cB)
//                (these make sum_j V_j W^R_ij = 1 and sum_j V_j x_ij W^R_ij = 0
//                 with W^R_ij = A_i (1 + B_i.x_ij) W_ij)
//   EOS          P_i = (gamma - 1) rho_i u_i
//   forces       j != i with r_ij < max(H_i, H_j):
//                  G_ij^c = d_cA_i (1+B_i.x_ij) W_ij + A_i (d_cB_i.x_ij + B_i^c) W_ij
//                           + A_i (1+B_i.x_ij) d_cW_ij
//                  G_ji   = the same with i <-> j (x_ji = -x_ij, h_j)
//                  F_ij   = -1/2 V_i V_j (P_i + P_j) (G_ij - G_ji)
//                  a_i    = (1/m_i) sum_j F_ij
//                  du_i/dt = -(1/(2 m_i)) sum_j F_ij . (v_i - v_j)
//   extras       over the gather support (j with r_ij < H_i), W^R_ij = A_i (1 + B_i.x_ij) W_ij,
//                G_ij its x_i-gradient (as in the forces):
//                  rhoR_i = sum_j m_j W^R_ij  (j = i included: m_i A_i W(0, h_i))
//                  dv_i[a][c] = sum_{j != i} V_j (v_j^a - v_i^a) G_ij^c,
//                  du_i[c]    = sum_{j != i} V_j (u_j - u_i) G_ij^c
//                (exact for linear fields, by the reproducing conditions)
//   viscosity    (optional in the forces) per force pair, s_k = x_ij . (dv_k x_ij),
//                  Phi = max(0, 4 s_i s_j / (s_i + s_j)^2)   (van Leer on s_i / s_j)
//                  w = v_i - v_j - Phi/2 (dv_i + dv_j) x_ij   (velocities reconstructed
//                                                          to the pair's midpoint)
//                  mu_k = min(0, h_k (w.x_ij) / (r^2 + eps_q h_k^2)),  c_k = sqrt(gamma (gamma-1) u_k)
//                  Q_k = rho_k (-C_l c_k mu_k + C_q mu_k^2)              (k = i, j)
//                and P_i + P_j in F_ij becomes P_i + P_j + Q_i + Q_j (still F_ij = -F_ji)
//   compatible   (optional energy partition) each pair's work W_ij = (v_j - v_i) . F_ij
//   energy         (= W_ji) is split f_ij W_ij to i and f_ji W_ij to j, f_ij + f_ji = 1:
//                  du_i/dt = (1/m_i) sum_j f_ij W_ij,
//                  f_ij = 1/2 [1 + sgn(W_ij) (u_j - u_i) / (|u_j - u_i| + eps_u (u_i + u_j))]
//                (heating goes mostly to the colder particle, cooling comes mostly
//                 from the hotter; f_ij = 1/2 gives the symmetric form above)
//   gravity      j != i with r_ij < r_c (all species):
//                  a_i = -G sum_j m_j x_ij [ (r^2 + eps^2)^(-3/2) - sum_k p_k r^(2k) ]
//   PM split     the polynomial stands for the long-range (particle-mesh)
//                part of the force, here that of a mesh potential filtered by
//                exp(-k^2 r_s^2): per unit mass f_L(r) = M(<r)/r^2 for a
//                Gaussian cloud of variance 2 r_s^2 per axis,
//                  f_L(r) = [erf(x) - (2x/sqrt(pi)) exp(-x^2)] / r^2,  x = r/(2 r_s),
//                and sum_k p_k s^k is the least-squares fit of f_L(sqrt s)/sqrt s
//                over s in [0, r_c^2] (oracle/__init__.py, fit_poly)
//   gravity adjoint  L = sum_i abar_i . a_i:  dL/dx by forward-mode dual numbers
//                and by central differences (masses held fixed)
//
// Moment storage order (40 values): m0, m1[3], m2[6] (xx xy xz yy yz zz),
// g0[3], g1[9] (g1[a][c], a-major), g2[18] (g2[ab][c], ab in the m2 order).
// Correction layout: dA[c] = d_cA, dB[a][c] = d_cB^a (a-major).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <map>
#include <tuple>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- scalars
// T is double for values; a forward-mode dual number for gradients.
struct Dual {
    double v, d;
    Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, s > 0 ? a.d / (2.0 * s) : 0.0}; }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
using std::sqrt;

// ---------------------------------------------------------------- operation counting
// Ops records every arithmetic operation into an expression graph (one per
// thread), so that the oracle's own per-pair code can be counted.  Each value
// carries the set of particles it depends on (bit 0: the particle whose sums
// are formed, bits 1 and 2: two of its neighbours).  A value that depends on
// one particle alone is per-particle work, computed once outside the pair loop;
// only operations on values that combine two particles are pair work.
// Identical operations are recorded once (common subexpressions), constants
// are folded, and the algebraic identities a+0, a*1, a*0, -(-a), and a sign
// moved out of products, quotients and differences are applied, so that
// evaluating a quantity from x_ji = -x_ij costs nothing beyond evaluating it
// from x_ij.  Counting: add, sub, mul, div, sqrt = 1 FLOP each (so a
// multiply-add is 2); negation is free (a sign on an operand).
struct OpNode {
    char op;    // 'L' leaf/constant, '+', '-', '*', '/', 'n' (negate), 's' (sqrt)
    int a, b;   // operand node ids
    unsigned mask;
    double v;
};

struct OpGraph {
    std::vector<OpNode> nodes;
    std::map<std::tuple<char, int, int>, int> memo;
    std::map<double, int> consts;
};
inline OpGraph& op_graph() {
    static thread_local OpGraph g;
    return g;
}

struct Ops {
    int id;
    Ops() : Ops(0.0) {}
    Ops(double c) {
        OpGraph& g = op_graph();
        auto it = g.consts.find(c);
        if (it != g.consts.end()) { id = it->second; return; }
        id = int(g.nodes.size());
        g.nodes.push_back({'L', -1, -1, 0u, c});
        g.consts[c] = id;
    }
    static Ops from_id(int i) { Ops o(0.0); o.id = i; return o; }
    // a new independent input value that depends on the particles in `mask`
    static Ops leaf(double v, unsigned mask) {
        OpGraph& g = op_graph();
        Ops o(0.0);
        o.id = int(g.nodes.size());
        g.nodes.push_back({'L', -1, -1, mask, v});
        return o;
    }
    const OpNode& node() const { return op_graph().nodes[id]; }
    bool is_const(double c) const { return node().op == 'L' && node().mask == 0u && node().v == c; }
    bool is_const() const { return node().op == 'L' && node().mask == 0u; }
};
inline double val(Ops a) { return a.node().v; }

inline Ops op_make(char op, Ops a, Ops b, double v) {
    OpGraph& g = op_graph();
    if (a.is_const() && (op == 'n' || op == 's' || b.is_const())) return Ops(v);  // constant folding
    auto key = std::make_tuple(op, a.id, b.id);
    auto it = g.memo.find(key);
    if (it != g.memo.end()) return Ops::from_id(it->second);
    const unsigned mask = a.node().mask | (b.id >= 0 ? b.node().mask : 0u);
    const int id = int(g.nodes.size());
    g.nodes.push_back({op, a.id, b.id, mask, v});
    g.memo[key] = id;
    return Ops::from_id(id);
}
inline Ops operator-(Ops a) {
    if (a.node().op == 'n') return Ops::from_id(a.node().a);
    OpGraph& g = op_graph();
    if (a.is_const()) return Ops(-val(a));
    auto key = std::make_tuple('n', a.id, -1);
    auto it = g.memo.find(key);
    if (it != g.memo.end()) return Ops::from_id(it->second);
    const int id = int(g.nodes.size());
    g.nodes.push_back({'n', a.id, -1, a.node().mask, -val(a)});
    g.memo[key] = id;
    return Ops::from_id(id);
}
inline bool is_neg(Ops a) { return a.node().op == 'n'; }
inline Ops un_neg(Ops a) { return Ops::from_id(a.node().a); }
inline Ops operator*(Ops a, Ops b) {
    if (a.is_const(0.0) || b.is_const(0.0)) return Ops(0.0);
    if (a.is_const(1.0)) return b;
    if (b.is_const(1.0)) return a;
    if (a.is_const(-1.0)) return -b;
    if (b.is_const(-1.0)) return -a;
    if (is_neg(a)) return -(un_neg(a) * b);
    if (is_neg(b)) return -(a * un_neg(b));
    if (a.id > b.id) std::swap(a, b);
    return op_make('*', a, b, val(a) * val(b));
}
inline Ops operator/(Ops a, Ops b) {
    if (a.is_const(0.0)) return Ops(0.0);
    if (b.is_const(1.0)) return a;
    if (is_neg(a)) return -(un_neg(a) / b);
    if (is_neg(b)) return -(a / un_neg(b));
    return op_make('/', a, b, val(a) / val(b));
}
Ops operator-(Ops a, Ops b);
inline Ops operator+(Ops a, Ops b) {
    if (a.is_const(0.0)) return b;
    if (b.is_const(0.0)) return a;
    if (is_neg(a) && is_neg(b)) return -(un_neg(a) + un_neg(b));
    if (is_neg(b)) return a - un_neg(b);
    if (is_neg(a)) return b - un_neg(a);
    if (a.id > b.id) std::swap(a, b);
    return op_make('+', a, b, val(a) + val(b));
}
inline Ops operator-(Ops a, Ops b) {
    if (b.is_const(0.0)) return a;
    if (a.is_const(0.0)) return -b;
    if (is_neg(b)) return a + un_neg(b);
    if (is_neg(a)) return -(un_neg(a) + b);
    if (a.id > b.id) return -(b - a);
    return op_make('-', a, b, val(a) - val(b));
}
inline Ops& operator+=(Ops& a, Ops b) { a = a + b; return a; }
inline Ops& operator-=(Ops& a, Ops b) { a = a - b; return a; }
inline bool operator<(Ops a, Ops b) { return val(a) < val(b); }
inline bool operator>=(Ops a, Ops b) { return val(a) >= val(b); }
inline Ops sqrt(Ops a) { return op_make('s', a, Ops::from_id(-1), std::sqrt(val(a))); }

inline void op_reset() {
    OpGraph& g = op_graph();
    g.nodes.clear();
    g.memo.clear();
    g.consts.clear();
}

// Pair work among the values needed for `roots`: operations whose operands
// combine the lane particle (bit 0) with a neighbour, or two neighbours.
inline int64_t pair_flops(const std::vector<Ops>& roots) {
    const OpGraph& g = op_graph();
    std::vector<char> seen(g.nodes.size(), 0);
    std::vector<int> stack;
    for (const Ops& r : roots) stack.push_back(r.id);
    int64_t count = 0;
    while (!stack.empty()) {
        const int id = stack.back();
        stack.pop_back();
        if (id < 0 || seen[id]) continue;
        seen[id] = 1;
        const OpNode& nd = g.nodes[id];
        if (nd.op == 'L') continue;
        if (nd.op != 'n' && __builtin_popcount(nd.mask) >= 2) ++count;
        stack.push_back(nd.a);
        stack.push_back(nd.b);
    }
    return count;
}

// Reverse-mode derivative of `out` with respect to `wanted`, recorded in the
// same graph: every node's adjoint is formed from its consumers' adjoints in
// reverse order of creation (the standard adjoint sweep, restricted to nodes
// that depend on a wanted input).  Returns the adjoint of each wanted input.
inline std::vector<Ops> reverse_sweep(Ops out, const std::vector<Ops>& wanted) {
    OpGraph& g = op_graph();
    const int top = out.id;
    std::vector<char> active(top + 1, 0);
    for (const Ops& w : wanted)
        if (w.id <= top) active[w.id] = 1;
    for (int id = 0; id <= top; ++id) {
        const OpNode nd = g.nodes[id];
        if (nd.op == 'L') continue;
        active[id] = (nd.a >= 0 && active[nd.a]) || (nd.b >= 0 && active[nd.b]);
    }
    std::vector<int> adj(top + 1, -1);  // adjoint node id, -1 = none yet
    adj[top] = Ops(1.0).id;
    auto add_to = [&](int target, Ops contrib) {
        if (target < 0 || !active[target]) return;
        adj[target] = adj[target] < 0 ? contrib.id : (Ops::from_id(adj[target]) + contrib).id;
    };
    for (int id = top; id >= 0; --id) {
        if (adj[id] < 0 || !active[id]) continue;
        const OpNode nd = g.nodes[id];
        const Ops z = Ops::from_id(id), zb = Ops::from_id(adj[id]);
        const Ops a = Ops::from_id(nd.a), b = Ops::from_id(nd.b);
        switch (nd.op) {
            case '+': add_to(nd.a, zb); add_to(nd.b, zb); break;
            case '-': add_to(nd.a, zb); add_to(nd.b, -zb); break;
            case 'n': add_to(nd.a, -zb); break;
            case '*': add_to(nd.a, zb * b); add_to(nd.b, zb * a); break;
            case '/': add_to(nd.a, zb / b); add_to(nd.b, -(zb * z / b)); break;
            case 's': add_to(nd.a, zb * (Ops(0.5) / z)); break;
            default: break;
        }
    }
    std::vector<Ops> res;
    for (const Ops& w : wanted) res.push_back(w.id <= top && adj[w.id] >= 0 ? Ops::from_id(adj[w.id]) : Ops(0.0));
    return res;
}

template <class T> T wrap(T d) {
    if (val(d) >= 0.5) d = d - T(1.0);
    else if (val(d) < -0.5) d = d + T(1.0);
    return d;
}

// ---------------------------------------------------------------- kernel
template <class T> T kernel_W(T r, double h) {
    const double H = 2.0 * h;
    T q = r / T(H);
    if (!(val(q) < 1.0)) return T(0.0);
    T t = T(1.0) - q;
    T t2 = t * t;
    T t6 = t2 * t2 * t2;
    return T(495.0 / (32.0 * kPi * H * H * H)) * t6 *
           (T(1.0) + T(6.0) * q + T(35.0 / 3.0) * q * q);
}

// grad_i W(|x_i - x_j|) = kernel_F * x_ij
template <class T> T kernel_F(T r, double h) {
    const double H = 2.0 * h;
    T q = r / T(H);
    if (!(val(q) < 1.0)) return T(0.0);
    T t = T(1.0) - q;
    T t5 = t * t * t * t * t;
    return T(-1155.0 / (4.0 * kPi * H * H * H * H * H)) * (T(1.0) + T(5.0) * q) * t5;
}

// ---------------------------------------------------------------- data
template <class T> struct Gas {
    int64_t n;
    const T *x, *y, *z, *vx, *vy, *vz, *u;
    const double *h, *m;
};

template <class T> struct Sep {
    T d[3];
    T r;
};

template <class T> Sep<T> separation(const Gas<T>& g, int64_t i, int64_t j) {
    Sep<T> s;
    s.d[0] = wrap(g.x[i] - g.x[j]);
    s.d[1] = wrap(g.y[i] - g.y[j]);
    s.d[2] = wrap(g.z[i] - g.z[j]);
    s.r = sqrt(s.d[0] * s.d[0] + s.d[1] * s.d[1] + s.d[2] * s.d[2]);
    return s;
}

// candidate set: either all particles (cand == nullptr) or an index list
struct Cand {
    const int64_t* idx;
    int64_t n;
    int64_t at(int64_t k) const { return idx ? idx[k] : k; }
};

// ---------------------------------------------------------------- volume
template <class T> T volume_sum(const Gas<T>& g, int64_t i, Cand c) {
    const double H = 2.0 * g.h[i];
    T S = kernel_W(T(0.0), g.h[i]);  // j = i
    for (int64_t k = 0; k < c.n; ++k) {
        const int64_t j = c.at(k);
        if (j == i) continue;
        Sep<T> s = separation(g, i, j);
        if (val(s.r) < H) S += kernel_W(s.r, g.h[i]);
    }
    return S;
}

// ---------------------------------------------------------------- moments
constexpr int kSym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};  // (a,b) -> xx xy xz yy yz zz

template <class T> struct Moments {
    T m0, m1[3], m2[6], g0[3], g1[3][3], g2[6][3];
    int nnb;  // neighbours j != i inside the support
};

template <class T> void moments_one(const Gas<T>& g, const T* V, int64_t i, Cand c, Moments<T>& M) {
    const double H = 2.0 * g.h[i];
    M.m0 = T(0.0);
    for (int a = 0; a < 3; ++a) { M.m1[a] = T(0.0); M.g0[a] = T(0.0); }
    for (int p = 0; p < 6; ++p) { M.m2[p] = T(0.0); for (int cc = 0; cc < 3; ++cc) M.g2[p][cc] = T(0.0); }
    for (int a = 0; a < 3; ++a) for (int cc = 0; cc < 3; ++cc) M.g1[a][cc] = T(0.0);
    M.nnb = 0;
    auto add = [&](int64_t j, const T x[3], T W, T Fv) {
        const T Vj = V[j];
        T dW[3] = {Fv * x[0], Fv * x[1], Fv * x[2]};
        M.m0 += Vj * W;
        for (int a = 0; a < 3; ++a) {
            M.m1[a] += Vj * x[a] * W;
            M.g0[a] += Vj * dW[a];
        }
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) M.m2[kSym[a][b]] += Vj * x[a] * x[b] * W;
        for (int a = 0; a < 3; ++a)
            for (int cc = 0; cc < 3; ++cc)
                M.g1[a][cc] += Vj * ((a == cc ? W : T(0.0)) + x[a] * dW[cc]);
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b)
                for (int cc = 0; cc < 3; ++cc)
                    M.g2[kSym[a][b]][cc] += Vj * ((a == cc ? x[b] * W : T(0.0)) +
                                                  (b == cc ? x[a] * W : T(0.0)) +
                                                  x[a] * x[b] * dW[cc]);
    };
    {   // j = i: x_ii = 0
        const T zero[3] = {T(0.0), T(0.0), T(0.0)};
        add(i, zero, kernel_W(T(0.0), g.h[i]), kernel_F(T(0.0), g.h[i]));
    }
    for (int64_t k = 0; k < c.n; ++k) {
        const int64_t j = c.at(k);
        if (j == i) continue;
        Sep<T> s = separation(g, i, j);
        if (!(val(s.r) < H)) continue;
        M.nnb += 1;
        add(j, s.d, kernel_W(s.r, g.h[i]), kernel_F(s.r, g.h[i]));
    }
}

// ---------------------------------------------------------------- corrections
template <class T> struct Corr {
    T A, B[3], dA[3], dB[3][3];  // dB[a][c] = d_c B^a
};

// Inverse of a symmetric 3x3 matrix by its adjugate; returns the determinant.
template <class T> T inverse_sym3(const T s[6], T inv[3][3]) {
    const T a = s[0], b = s[1], c = s[2], d = s[3], e = s[4], f = s[5];
    // matrix [[a b c][b d e][c e f]]
    T c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    T c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    T det = a * c00 + b * c01 + c * c02;
    T r = T(1.0) / det;
    inv[0][0] = c00 * r; inv[0][1] = c01 * r; inv[0][2] = c02 * r;
    inv[1][0] = c01 * r; inv[1][1] = c11 * r; inv[1][2] = c12 * r;
    inv[2][0] = c02 * r; inv[2][1] = c12 * r; inv[2][2] = c22 * r;
    return det;
}

// Returns 1 when the zeroth-order fallback was taken (fewer than 4 neighbours
// or a near-singular second moment), 0 otherwise.
template <class T> int solve_corrections(const Moments<T>& M, Corr<T>& C) {
    T inv[3][3];
    T det = inverse_sym3(M.m2, inv);
    T tr3 = (M.m2[0] + M.m2[3] + M.m2[5]) / T(3.0);
    const bool singular = M.nnb < 4 || !(val(det) > 1e-12 * val(tr3) * val(tr3) * val(tr3));
    if (singular) {
        C.A = T(1.0) / M.m0;
        for (int cc = 0; cc < 3; ++cc) {
            C.B[cc] = T(0.0);
            C.dA[cc] = -M.g0[cc] / (M.m0 * M.m0);
            for (int a = 0; a < 3; ++a) C.dB[a][cc] = T(0.0);
        }
        return 1;
    }
    for (int a = 0; a < 3; ++a) {
        T s = T(0.0);
        for (int b = 0; b < 3; ++b) s += inv[a][b] * M.m1[b];
        C.B[a] = -s;
    }
    T BM1 = C.B[0] * M.m1[0] + C.B[1] * M.m1[1] + C.B[2] * M.m1[2];
    C.A = T(1.0) / (M.m0 + BM1);
    for (int cc = 0; cc < 3; ++cc) {
        // rhs^a = g1[a][c] + sum_b g2[ab][c] B^b
        T rhs[3];
        for (int a = 0; a < 3; ++a) {
            T s = M.g1[a][cc];
            for (int b = 0; b < 3; ++b) s += M.g2[kSym[a][b]][cc] * C.B[b];
            rhs[a] = s;
        }
        for (int a = 0; a < 3; ++a) {
            T s = T(0.0);
            for (int b = 0; b < 3; ++b) s += inv[a][b] * rhs[b];
            C.dB[a][cc] = -s;
        }
        T s = M.g0[cc];
        for (int a = 0; a < 3; ++a) s += C.B[a] * M.g1[a][cc] + M.m1[a] * C.dB[a][cc];
        C.dA[cc] = -(C.A * C.A) * s;
    }
    return 0;
}

// ---------------------------------------------------------------- forces
// gradient of the corrected kernel of particle `s` seen from separation x = x_s - x_o
template <class T> void corrected_gradient(const Corr<T>& C, const T x[3], T W, T Fv, T G[3]) {
    T lin = T(1.0) + C.B[0] * x[0] + C.B[1] * x[1] + C.B[2] * x[2];
    for (int cc = 0; cc < 3; ++cc) {
        T dBx = C.dB[0][cc] * x[0] + C.dB[1][cc] * x[1] + C.dB[2][cc] * x[2];
        G[cc] = C.dA[cc] * lin * W + C.A * (dBx + C.B[cc]) * W + C.A * lin * (Fv * x[cc]);
    }
}

// One ordered pair of the force pass: F_ij and F_ij . (v_i - v_j).
template <class T> void accel_pair(const Gas<T>& g, const T* V, const T* rho, const Corr<T>* C,
                                   double gamma, int64_t i, int64_t j, const Sep<T>& s, const T& Pi,
                                   T F[3], T& Fdotv) {
    const T Pj = T(gamma - 1.0) * rho[j] * g.u[j];
    T xji[3] = {-s.d[0], -s.d[1], -s.d[2]};
    T Gij[3], Gji[3];
    corrected_gradient(C[i], s.d, kernel_W(s.r, g.h[i]), kernel_F(s.r, g.h[i]), Gij);
    corrected_gradient(C[j], xji, kernel_W(s.r, g.h[j]), kernel_F(s.r, g.h[j]), Gji);
    const T coef = T(-0.5) * V[i] * V[j] * (Pi + Pj);
    T vij[3] = {g.vx[i] - g.vx[j], g.vy[i] - g.vy[j], g.vz[i] - g.vz[j]};
    Fdotv = T(0.0);
    for (int cc = 0; cc < 3; ++cc) {
        F[cc] = coef * (Gij[cc] - Gji[cc]);
        Fdotv += F[cc] * vij[cc];
    }
}

// ---------------------------------------------------------------- extras
// CRK density and reproducing-kernel gradients of v and u of particle i.
template <class T> void extras_one(const Gas<T>& g, const T* V, const Corr<T>* C, int64_t i, Cand c,
                                   T& rhoR, T dv[3][3], T du[3]) {
    const double H = 2.0 * g.h[i];
    const Corr<T>& Ci = C[i];
    rhoR = T(g.m[i]) * Ci.A * kernel_W(T(0.0), g.h[i]);  // j = i: x_ii = 0
    for (int a = 0; a < 3; ++a) {
        du[a] = T(0.0);
        for (int cc = 0; cc < 3; ++cc) dv[a][cc] = T(0.0);
    }
    const T vi[3] = {g.vx[i], g.vy[i], g.vz[i]};
    for (int64_t k = 0; k < c.n; ++k) {
        const int64_t j = c.at(k);
        if (j == i) continue;
        Sep<T> s = separation(g, i, j);
        if (!(val(s.r) < H)) continue;
        const T W = kernel_W(s.r, g.h[i]);
        const T lin = T(1.0) + Ci.B[0] * s.d[0] + Ci.B[1] * s.d[1] + Ci.B[2] * s.d[2];
        rhoR += T(g.m[j]) * Ci.A * lin * W;
        T G[3];
        corrected_gradient(Ci, s.d, W, kernel_F(s.r, g.h[i]), G);
        const T vj[3] = {g.vx[j], g.vy[j], g.vz[j]};
        const T fu = g.u[j] - g.u[i];
        for (int cc = 0; cc < 3; ++cc) {
            for (int a = 0; a < 3; ++a) dv[a][cc] += V[j] * (vj[a] - vi[a]) * G[cc];
            du[cc] += V[j] * fu * G[cc];
        }
    }
}

// Artificial viscosity parameters and the velocity gradients it reads
// (dv[9 i + 3 a + c] = d_c v^a of particle i).
template <class T> struct Visc {
    const T* dv = nullptr;
    double Cl = 1.0, Cq = 2.0, eps_q = 0.01;
};

// Q_i + Q_j of one force pair (see the header).
template <class T> T visc_pair(const Gas<T>& g, const T* rho, double gamma, const Visc<T>& q, int64_t i,
                               int64_t j, const Sep<T>& s) {
    T Di[3], Dj[3];
    for (int a = 0; a < 3; ++a) {
        Di[a] = T(0.0);
        Dj[a] = T(0.0);
        for (int cc = 0; cc < 3; ++cc) {
            Di[a] += q.dv[9 * i + 3 * a + cc] * s.d[cc];
            Dj[a] += q.dv[9 * j + 3 * a + cc] * s.d[cc];
        }
    }
    const T si = s.d[0] * Di[0] + s.d[1] * Di[1] + s.d[2] * Di[2];
    const T sj = s.d[0] * Dj[0] + s.d[1] * Dj[1] + s.d[2] * Dj[2];
    T phi = T(0.0);
    if (val(si) * val(sj) > 0.0) phi = T(4.0) * si * sj / ((si + sj) * (si + sj));
    const T vi[3] = {g.vx[i], g.vy[i], g.vz[i]}, vj[3] = {g.vx[j], g.vy[j], g.vz[j]};
    T wx = T(0.0);
    for (int a = 0; a < 3; ++a) wx += (vi[a] - vj[a] - T(0.5) * phi * (Di[a] + Dj[a])) * s.d[a];
    const T r2 = s.r * s.r;
    T Q = T(0.0);
    const int64_t side[2] = {i, j};
    for (int k = 0; k < 2; ++k) {
        const int64_t p = side[k];
        const double hp = g.h[p];
        T mu = T(hp) * wx / (r2 + T(q.eps_q * hp * hp));
        if (!(val(mu) < 0.0)) mu = T(0.0);
        const T cs = sqrt(T(gamma * (gamma - 1.0)) * g.u[p]);
        Q += rho[p] * (T(-q.Cl) * cs * mu + T(q.Cq) * mu * mu);
    }
    return Q;
}

// Share of a pair's work W_ij = (v_j - v_i) . F_ij that goes to particle i
// under the compatible energy partition (see the header); f_ij + f_ji = 1.
template <class T> T compat_share(const T& ui, const T& uj, const T& W, double eps_u) {
    const T d = uj - ui;
    const T ad = val(d) < 0.0 ? -d : d;
    const T den = ad + T(eps_u) * (ui + uj);
    if (!(val(den) > 0.0)) return T(0.5);
    const double sw = val(W) > 0.0 ? 1.0 : (val(W) < 0.0 ? -1.0 : 0.0);
    return T(0.5) * (T(1.0) + T(sw) * d / den);
}

template <class T> void accel_one(const Gas<T>& g, const T* V, const T* rho, const Corr<T>* C,
                                  double gamma, int64_t i, Cand c, T a[3], T& dudt,
                                  const Visc<T>* visc = nullptr, const double* compat_eps = nullptr) {
    const T Pi = T(gamma - 1.0) * rho[i] * g.u[i];
    a[0] = a[1] = a[2] = T(0.0);
    dudt = T(0.0);
    for (int64_t k = 0; k < c.n; ++k) {
        const int64_t j = c.at(k);
        if (j == i) continue;
        Sep<T> s = separation(g, i, j);
        const double Hi = 2.0 * g.h[i], Hj = 2.0 * g.h[j];
        if (!(val(s.r) < std::max(Hi, Hj))) continue;
        T F[3], Fdotv;
        accel_pair(g, V, rho, C, gamma, i, j, s, visc ? Pi + visc_pair(g, rho, gamma, *visc, i, j, s) : Pi,
                   F, Fdotv);
        for (int cc = 0; cc < 3; ++cc) a[cc] += F[cc];
        if (compat_eps) {
            const T W = -Fdotv;  // (v_j - v_i) . F_ij
            dudt += compat_share(g.u[i], g.u[j], W, *compat_eps) * W;
        } else {
            dudt += Fdotv;
        }
    }
    const T mi = T(g.m[i]);
    for (int cc = 0; cc < 3; ++cc) a[cc] = a[cc] / mi;
    dudt = compat_eps ? dudt / mi : T(-0.5) * dudt / mi;
}

// ---------------------------------------------------------------- gravity
// a_i for j != i with r_ij < r_c over the candidates (all species).
template <class T> void gravity_one(const Gas<T>& g, const T* m, double G, double eps, double r_cut,
                                    const double* poly, int64_t i, Cand c, T a[3]) {
    a[0] = a[1] = a[2] = T(0.0);
    for (int64_t k = 0; k < c.n; ++k) {
        const int64_t j = c.at(k);
        if (j == i) continue;
        Sep<T> s = separation(g, i, j);
        if (!(val(s.r) < r_cut)) continue;
        const T r2 = s.r * s.r;
        T f = T(1.0) / ((r2 + T(eps * eps)) * sqrt(r2 + T(eps * eps)));
        if (poly) {
            T rk = T(1.0);
            for (int p = 0; p < 6; ++p) { f -= T(poly[p]) * rk; rk = rk * r2; }
        }
        for (int cc = 0; cc < 3; ++cc) a[cc] -= T(G) * m[j] * s.d[cc] * f;
    }
}

// ---------------------------------------------------------------- closure
// Everything the forces of a target particle t depend on lies within three
// support radii of t: the forces need corrections of t's neighbours (one hop),
// the corrections need volumes of their neighbours (two hops) and those
// volumes need the positions of their neighbours (three hops).  A brute-force
// scan collects that pool; the chain is then evaluated by brute force inside it.
template <class T> void gather_pool(const Gas<T>& g, int64_t t, double R, std::vector<int64_t>& pool) {
    pool.clear();
    for (int64_t j = 0; j < g.n; ++j) {
        Sep<T> s = separation(g, t, j);
        if (val(s.r) < R) pool.push_back(j);
    }
}

// ---------------------------------------------------------------- gradients
// L = sum_i w_i |a_i|^2 + sum_i c_i du_i/dt with h and m held fixed.  For one
// coordinate theta (a position, velocity or u component of particle p) only
// the particles in theta's dependency cone change:
//   D1: volumes that depend on x_p   = {p} and every k with p inside k's support
//   D2: corrections that depend on D1 or x_p = D1 and every k with a D1 particle inside k's support
//   D3: forces that depend on D1, D2 or p = D1 u D2 and all their force neighbours
// dL/dtheta is evaluated by forward-mode dual numbers over the cone and, as a
// check, by central differences over the same cone; every other particle keeps
// its baseline (brute-force FP64) values.  Neighbour lists are built by brute
// force once (all j with r_ij < max(2h_i, 2h_j)).
struct NbrLists {
    std::vector<int64_t> off, idx;
    Cand of(int64_t i) const { return Cand{idx.data() + off[i], off[i + 1] - off[i]}; }
};

NbrLists brute_force_lists(const Gas<double>& g) {
    const int64_t n = g.n;
    std::vector<std::vector<int64_t>> L(n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            Sep<double> s = separation(g, i, j);
            if (s.r < 2.0 * std::max(g.h[i], g.h[j])) L[i].push_back(j);
        }
    }
    NbrLists out;
    out.off.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) out.off[i + 1] = out.off[i] + (int64_t)L[i].size();
    out.idx.resize(out.off[n]);
    for (int64_t i = 0; i < n; ++i) std::copy(L[i].begin(), L[i].end(), out.idx.begin() + out.off[i]);
    return out;
}

struct Cone {
    std::vector<int64_t> d1, d2, d3;
};

// gather neighbours of k (inside k's own support) are a subset of its force list
Cone dependency_cone(const Gas<double>& g, const NbrLists& nb, int64_t p, int kind) {
    const int64_t n = g.n;
    std::vector<char> in1(n, 0), in2(n, 0), in3(n, 0);
    Cone c;
    auto add = [](std::vector<char>& m, std::vector<int64_t>& v, int64_t k) {
        if (!m[k]) { m[k] = 1; v.push_back(k); }
    };
    if (kind < 3) {
        add(in1, c.d1, p);
        Cand cp = nb.of(p);
        for (int64_t t = 0; t < cp.n; ++t) {
            const int64_t k = cp.at(t);
            if (separation(g, k, p).r < 2.0 * g.h[k]) add(in1, c.d1, k);
        }
        for (int64_t l : c.d1) {
            add(in2, c.d2, l);
            Cand cl = nb.of(l);
            for (int64_t t = 0; t < cl.n; ++t) {
                const int64_t k = cl.at(t);
                if (separation(g, k, l).r < 2.0 * g.h[k]) add(in2, c.d2, k);
            }
        }
        for (int64_t l : c.d2) {
            add(in3, c.d3, l);
            Cand cl = nb.of(l);
            for (int64_t t = 0; t < cl.n; ++t) add(in3, c.d3, cl.at(t));
        }
    } else {
        // velocity or u of p: only the force pass of p and its neighbours
        add(in3, c.d3, p);
        Cand cp = nb.of(p);
        for (int64_t t = 0; t < cp.n; ++t) add(in3, c.d3, cp.at(t));
    }
    return c;
}

// Loss restricted to the cone's force set, with the cone's volumes and
// corrections recomputed from the (possibly perturbed or dual) inputs.
template <class T>
T cone_loss(const Gas<T>& g, const NbrLists& nb, const Cone& c, double gamma, const double* w,
            const double* cw, std::vector<T>& V, std::vector<T>& rho, std::vector<Corr<T>>& C) {
    for (int64_t k : c.d1) {
        T S = volume_sum(g, k, nb.of(k));
        V[k] = T(1.0) / S;
        rho[k] = T(g.m[k]) * S;
    }
    for (int64_t k : c.d2) {
        Moments<T> M;
        moments_one(g, V.data(), k, nb.of(k), M);
        solve_corrections(M, C[k]);
    }
    T L = T(0.0);
    for (int64_t i : c.d3) {
        T a[3], du;
        accel_one(g, V.data(), rho.data(), C.data(), gamma, i, nb.of(i), a, du);
        L += T(w[i]) * (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) + T(cw[i]) * du;
    }
    return L;
}


// ---------------------------------------------------------------- gradient with the viscosity
// L = sum_i w_i |a_i|^2 + sum_i c_i du_i/dt for the chain volume -> corrections
// -> extras (velocity gradients) -> forces with the artificial viscosity
// (h and m held fixed).  Every particle's chain is evaluated (small inputs):
// forward-mode dual numbers for dL/dtheta and central differences as a check.
template <class T>
T visc_chain_loss(const Gas<T>& g, const NbrLists& nb, double gamma, const Visc<double>& qp, const double* w,
                  const double* cw) {
    const int64_t n = g.n;
    std::vector<T> V(n), rho(n), dv(9 * n);
    std::vector<Corr<T>> C(n);
    for (int64_t k = 0; k < n; ++k) {
        const T S = volume_sum(g, k, nb.of(k));
        V[k] = T(1.0) / S;
        rho[k] = T(g.m[k]) * S;
    }
    for (int64_t k = 0; k < n; ++k) {
        Moments<T> M;
        moments_one(g, V.data(), k, nb.of(k), M);
        solve_corrections(M, C[k]);
    }
    for (int64_t k = 0; k < n; ++k) {
        T rhoR, d[3][3], du[3];
        extras_one(g, V.data(), C.data(), k, nb.of(k), rhoR, d, du);
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) dv[9 * k + 3 * a + c] = d[a][c];
    }
    Visc<T> q;
    q.dv = dv.data();
    q.Cl = qp.Cl;
    q.Cq = qp.Cq;
    q.eps_q = qp.eps_q;
    T L = T(0.0);
    for (int64_t i = 0; i < n; ++i) {
        T a[3], du;
        accel_one(g, V.data(), rho.data(), C.data(), gamma, i, nb.of(i), a, du, &q);
        L += T(w[i]) * (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) + T(cw[i]) * du;
    }
    return L;
}


// ---------------------------------------------------------------- operation counts per pair
// The algorithmic work of each pass per ordered pair inside its radius, counted
// on the oracle's own code with the Ops scalar: the pass is evaluated for one
// lane particle with one neighbour and with two neighbours, and the pair work
// of the second minus that of the first is the cost of one more pair (the
// accumulation into the lane's sums included, per-particle work excluded).
//
// The adjoint passes are counted as the reverse-mode derivative of the pair's
// contribution to a loss, with respect to the lane particle's own inputs (the
// gather form: every lane accumulates its own adjoints only):
//   volume adjoint   l = sum_j [Sb_i W(r_ij, h_i) + Sb_j W(r_ij, h_j)],  d/dx_i
//   moments adjoint  l = Mb_i . M_i + sum_j Mb_j . (V_i phi(x_ji, h_j)),  d/dx_i, d/dV_i
//   force adjoint    l = sum_j [F_ij . (ab_i/m_i - ab_j/m_j)
//                               - (db_i/2m_i + db_j/2m_j) F_ij . (v_i - v_j)]
//                    with respect to x_i, v_i, V_i, rho_i, u_i and A_i, B_i, dA_i, dB_i
// where Sb, Mb, ab, db are the upstream adjoints (per-particle inputs), phi the
// 40 moment integrands of the moments pass, and the force adjoint's l is the
// pair's whole share of L = sum_k ab_k . a_k + db_k du_k/dt (F_ji = -F_ij).
namespace flops {

constexpr int kMaxP = 3;  // the lane particle and up to two neighbours

struct Setup {
    int np;
    std::vector<Ops> x, y, z, vx, vy, vz, u, V, rho, m;
    std::vector<double> h, md;
    std::vector<Corr<Ops>> C;
    Gas<Ops> g;
};

Setup make(int nbrs) {
    op_reset();
    const double px[kMaxP] = {0.5, 0.521, 0.482}, py[kMaxP] = {0.5, 0.493, 0.514},
                 pz[kMaxP] = {0.5, 0.507, 0.491};
    Setup s;
    s.np = nbrs + 1;
    for (int p = 0; p < s.np; ++p) {
        const unsigned mk = 1u << p;
        auto L = [&](double v) { return Ops::leaf(v, mk); };
        s.x.push_back(L(px[p])); s.y.push_back(L(py[p])); s.z.push_back(L(pz[p]));
        s.vx.push_back(L(0.01 * (p + 1))); s.vy.push_back(L(-0.02 * p)); s.vz.push_back(L(0.015));
        s.u.push_back(L(1.0 + 0.1 * p));
        s.V.push_back(L(1.0e-3 * (1.0 + 0.05 * p)));
        s.rho.push_back(L(1.0 + 0.02 * p));
        s.m.push_back(L(1.0e-3));
        s.h.push_back(0.05 + 0.002 * p);
        s.md.push_back(1.0e-3);
        Corr<Ops> c;
        c.A = L(1.0 + 0.01 * p);
        for (int a = 0; a < 3; ++a) {
            c.B[a] = L(0.1 * (a + 1));
            c.dA[a] = L(0.2 * (a - 1));
            for (int b = 0; b < 3; ++b) c.dB[a][b] = L(0.05 * (a + 2 * b + 1));
        }
        s.C.push_back(c);
    }
    s.g.n = s.np;
    s.g.x = s.x.data(); s.g.y = s.y.data(); s.g.z = s.z.data();
    s.g.vx = s.vx.data(); s.g.vy = s.vy.data(); s.g.vz = s.vz.data(); s.g.u = s.u.data();
    s.g.h = s.h.data(); s.g.m = s.md.data();
    return s;
}

int64_t volume(int nbrs) {
    Setup s = make(nbrs);
    return pair_flops({volume_sum(s.g, 0, Cand{nullptr, s.np})});
}

int64_t moments(int nbrs) {
    Setup s = make(nbrs);
    Moments<Ops> M;
    moments_one(s.g, s.V.data(), 0, Cand{nullptr, s.np}, M);
    std::vector<Ops> roots{M.m0};
    for (int a = 0; a < 3; ++a) { roots.push_back(M.m1[a]); roots.push_back(M.g0[a]); }
    for (int p = 0; p < 6; ++p) {
        roots.push_back(M.m2[p]);
        for (int c = 0; c < 3; ++c) roots.push_back(M.g2[p][c]);
    }
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) roots.push_back(M.g1[a][c]);
    return pair_flops(roots);
}

int64_t accel(int nbrs) {
    Setup s = make(nbrs);
    Ops a[3], du;
    accel_one(s.g, s.V.data(), s.rho.data(), s.C.data(), 5.0 / 3.0, 0, Cand{nullptr, s.np}, a, du);
    return pair_flops({a[0], a[1], a[2], du});
}

int64_t gravity(int nbrs, bool poly) {
    Setup s = make(nbrs);
    const double p6[6] = {1.0, -2.0, 3.0, 0.5, -0.25, 0.125};
    Ops a[3];
    gravity_one(s.g, s.m.data(), 1.0, 1e-3, 0.2, poly ? p6 : nullptr, 0, Cand{nullptr, s.np}, a);
    return pair_flops({a[0], a[1], a[2]});
}

int64_t volume_adj(int nbrs) {
    Setup s = make(nbrs);
    std::vector<Ops> Sb;
    for (int p = 0; p < s.np; ++p) Sb.push_back(Ops::leaf(0.3 + 0.1 * p, 1u << p));
    Ops l(0.0);
    for (int j = 1; j < s.np; ++j) {
        Sep<Ops> sp = separation(s.g, 0, j);
        l += Sb[0] * kernel_W(sp.r, s.h[0]) + Sb[j] * kernel_W(sp.r, s.h[j]);
    }
    return pair_flops(reverse_sweep(l, {s.x[0], s.y[0], s.z[0]}));
}

std::vector<Ops> moment_list(const Moments<Ops>& M) {
    std::vector<Ops> r{M.m0};
    for (int a = 0; a < 3; ++a) r.push_back(M.m1[a]);
    for (int p = 0; p < 6; ++p) r.push_back(M.m2[p]);
    for (int a = 0; a < 3; ++a) r.push_back(M.g0[a]);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) r.push_back(M.g1[a][c]);
    for (int p = 0; p < 6; ++p)
        for (int c = 0; c < 3; ++c) r.push_back(M.g2[p][c]);
    return r;
}

int64_t moments_adj(int nbrs) {
    Setup s = make(nbrs);
    Ops l(0.0);
    for (int p = 0; p < s.np; ++p) {
        std::vector<Ops> Mb;
        for (int k = 0; k < 40; ++k) Mb.push_back(Ops::leaf(0.01 * (k + 1) + 0.1 * p, 1u << p));
        Moments<Ops> M;
        const int64_t lane = 0;
        if (p == 0) moments_one(s.g, s.V.data(), 0, Cand{nullptr, s.np}, M);
        else moments_one(s.g, s.V.data(), p, Cand{&lane, 1}, M);
        const std::vector<Ops> ml = moment_list(M);
        for (int k = 0; k < 40; ++k) l += Mb[k] * ml[k];
    }
    return pair_flops(reverse_sweep(l, {s.x[0], s.y[0], s.z[0], s.V[0]}));
}

int64_t accel_adj(int nbrs) {
    Setup s = make(nbrs);
    std::vector<std::vector<Ops>> w(s.np);
    std::vector<Ops> kap;
    for (int p = 0; p < s.np; ++p) {
        for (int c = 0; c < 3; ++c) w[p].push_back(Ops::leaf(0.2 * (c + 1) - 0.1 * p, 1u << p));
        kap.push_back(Ops::leaf(0.05 + 0.01 * p, 1u << p));
    }
    const Ops Pi = Ops(5.0 / 3.0 - 1.0) * s.rho[0] * s.u[0];
    Ops l(0.0);
    for (int j = 1; j < s.np; ++j) {
        Sep<Ops> sp = separation(s.g, 0, j);
        Ops F[3], Fv;
        accel_pair(s.g, s.V.data(), s.rho.data(), s.C.data(), 5.0 / 3.0, 0, j, sp, Pi, F, Fv);
        for (int c = 0; c < 3; ++c) l += F[c] * (w[0][c] - w[j][c]);
        l -= (kap[0] + kap[j]) * Fv;
    }
    std::vector<Ops> wanted{s.x[0], s.y[0], s.z[0], s.vx[0], s.vy[0], s.vz[0], s.V[0], s.rho[0], s.u[0],
                            s.C[0].A};
    for (int a = 0; a < 3; ++a) {
        wanted.push_back(s.C[0].B[a]);
        wanted.push_back(s.C[0].dA[a]);
        for (int c = 0; c < 3; ++c) wanted.push_back(s.C[0].dB[a][c]);
    }
    return pair_flops(reverse_sweep(l, wanted));
}

int64_t gravity_adj(int nbrs, bool poly) {
    Setup s = make(nbrs);
    const double p6[6] = {1.0, -2.0, 3.0, 0.5, -0.25, 0.125};
    std::vector<std::vector<Ops>> w(s.np);
    for (int p = 0; p < s.np; ++p)
        for (int c = 0; c < 3; ++c) w[p].push_back(Ops::leaf(0.2 * (c + 1) - 0.1 * p, 1u << p));
    // L = abar_0 . a_0 + sum_j abar_j . (a_j's term from particle 0)
    Ops a0[3];
    gravity_one(s.g, s.m.data(), 1.0, 1e-3, 0.2, poly ? p6 : nullptr, 0, Cand{nullptr, s.np}, a0);
    Ops l = w[0][0] * a0[0] + w[0][1] * a0[1] + w[0][2] * a0[2];
    const int64_t zero = 0;
    for (int j = 1; j < s.np; ++j) {
        Ops aj[3];
        gravity_one(s.g, s.m.data(), 1.0, 1e-3, 0.2, poly ? p6 : nullptr, j, Cand{&zero, 1}, aj);
        l += w[j][0] * aj[0] + w[j][1] * aj[1] + w[j][2] * aj[2];
    }
    return pair_flops(reverse_sweep(l, {s.x[0], s.y[0], s.z[0]}));
}

int64_t extras(int nbrs) {
    Setup s = make(nbrs);
    Ops r, dv[3][3], du[3];
    extras_one(s.g, s.V.data(), s.C.data(), 0, Cand{nullptr, s.np}, r, dv, du);
    std::vector<Ops> roots{r, du[0], du[1], du[2]};
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) roots.push_back(dv[a][c]);
    return pair_flops(roots);
}

int64_t accel_visc(int nbrs) {
    Setup s = make(nbrs);
    std::vector<Ops> dv;
    for (int p = 0; p < s.np; ++p)
        for (int k = 0; k < 9; ++k) dv.push_back(Ops::leaf(0.03 * (k + 1) - 0.02 * p, 1u << p));
    Visc<Ops> q;
    q.dv = dv.data();
    Ops a[3], du;
    accel_one(s.g, s.V.data(), s.rho.data(), s.C.data(), 5.0 / 3.0, 0, Cand{nullptr, s.np}, a, du, &q);
    return pair_flops({a[0], a[1], a[2], du});
}

// the viscous force pair's share of the loss, reversed for particle 0's
// inputs (those of the inviscid form and its velocity gradient)
int64_t accel_visc_adj(int nbrs) {
    Setup s = make(nbrs);
    std::vector<std::vector<Ops>> w(s.np);
    std::vector<Ops> kap, dv;
    for (int p = 0; p < s.np; ++p) {
        for (int c = 0; c < 3; ++c) w[p].push_back(Ops::leaf(0.2 * (c + 1) - 0.1 * p, 1u << p));
        kap.push_back(Ops::leaf(0.05 + 0.01 * p, 1u << p));
        for (int k = 0; k < 9; ++k) dv.push_back(Ops::leaf(0.03 * (k + 1) - 0.02 * p, 1u << p));
    }
    Visc<Ops> q;
    q.dv = dv.data();
    const Ops Pi = Ops(5.0 / 3.0 - 1.0) * s.rho[0] * s.u[0];
    Ops l(0.0);
    for (int j = 1; j < s.np; ++j) {
        Sep<Ops> sp = separation(s.g, 0, j);
        Ops F[3], Fv;
        accel_pair(s.g, s.V.data(), s.rho.data(), s.C.data(), 5.0 / 3.0, 0, j, sp,
                   Pi + visc_pair(s.g, s.rho.data(), 5.0 / 3.0, q, 0, j, sp), F, Fv);
        for (int c = 0; c < 3; ++c) l += F[c] * (w[0][c] - w[j][c]);
        l -= (kap[0] + kap[j]) * Fv;
    }
    std::vector<Ops> wanted{s.x[0], s.y[0], s.z[0], s.vx[0], s.vy[0], s.vz[0], s.V[0], s.rho[0], s.u[0],
                            s.C[0].A};
    for (int a = 0; a < 3; ++a) {
        wanted.push_back(s.C[0].B[a]);
        wanted.push_back(s.C[0].dA[a]);
        for (int c = 0; c < 3; ++c) wanted.push_back(s.C[0].dB[a][c]);
    }
    for (int k = 0; k < 9; ++k) wanted.push_back(dv[k]);
    return pair_flops(reverse_sweep(l, wanted));
}

// l = dvb_0 . dv_0 + sum_j dvb_j . (particle 0's term in dv_j), reversed for
// particle 0's position, velocity, volume and corrections
int64_t extras_adj(int nbrs) {
    Setup s = make(nbrs);
    std::vector<std::vector<Ops>> b(s.np);
    for (int p = 0; p < s.np; ++p)
        for (int k = 0; k < 9; ++k) b[p].push_back(Ops::leaf(0.1 * (k + 1) - 0.07 * p, 1u << p));
    Ops r, dv[3][3], du[3];
    extras_one(s.g, s.V.data(), s.C.data(), 0, Cand{nullptr, s.np}, r, dv, du);
    Ops l(0.0);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) l += b[0][3 * a + c] * dv[a][c];
    const int64_t zero = 0;
    for (int j = 1; j < s.np; ++j) {
        extras_one(s.g, s.V.data(), s.C.data(), j, Cand{&zero, 1}, r, dv, du);
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) l += b[j][3 * a + c] * dv[a][c];
    }
    std::vector<Ops> wanted{s.x[0], s.y[0], s.z[0], s.vx[0], s.vy[0], s.vz[0], s.V[0], s.C[0].A};
    for (int a = 0; a < 3; ++a) {
        wanted.push_back(s.C[0].B[a]);
        wanted.push_back(s.C[0].dA[a]);
        for (int c = 0; c < 3; ++c) wanted.push_back(s.C[0].dB[a][c]);
    }
    return pair_flops(reverse_sweep(l, wanted));
}

int64_t accel_compat(int nbrs) {
    Setup s = make(nbrs);
    Ops a[3], du;
    const double eps_u = 0.1;
    accel_one(s.g, s.V.data(), s.rho.data(), s.C.data(), 5.0 / 3.0, 0, Cand{nullptr, s.np}, a, du,
              static_cast<const Visc<Ops>*>(nullptr), &eps_u);
    return pair_flops({a[0], a[1], a[2], du});
}

}  // namespace flops

}  // namespace

// ====================================================================== C ABI
extern "C" {

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static Gas<double> make_gas(int64_t n, const double* x, const double* y, const double* z,
                            const double* vx, const double* vy, const double* vz,
                            const double* u, const double* h, const double* m) {
    Gas<double> g;
    g.n = n; g.x = x; g.y = y; g.z = z; g.vx = vx; g.vy = vy; g.vz = vz; g.u = u; g.h = h; g.m = m;
    return g;
}

// V_i, rho_i for i in targets (all when targets == NULL); outputs have nt entries.
int oracle_volume(int64_t n, const double* x, const double* y, const double* z, const double* h,
                  const double* m, int64_t nt, const int64_t* targets, double* V, double* rho) {
    Gas<double> g = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, h, m);
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double S = volume_sum(g, i, Cand{nullptr, n});
        V[k] = 1.0 / S;
        rho[k] = m[i] * S;
    }
    return 0;
}

// Raw moments (40 per target, storage order above) and neighbour counts.
int oracle_moments(int64_t n, const double* x, const double* y, const double* z, const double* h,
                   const double* V, int64_t nt, const int64_t* targets, double* M40, int32_t* nnb) {
    Gas<double> g = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, h, nullptr);
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        Moments<double> M;
        moments_one(g, V, i, Cand{nullptr, n}, M);
        double* o = M40 + 40 * k;
        o[0] = M.m0;
        for (int a = 0; a < 3; ++a) o[1 + a] = M.m1[a];
        for (int p = 0; p < 6; ++p) o[4 + p] = M.m2[p];
        for (int a = 0; a < 3; ++a) o[10 + a] = M.g0[a];
        for (int a = 0; a < 3; ++a) for (int c = 0; c < 3; ++c) o[13 + 3 * a + c] = M.g1[a][c];
        for (int p = 0; p < 6; ++p) for (int c = 0; c < 3; ++c) o[22 + 3 * p + c] = M.g2[p][c];
        if (nnb) nnb[k] = M.nnb;
    }
    return 0;
}

// A (nt), B (3 nt), dA (3 nt), dB (9 nt); returns the number of fallbacks.
int64_t oracle_corrections(int64_t n, const double* x, const double* y, const double* z,
                           const double* h, const double* V, int64_t nt, const int64_t* targets,
                           double* A, double* B, double* dA, double* dB) {
    Gas<double> g = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, h, nullptr);
    const int64_t cnt = targets ? nt : n;
    int64_t fallbacks = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : fallbacks)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        Moments<double> M;
        moments_one(g, V, i, Cand{nullptr, n}, M);
        Corr<double> C;
        fallbacks += solve_corrections(M, C);
        A[k] = C.A;
        for (int a = 0; a < 3; ++a) {
            B[3 * k + a] = C.B[a];
            dA[3 * k + a] = C.dA[a];
            for (int c = 0; c < 3; ++c) dB[9 * k + 3 * a + c] = C.dB[a][c];
        }
    }
    return fallbacks;
}

// Accelerations and du/dt for targets; V, rho and corrections for ALL particles.
int oracle_accel(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                 const double* vy, const double* vz, const double* u, const double* h,
                 const double* m, const double* V, const double* rho, const double* A,
                 const double* B, const double* dA, const double* dB, double gamma, int64_t nt,
                 const int64_t* targets, double* ax, double* ay, double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double a[3], du;
        accel_one(g, V, rho, C.data(), gamma, i, Cand{nullptr, n}, a, du);
        ax[k] = a[0]; ay[k] = a[1]; az[k] = a[2]; dudt[k] = du;
    }
    return 0;
}

// CRK density and velocity / energy gradients for targets (all when NULL).
int oracle_extras(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                  const double* vy, const double* vz, const double* u, const double* h,
                  const double* m, const double* V, const double* A, const double* B,
                  const double* dA, const double* dB, int64_t nt, const int64_t* targets,
                  double* rhoR, double* dv, double* du) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double r, v[3][3], e[3];
        extras_one(g, V, C.data(), i, Cand{nullptr, n}, r, v, e);
        rhoR[k] = r;
        for (int a = 0; a < 3; ++a) {
            du[3 * k + a] = e[a];
            for (int c = 0; c < 3; ++c) dv[9 * k + 3 * a + c] = v[a][c];
        }
    }
    return 0;
}

// Forces with the artificial viscosity (dv: the velocity gradients, 9 per particle).
int oracle_accel_visc(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                      const double* vy, const double* vz, const double* u, const double* h,
                      const double* m, const double* V, const double* rho, const double* A,
                      const double* B, const double* dA, const double* dB, const double* dv,
                      double Cl, double Cq, double eps_q, double gamma, int64_t nt,
                      const int64_t* targets, double* ax, double* ay, double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
    Visc<double> q;
    q.dv = dv;
    q.Cl = Cl;
    q.Cq = Cq;
    q.eps_q = eps_q;
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double a[3], du;
        accel_one(g, V, rho, C.data(), gamma, i, Cand{nullptr, n}, a, du, &q);
        ax[k] = a[0]; ay[k] = a[1]; az[k] = a[2]; dudt[k] = du;
    }
    return 0;
}

// Forces with the compatible energy partition (dv NULL: no viscosity).
int oracle_accel_compat(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                        const double* vy, const double* vz, const double* u, const double* h,
                        const double* m, const double* V, const double* rho, const double* A,
                        const double* B, const double* dA, const double* dB, const double* dv,
                        double Cl, double Cq, double eps_q, double eps_u, double gamma, int64_t nt,
                        const int64_t* targets, double* ax, double* ay, double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
    Visc<double> q;
    q.dv = dv;
    q.Cl = Cl;
    q.Cq = Cq;
    q.eps_q = eps_q;
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double a[3], du;
        accel_one(g, V, rho, C.data(), gamma, i, Cand{nullptr, n}, a, du, dv ? &q : static_cast<Visc<double>*>(nullptr),
                  &eps_u);
        ax[k] = a[0]; ay[k] = a[1]; az[k] = a[2]; dudt[k] = du;
    }
    return 0;
}

// Momentum and energy totals over all particles:
// [sum m a_x, sum m a_y, sum m a_z, sum m (v.a + du/dt), sum m |a|,
//  sum m (|v.a| + |du/dt|), sum m du/dt, sum m v.a]
int oracle_totals(int64_t n, const double* m, const double* vx, const double* vy, const double* vz,
                  const double* ax, const double* ay, const double* az, const double* dudt,
                  double* totals) {
    for (int k = 0; k < 8; ++k) totals[k] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double va = vx[i] * ax[i] + vy[i] * ay[i] + vz[i] * az[i];
        totals[0] += m[i] * ax[i];
        totals[1] += m[i] * ay[i];
        totals[2] += m[i] * az[i];
        totals[3] += m[i] * (va + dudt[i]);
        totals[4] += m[i] * std::sqrt(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
        totals[5] += m[i] * (std::fabs(va) + std::fabs(dudt[i]));
        totals[6] += m[i] * dudt[i];
        totals[7] += m[i] * va;
    }
    return 0;
}

// Full chain V -> corrections -> forces for target particles, each evaluated
// by brute force inside its own three-hop pool (see Closure above).  Outputs
// per target: V, rho, A, B[3], dA[3], dB[9], a[3], du/dt.
int64_t oracle_hydro_targets(int64_t n, const double* x, const double* y, const double* z,
                             const double* vx, const double* vy, const double* vz, const double* u,
                             const double* h, const double* m, double gamma, int64_t nt,
                             const int64_t* targets, double* V_o, double* rho_o, double* A_o,
                             double* B_o, double* dA_o, double* dB_o, double* ax, double* ay,
                             double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    double Hmax = 0.0;
    for (int64_t i = 0; i < n; ++i) Hmax = std::max(Hmax, 2.0 * h[i]);
    const double R = 3.0 * Hmax * (1.0 + 1e-12);
    int64_t fallbacks = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fallbacks)
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t t = targets[k];
        std::vector<int64_t> pool;
        gather_pool(g, t, R, pool);
        const int64_t np = (int64_t)pool.size();
        // local copy of the pool's particles (pool-local indices)
        std::vector<double> lx(np), ly(np), lz(np), lvx(np), lvy(np), lvz(np), lu(np), lh(np), lm(np);
        int64_t lt = -1;
        for (int64_t p = 0; p < np; ++p) {
            const int64_t j = pool[p];
            lx[p] = x[j]; ly[p] = y[j]; lz[p] = z[j]; lvx[p] = vx[j]; lvy[p] = vy[j]; lvz[p] = vz[j];
            lu[p] = u[j]; lh[p] = h[j]; lm[p] = m[j];
            if (j == t) lt = p;
        }
        Gas<double> lg = make_gas(np, lx.data(), ly.data(), lz.data(), lvx.data(), lvy.data(),
                                  lvz.data(), lu.data(), lh.data(), lm.data());
        const Cand all{nullptr, np};
        // S1: the target and its force neighbours; S2: S1 and their gather neighbours
        std::vector<char> in1(np, 0), in2(np, 0);
        in1[lt] = 1;
        for (int64_t p = 0; p < np; ++p) {
            if (p == lt) continue;
            Sep<double> s = separation(lg, lt, p);
            if (s.r < std::max(2.0 * lh[lt], 2.0 * lh[p])) in1[p] = 1;
        }
        for (int64_t p = 0; p < np; ++p) {
            if (!in1[p]) continue;
            in2[p] = 1;
            for (int64_t q = 0; q < np; ++q) {
                Sep<double> s = separation(lg, p, q);
                if (s.r < 2.0 * lh[p]) in2[q] = 1;
            }
        }
        std::vector<double> lV(np, 0.0), lrho(np, 0.0);
        for (int64_t p = 0; p < np; ++p) {
            if (!in2[p]) continue;
            double S = volume_sum(lg, p, all);
            lV[p] = 1.0 / S;
            lrho[p] = lm[p] * S;
        }
        std::vector<Corr<double>> lC(np);
        for (int64_t p = 0; p < np; ++p) {
            if (!in1[p]) continue;
            Moments<double> M;
            moments_one(lg, lV.data(), p, all, M);
            int fb = solve_corrections(M, lC[p]);
            if (p == lt) fallbacks += fb;
        }
        double a[3], du;
        accel_one(lg, lV.data(), lrho.data(), lC.data(), gamma, lt, all, a, du);
        V_o[k] = lV[lt];
        rho_o[k] = lrho[lt];
        const Corr<double>& C = lC[lt];
        A_o[k] = C.A;
        for (int q = 0; q < 3; ++q) {
            B_o[3 * k + q] = C.B[q];
            dA_o[3 * k + q] = C.dA[q];
            for (int c = 0; c < 3; ++c) dB_o[9 * k + 3 * q + c] = C.dB[q][c];
        }
        ax[k] = a[0]; ay[k] = a[1]; az[k] = a[2]; dudt[k] = du;
    }
    return fallbacks;
}

// Short-range gravity for targets (all when targets == NULL).  poly may be NULL.
int oracle_gravity(int64_t n, const double* x, const double* y, const double* z, const double* m,
                   double G, double eps, double r_cut, const double* poly, int64_t nt,
                   const int64_t* targets, double* ax, double* ay, double* az) {
    Gas<double> g = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, nullptr, m);
    const int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        double a[3];
        gravity_one(g, m, G, eps, r_cut, poly, i, Cand{nullptr, n}, a);
        ax[k] = a[0]; ay[k] = a[1]; az[k] = a[2];
    }
    return 0;
}

// Ordered-pair interaction counts (j != i) for targets (all when NULL):
// mode 0: r < 2 h_i (volume, moments); 1: r < 2 max(h_i, h_j) (forces);
// 2: r < r_fixed (gravity; h unused).
int64_t oracle_count_pairs(int64_t n, const double* x, const double* y, const double* z,
                           const double* h, int mode, double r_fixed, int64_t nt,
                           const int64_t* targets, int32_t* per_target) {
    Gas<double> g = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, h, nullptr);
    const int64_t cnt = targets ? nt : n;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t k = 0; k < cnt; ++k) {
        const int64_t i = targets ? targets[k] : k;
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            Sep<double> s = separation(g, i, j);
            double R = mode == 0 ? 2.0 * h[i] : mode == 1 ? 2.0 * std::max(h[i], h[j]) : r_fixed;
            if (s.r < R) ++c;
        }
        if (per_target) per_target[k] = c;
        total += c;
    }
    return total;
}


// FLOP per ordered pair inside the pass radius, counted on the oracle's code
// (see the flops namespace): [volume, moments, accel, gravity, gravity with the
// polynomial term, volume adjoint, moments adjoint, force adjoint, extras, force
// pass with the viscosity, gravity adjoint, gravity adjoint with the polynomial,
// force pass with the compatible energy partition, viscous force adjoint, Extras
// adjoint].
void oracle_flops(double* out) {
    using namespace flops;
    out[0] = double(volume(2) - volume(1));
    out[1] = double(moments(2) - moments(1));
    out[2] = double(accel(2) - accel(1));
    out[3] = double(gravity(2, false) - gravity(1, false));
    out[4] = double(gravity(2, true) - gravity(1, true));
    out[5] = double(volume_adj(2) - volume_adj(1));
    out[6] = double(moments_adj(2) - moments_adj(1));
    out[7] = double(accel_adj(2) - accel_adj(1));
    out[8] = double(extras(2) - extras(1));
    out[9] = double(accel_visc(2) - accel_visc(1));
    out[10] = double(gravity_adj(2, false) - gravity_adj(1, false));
    out[11] = double(gravity_adj(2, true) - gravity_adj(1, true));
    out[12] = double(accel_compat(2) - accel_compat(1));
    out[13] = double(accel_visc_adj(2) - accel_visc_adj(1));
    out[14] = double(extras_adj(2) - extras_adj(1));
    op_reset();
}

// Counts of small expressions, which pin the counting rules (a, c depend on the
// lane particle, b and e on a neighbour):
//   [0] a*b + c   [1] (a*c)*b   [2] (a-b)*(a-b) + (a-b)*(a-b)   [3] {(a-b)^2, (b-a)^2}
//   [4] d/da of (a*b)*(a*b)   [5] sqrt(a*b)/c   [6] d/da of sqrt(a - b)   [7] e*b
void oracle_flops_selftest(double* out) {
    auto run = [](int k) -> int64_t {
        op_reset();
        const Ops a = Ops::leaf(1.5, 1u), c = Ops::leaf(0.7, 1u), b = Ops::leaf(0.25, 2u),
                  e = Ops::leaf(2.0, 2u);
        switch (k) {
            case 0: return pair_flops({a * b + c});
            case 1: return pair_flops({(a * c) * b});
            case 2: { const Ops d = a - b; return pair_flops({d * d + d * d}); }
            case 3: { const Ops d = a - b, f = b - a; return pair_flops({d * d, f * f}); }
            case 4: { const Ops t = a * b; return pair_flops(reverse_sweep(t * t, {a})); }
            case 5: return pair_flops({sqrt(a * b) / c});
            case 6: return pair_flops(reverse_sweep(sqrt(a - b), {a}));
            case 7: return pair_flops({e * b});
        }
        return -1;
    };
    for (int k = 0; k < 8; ++k) out[k] = double(run(k));
    op_reset();
}


// The three hydro passes for target particles over precomputed candidate
// lists (CSR: the candidates of targets[k] are idx[off[k] .. off[k+1])), for
// timing the oracle's arithmetic without its brute-force search.  Each pass
// still tests its own radius on every candidate.  V, rho and the corrections
// of all n particles are inputs (the volume and corrections outputs of the
// targets are written to V_o, A_o, ax, dudt).  Returns the number of in-radius
// ordered pairs of the volume and moments passes (2 x those with r < 2h_i);
// the force pass evaluates the pairs with r < 2 max(h_i, h_j) among the
// candidates (all of them when the lists hold exactly those).
int64_t oracle_passes_listed(int64_t n, const double* x, const double* y, const double* z,
                             const double* vx, const double* vy, const double* vz, const double* u,
                             const double* h, const double* m, double gamma, const double* V,
                             const double* rho, const double* A, const double* B, const double* dA,
                             const double* dB, int64_t nt, const int64_t* targets, const int64_t* off,
                             const int64_t* idx, int threads, double* V_o, double* A_o, double* ax,
                             double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
    int64_t pairs = 0;
#ifdef _OPENMP
    const int nth = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pairs) num_threads(nth)
#endif
    for (int64_t k = 0; k < nt; ++k) {
        const int64_t i = targets[k];
        const Cand c{idx + off[k], off[k + 1] - off[k]};
        V_o[k] = 1.0 / volume_sum(g, i, c);
        Moments<double> M;
        moments_one(g, V, i, c, M);
        Corr<double> Ci;
        solve_corrections(M, Ci);
        A_o[k] = Ci.A;
        double a[3], du;
        accel_one(g, V, rho, C.data(), gamma, i, c, a, du);
        ax[k] = a[0];
        dudt[k] = du;
        pairs += 2 * int64_t(M.nnb);
    }
    return pairs;
}


// Short-range gravity of target particles over precomputed candidate lists
// (CSR as in oracle_passes_listed), for timing the oracle's arithmetic
// without its brute-force search; the cutoff is still tested per candidate.
int oracle_gravity_listed(int64_t n, const double* x, const double* y, const double* z, const double* m,
                          double G, double eps, double r_cut, const double* poly, int64_t nt,
                          const int64_t* targets, const int64_t* off, const int64_t* idx, int threads,
                          double* ax, double* ay, double* az) {
    Gas<double> g = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, nullptr, m);
#ifdef _OPENMP
    const int nth = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
#endif
    for (int64_t k = 0; k < nt; ++k) {
        double a[3];
        gravity_one(g, m, G, eps, r_cut, poly, targets[k], Cand{idx + off[k], off[k + 1] - off[k]}, a);
        ax[k] = a[0]; ay[k] = a[1]; az[k] = a[2];
    }
    return 0;
}


// The full forward chain (volumes, corrections, forces, totals) of all n
// particles with the candidates of particle i taken from a precomputed list
// (CSR: idx[off[i] .. off[i+1])) instead of a scan of every particle.  Each
// pass still tests its own radius on every candidate, so with lists that hold
// every j within max(2h_i, 2h_j) in increasing index order the result is the
// brute-force chain's bit for bit (the same terms summed in the same order).
// Outputs as oracle_hydro_targets for all particles; returns the fallbacks.
int64_t oracle_hydro_listed(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                            const double* vy, const double* vz, const double* u, const double* h,
                            const double* m, double gamma, const int64_t* off, const int64_t* idx,
                            double* V_o, double* rho_o, double* A_o, double* B_o, double* dA_o,
                            double* dB_o, double* ax, double* ay, double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    auto cand = [&](int64_t i) { return Cand{idx + off[i], off[i + 1] - off[i]}; };
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const double S = volume_sum(g, i, cand(i));
        V_o[i] = 1.0 / S;
        rho_o[i] = m[i] * S;
    }
    std::vector<Corr<double>> C(n);
    int64_t fallbacks = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : fallbacks)
    for (int64_t i = 0; i < n; ++i) {
        Moments<double> M;
        moments_one(g, V_o, i, cand(i), M);
        fallbacks += solve_corrections(M, C[i]);
        A_o[i] = C[i].A;
        for (int a = 0; a < 3; ++a) {
            B_o[3 * i + a] = C[i].B[a];
            dA_o[3 * i + a] = C[i].dA[a];
            for (int c = 0; c < 3; ++c) dB_o[9 * i + 3 * a + c] = C[i].dB[a][c];
        }
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double a[3], du;
        accel_one(g, V_o, rho_o, C.data(), gamma, i, cand(i), a, du);
        ax[i] = a[0]; ay[i] = a[1]; az[i] = a[2]; dudt[i] = du;
    }
    return fallbacks;
}

// Extras of all particles, then their forces with the artificial viscosity,
// over precomputed candidate lists (V, rho and the corrections given).
int oracle_visc_listed(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                       const double* vy, const double* vz, const double* u, const double* h,
                       const double* m, double gamma, double Cl, double Cq, double eps_q, const int64_t* off,
                       const int64_t* idx, const double* V, const double* rho, const double* A,
                       const double* B, const double* dA, const double* dB, double* rhoR_o, double* dv_o,
                       double* du_o, double* ax, double* ay, double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    auto cand = [&](int64_t i) { return Cand{idx + off[i], off[i + 1] - off[i]}; };
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double r, v[3][3], e[3];
        extras_one(g, V, C.data(), i, cand(i), r, v, e);
        rhoR_o[i] = r;
        for (int a = 0; a < 3; ++a) {
            du_o[3 * i + a] = e[a];
            for (int c = 0; c < 3; ++c) dv_o[9 * i + 3 * a + c] = v[a][c];
        }
    }
    Visc<double> q;
    q.dv = dv_o;
    q.Cl = Cl;
    q.Cq = Cq;
    q.eps_q = eps_q;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double a[3], du;
        accel_one(g, V, rho, C.data(), gamma, i, cand(i), a, du, &q);
        ax[i] = a[0]; ay[i] = a[1]; az[i] = a[2]; dudt[i] = du;
    }
    return 0;
}

// Forces with the compatible energy partition (no viscosity) of all particles
// over precomputed lists, from the oracle's own V, rho and corrections.  With
// exact lists it equals oracle_accel_compat bit for bit.
int oracle_compat_listed(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                         const double* vy, const double* vz, const double* u, const double* h, const double* m,
                         double gamma, double eps_u, const int64_t* off, const int64_t* idx, const double* V,
                         const double* rho, const double* A, const double* B, const double* dA, const double* dB,
                         double* ax, double* ay, double* az, double* dudt) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    auto cand = [&](int64_t i) { return Cand{idx + off[i], off[i + 1] - off[i]}; };
    std::vector<Corr<double>> C(n);
    for (int64_t i = 0; i < n; ++i) {
        C[i].A = A[i];
        for (int a = 0; a < 3; ++a) {
            C[i].B[a] = B[3 * i + a];
            C[i].dA[a] = dA[3 * i + a];
            for (int c = 0; c < 3; ++c) C[i].dB[a][c] = dB[9 * i + 3 * a + c];
        }
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double a[3], du;
        accel_one(g, V, rho, C.data(), gamma, i, cand(i), a, du, static_cast<Visc<double>*>(nullptr), &eps_u);
        ax[i] = a[0]; ay[i] = a[1]; az[i] = a[2]; dudt[i] = du;
    }
    return 0;
}

// Kernel values for pinning: W(r, h) and F(r, h) at n radii.
void oracle_kernel(int64_t n, const double* r, double h, double* W, double* F) {
    for (int64_t k = 0; k < n; ++k) {
        W[k] = kernel_W(r[k], h);
        F[k] = kernel_F(r[k], h);
    }
}


// dL/dtheta for ncoord coordinates: kind 0-2 = x, y, z; 3-5 = vx, vy, vz; 6 = u
// of particle part[k].  g_dual: forward-mode dual numbers; g_fd: central
// differences with step fd_step (absolute; positions in box units, velocities
// as given, u relative: fd_step * u_p).
int oracle_grad(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                const double* vy, const double* vz, const double* u, const double* h,
                const double* m, double gamma, const double* w, const double* cw, int64_t ncoord,
                const int64_t* part, const int32_t* kind, double fd_step, double* g_dual,
                double* g_fd, int64_t* cone_sizes) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    const NbrLists nb = brute_force_lists(g);
    // baseline values over all particles (brute force through the exact lists)
    std::vector<double> V0(n), rho0(n);
    std::vector<Corr<double>> C0(n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double S = volume_sum(g, i, nb.of(i));
        V0[i] = 1.0 / S;
        rho0[i] = m[i] * S;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        Moments<double> M;
        moments_one(g, V0.data(), i, nb.of(i), M);
        solve_corrections(M, C0[i]);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ncoord; ++k) {
        const int64_t p = part[k];
        const int kd = kind[k];
        const Cone cone = dependency_cone(g, nb, p, kd);
        cone_sizes[3 * k + 0] = (int64_t)cone.d1.size();
        cone_sizes[3 * k + 1] = (int64_t)cone.d2.size();
        cone_sizes[3 * k + 2] = (int64_t)cone.d3.size();
        // dual numbers: every input as a constant except theta
        {
            std::vector<Dual> f[7];
            const double* src[7] = {x, y, z, vx, vy, vz, u};
            for (int a = 0; a < 7; ++a) {
                f[a].resize(n);
                for (int64_t i = 0; i < n; ++i) f[a][i] = Dual(src[a][i], 0.0);
            }
            f[kd][p].d = 1.0;
            Gas<Dual> gd;
            gd.n = n; gd.x = f[0].data(); gd.y = f[1].data(); gd.z = f[2].data();
            gd.vx = f[3].data(); gd.vy = f[4].data(); gd.vz = f[5].data(); gd.u = f[6].data();
            gd.h = h; gd.m = m;
            std::vector<Dual> V(n), rho(n);
            std::vector<Corr<Dual>> C(n);
            for (int64_t i = 0; i < n; ++i) { V[i] = Dual(V0[i]); rho[i] = Dual(rho0[i]); }
            for (int64_t i : cone.d3) {
                C[i].A = Dual(C0[i].A);
                for (int a = 0; a < 3; ++a) {
                    C[i].B[a] = Dual(C0[i].B[a]);
                    C[i].dA[a] = Dual(C0[i].dA[a]);
                    for (int c = 0; c < 3; ++c) C[i].dB[a][c] = Dual(C0[i].dB[a][c]);
                }
                for (int64_t t = nb.off[i]; t < nb.off[i + 1]; ++t) {
                    const int64_t j = nb.idx[t];
                    C[j].A = Dual(C0[j].A);
                    for (int a = 0; a < 3; ++a) {
                        C[j].B[a] = Dual(C0[j].B[a]);
                        C[j].dA[a] = Dual(C0[j].dA[a]);
                        for (int c = 0; c < 3; ++c) C[j].dB[a][c] = Dual(C0[j].dB[a][c]);
                    }
                }
            }
            g_dual[k] = cone_loss(gd, nb, cone, gamma, w, cw, V, rho, C).d;
        }
        // central differences over the same cone
        {
            std::vector<double> f[7];
            const double* src[7] = {x, y, z, vx, vy, vz, u};
            for (int a = 0; a < 7; ++a) f[a].assign(src[a], src[a] + n);
            const double step = kd == 6 ? fd_step * u[p] : fd_step;
            double Lpm[2];
            for (int sgn = 0; sgn < 2; ++sgn) {
                f[kd][p] = src[kd][p] + (sgn == 0 ? step : -step);
                Gas<double> gp = make_gas(n, f[0].data(), f[1].data(), f[2].data(), f[3].data(),
                                          f[4].data(), f[5].data(), f[6].data(), h, m);
                std::vector<double> V(V0), rho(rho0);
                std::vector<Corr<double>> C(C0);
                Lpm[sgn] = cone_loss(gp, nb, cone, gamma, w, cw, V, rho, C);
            }
            g_fd[k] = (Lpm[0] - Lpm[1]) / (2.0 * step);
        }
    }
    return 0;
}

// ---------------------------------------------------------------- PM-filtered split
// F(x) = erf(x) - (2x/sqrt(pi)) exp(-x^2) = (4/sqrt(pi)) int_0^x t^2 exp(-t^2) dt:
// the series of the integral for small x (where the closed form cancels), the
// closed form beyond.
static double split_F(double x) {
    if (x < 0.5) {
        double term = x * x * x, sum = 0.0, fact = 1.0;
        for (int k = 0; k < 30; ++k) {
            if (k > 0) fact *= double(k);
            const double t = (k % 2 ? -1.0 : 1.0) * term / (fact * double(2 * k + 3));
            sum += t;
            term *= x * x;
            if (std::fabs(t) < 1e-18 * std::fabs(sum)) break;
        }
        return 4.0 / std::sqrt(kPi) * sum;
    }
    return std::erf(x) - 2.0 * x / std::sqrt(kPi) * std::exp(-x * x);
}

// Long-range force per unit mass at separations r (r > 0), filter scale r_s.
void oracle_long_range_force(int64_t n, const double* r, double r_s, double* f) {
    for (int64_t k = 0; k < n; ++k) f[k] = split_F(r[k] / (2.0 * r_s)) / (r[k] * r[k]);
}

// dL/dtheta of the viscous chain (visc_chain_loss) at ncoord coordinates kind
// 0-6 (x, y, z, vx, vy, vz, u) of particle part[k]: dual numbers (g_dual) and
// central differences (g_fd; step fd_step, relative for u).
int oracle_grad_visc(int64_t n, const double* x, const double* y, const double* z, const double* vx,
                     const double* vy, const double* vz, const double* u, const double* h, const double* m,
                     double gamma, double Cl, double Cq, double eps_q, const double* w, const double* cw,
                     int64_t ncoord, const int64_t* part, const int32_t* kind, double fd_step, double* g_dual,
                     double* g_fd) {
    Gas<double> g = make_gas(n, x, y, z, vx, vy, vz, u, h, m);
    const NbrLists nb = brute_force_lists(g);
    Visc<double> qp;
    qp.Cl = Cl;
    qp.Cq = Cq;
    qp.eps_q = eps_q;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ncoord; ++k) {
        const int64_t p = part[k];
        const int kd = kind[k];
        {
            std::vector<Dual> f[7];
            const double* src[7] = {x, y, z, vx, vy, vz, u};
            for (int a = 0; a < 7; ++a) {
                f[a].resize(n);
                for (int64_t i = 0; i < n; ++i) f[a][i] = Dual(src[a][i], 0.0);
            }
            f[kd][p].d = 1.0;
            Gas<Dual> gd;
            gd.n = n; gd.x = f[0].data(); gd.y = f[1].data(); gd.z = f[2].data();
            gd.vx = f[3].data(); gd.vy = f[4].data(); gd.vz = f[5].data(); gd.u = f[6].data();
            gd.h = h; gd.m = m;
            g_dual[k] = visc_chain_loss(gd, nb, gamma, qp, w, cw).d;
        }
        {
            std::vector<double> f[7];
            const double* src[7] = {x, y, z, vx, vy, vz, u};
            for (int a = 0; a < 7; ++a) f[a].assign(src[a], src[a] + n);
            const double step = kd == 6 ? fd_step * u[p] : fd_step;
            double Lpm[2];
            for (int sgn = 0; sgn < 2; ++sgn) {
                f[kd][p] = src[kd][p] + (sgn == 0 ? step : -step);
                Gas<double> gp = make_gas(n, f[0].data(), f[1].data(), f[2].data(), f[3].data(),
                                          f[4].data(), f[5].data(), f[6].data(), h, m);
                Lpm[sgn] = visc_chain_loss(gp, nb, gamma, qp, w, cw);
            }
            g_fd[k] = (Lpm[0] - Lpm[1]) / (2.0 * step);
        }
    }
    return 0;
}

// dL/dx for L = sum_i abar_i . a_i, a the short-range gravity of every
// particle (masses fixed), at ncoord coordinates kind 0-2 (x, y, z) of
// particle part[k].  A coordinate of p changes a_p and the a_j of every j
// within r_c of p; only those enter.  g_dual: forward-mode dual numbers;
// g_fd: central differences with absolute step fd_step.
int oracle_gravity_grad(int64_t n, const double* x, const double* y, const double* z, const double* m,
                        double G, double eps, double r_cut, const double* poly, const double* abar,
                        int64_t ncoord, const int64_t* part, const int32_t* kind, double fd_step,
                        double* g_dual, double* g_fd) {
    Gas<double> g0 = make_gas(n, x, y, z, nullptr, nullptr, nullptr, nullptr, nullptr, m);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ncoord; ++k) {
        const int64_t p = part[k];
        const int kd = kind[k];
        std::vector<int64_t> affected{p};
        for (int64_t j = 0; j < n; ++j)
            if (j != p && separation(g0, p, j).r < r_cut) affected.push_back(j);
        {
            std::vector<Dual> f[3], md(n);
            const double* src[3] = {x, y, z};
            for (int a = 0; a < 3; ++a) {
                f[a].resize(n);
                for (int64_t i = 0; i < n; ++i) f[a][i] = Dual(src[a][i], 0.0);
            }
            for (int64_t i = 0; i < n; ++i) md[i] = Dual(m[i], 0.0);
            f[kd][p].d = 1.0;
            Gas<Dual> gd;
            gd.n = n; gd.x = f[0].data(); gd.y = f[1].data(); gd.z = f[2].data();
            gd.vx = gd.vy = gd.vz = gd.u = nullptr; gd.h = nullptr; gd.m = m;
            Dual L(0.0);
            for (int64_t i : affected) {
                Dual a[3];
                gravity_one(gd, md.data(), G, eps, r_cut, poly, i, Cand{nullptr, n}, a);
                for (int c = 0; c < 3; ++c) L += Dual(abar[3 * i + c]) * a[c];
            }
            g_dual[k] = L.d;
        }
        {
            std::vector<double> f[3];
            const double* src[3] = {x, y, z};
            for (int a = 0; a < 3; ++a) f[a].assign(src[a], src[a] + n);
            double Lpm[2];
            for (int sgn = 0; sgn < 2; ++sgn) {
                f[kd][p] = src[kd][p] + (sgn == 0 ? fd_step : -fd_step);
                Gas<double> gp = make_gas(n, f[0].data(), f[1].data(), f[2].data(), nullptr, nullptr, nullptr,
                                          nullptr, nullptr, m);
                double L = 0.0;
                for (int64_t i : affected) {
                    double a[3];
                    gravity_one(gp, m, G, eps, r_cut, poly, i, Cand{nullptr, n}, a);
                    for (int c = 0; c < 3; ++c) L += abar[3 * i + c] * a[c];
                }
                Lpm[sgn] = L;
            }
            g_fd[k] = (Lpm[0] - Lpm[1]) / (2.0 * fd_step);
        }
    }
    return 0;
}

}  // extern "C"

