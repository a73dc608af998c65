// Compile-time sizes and the constant tables shared by host and device code.
//
// Sizes per polynomial degree N (Section 2, eq. modalForm2D: Np =
// (N+1)(N+2)/2).  Volume rule: collapsed Gauss-Legendre x Gauss-Jacobi(1,0)
// with ceil(3N/2) points per direction (exact to degree 3N-1, enough for
// grad(psi) . u^2/2).  Edge rule: Gauss-Legendre with ceil((3N+1)/2) points
// (exact to degree 3N).  Projection rule for initial data: N+4 points per
// direction (exact to degree 2N+7).
#pragma once

namespace cswdg {

template <int N>
struct Dims {
    static constexpr int NP = (N + 1) * (N + 2) / 2;
    static constexpr int NV1 = (3 * N + 1) / 2;
    static constexpr int NQ = NV1 * NV1;
    static constexpr int NE = (3 * N + 2) / 2;
    static constexpr int NI1 = N + 4;
    static constexpr int NQI = NI1 * NI1;
    // limiter: degree of the top least-squares polynomial (quadratic for
    // N = 1, quartic for N = 2, 3), number of scaled monomials of degree
    // 1..DTOP, pieces per neighbour
    static constexpr int DTOP = (N == 1) ? 2 : 4;
    static constexpr int NMONO = (DTOP == 2) ? 5 : 14;
    static constexpr int NPIECE = (N == 1) ? 3 : 7;
    static constexpr int NTOPROWS = (N == 1) ? 9 : 15;
    static constexpr int NBP = NMONO * (NMONO + 1) / 2;
};

// Per-degree device tables (constant memory).
template <int N>
struct Tab {
    using D = Dims<N>;
    double V[D::NQ][D::NP];      // psi_n at volume points
    double wDr[D::NQ][D::NP];    // w_q dpsi_n/dr
    double wDs[D::NQ][D::NP];    // w_q dpsi_n/ds
    double PF[3][D::NE][D::NP];  // psi_n at the points of face f
    double wPF[3][D::NE][D::NP]; // w_g psi_n at the points of face f
    double we[D::NE];            // edge weights (sum 2)
    double es[D::NE];            // position of edge point g along its face, in (0, 1) from vertex f to f+1
    double wmean[D::NP];         // mean of psi_n over the reference triangle
    double PMID[3][D::NP];       // psi_n at the midpoint of face f
};

// The residual's tables in single precision (FP32-bulk mode).
template <int N>
struct TabF {
    using D = Dims<N>;
    float V[D::NQ][D::NP];
    float wDr[D::NQ][D::NP];
    float wDs[D::NQ][D::NP];
    float PF[3][D::NE][D::NP];
    float wPF[3][D::NE][D::NP];
};

// Layout of the per-element limiter operator record (doubles).
template <int N>
struct OpLayout {
    using D = Dims<N>;
    static constexpr int AVG = 0;                                  // [3][NPIECE][NP] subcell-average functionals
    static constexpr int X2 = AVG + 3 * D::NPIECE * D::NP;         // [2][3]   pinv, linear level
    static constexpr int X3 = X2 + 2 * 3;                          // [5][9]   pinv, quadratic level
    static constexpr int X5 = X3 + 5 * 9;                          // [14][15] pinv, quartic level (N >= 2)
    static constexpr int BP = X5 + ((N >= 2) ? 14 * 15 : 0);      // packed upper triangle of the beta matrix
    static constexpr int MINV = BP + D::NBP;                      // [3][2][2] inverse centroid-difference matrices
    static constexpr int PM = MINV + 12;                          // [NP-1][NMONO] projection onto psi_1..
    static constexpr int GBASE = PM + (D::NP - 1) * D::NMONO;      // base b of the linear weights b^(l-1): 1/h0 or 10
    static constexpr int AREA0 = GBASE + 1;                        // area of Delta0
    static constexpr int VALID = AREA0 + 1;                        // 1 = full-rank stencil
    static constexpr int RAW = VALID + 1;
    static constexpr int LEN = (RAW + 7) / 8 * 8;                  // padded to 64 bytes
};

}  // namespace cswdg
