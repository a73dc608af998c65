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

// Top member of the N >= 2 reconstruction hierarchy (Section 3.2, Steps
// 1-2 for P2).  The text builds p_4 from the cubic q_4 (eq.
// equivalentOrder3, three weights gamma_{.,4}) and p_5 from the quartic q_5
// (eq. equivalentOrder4) and then combines four members with gamma_{.,5}:
//   kTopQuartic    p_top from q_5 by eq. equivalentOrder4 (four weights);
//   kTopQuadratic  the three members of N = 1 (q_3 on top, gamma_{.,3});
//   kTopCubic      p_4 from q_4 by eq. equivalentOrder3 as printed, the
//                  members {p_1, p_2, p_3, p_4} combined with gamma_{.,5};
//   kTopCubicTel   q_4 in place of q_5 in eq. equivalentOrder4.
constexpr int kTopQuartic = 0, kTopQuadratic = 1, kTopCubic = 2, kTopCubicTel = 3, kTopSextic = 4;

template <int N>
struct Dims {
    static constexpr int NP = (N + 1) * (N + 2) / 2;
    static constexpr int NV1 = (3 * N + 1) / 2;
    static constexpr int NQ = NV1 * NV1;
    static constexpr int NE = (3 * N + 2) / 2;
    static constexpr int NI1 = N + 4;
    static constexpr int NQI = NI1 * NI1;
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

// Layout of the per-element limiter operator record (doubles) for degree N
// and top member QT.  A hierarchy with a fourth member (N >= 2, QT not
// kTopQuadratic) reads all seven pieces per neighbour (S1, S2, S3 and the
// cut pieces S2', S21, S3', S31) and writes its reconstruction in the NT
// monomials of the top level (9 cubic or 14 quartic); the sextic top (N = 3)
// also reads the ten pieces of T5 per neighbour (each T4 piece halved by the
// median from the neighbour's centroid) and writes 27 monomials of degree
// 1..6; the three-member hierarchy (N = 1, or kTopQuadratic) reads the
// three centroid pieces and writes the reconstruction in the 5 monomials of
// degree 1..2.
template <int N, int QT>
struct OpLayout {
    using D = Dims<N>;
    static constexpr bool FOUR = (N >= 2) && QT != kTopQuadratic;
    static constexpr bool SEXT = (N == 3) && QT == kTopSextic;
    static constexpr int NT = !FOUR ? 0 : (SEXT ? 27 : ((QT == kTopCubic || QT == kTopCubicTel) ? 9 : 14));
    static constexpr int DR = !FOUR ? 2 : (SEXT ? 6 : (NT == 9 ? 3 : 4));  // degree of the reconstruction
    static constexpr int NPC = SEXT ? 17 : (FOUR ? 7 : 3);            // pieces per neighbour
    static constexpr int NROW = SEXT ? 30 : 15;                       // rows of the top level (T5 or T4)
    static constexpr int NM = FOUR ? NT : 5;                        // monomials of the reconstruction
    static constexpr int NBP = NM * (NM + 1) / 2;
    static constexpr int AVG = 0;                                   // [3][NPC][NP] subcell-average functionals
    static constexpr int X2 = AVG + 3 * NPC * D::NP;                // [2][3]   pinv, linear level
    static constexpr int X3 = X2 + 2 * 3;                           // [5][9]   pinv, quadratic level
    static constexpr int X5 = X3 + 5 * 9;                           // [NT][NROW] pinv, top level on T4 or T5
    static constexpr int BP = X5 + NT * NROW;                       // packed upper triangle of the beta matrix
    static constexpr int BPL = BP + NBP;                            // the same over derivative orders 1..N only
    static constexpr int MINV = BPL + NBP;                          // [3][2][2] inverse centroid-difference matrices
    static constexpr int PM = MINV + 12;                            // [NP-1][NM] projection onto psi_1..
    static constexpr int GBASE = PM + (D::NP - 1) * NM;             // base b of the linear weights b^(l-1): 1/h0 or 10
    static constexpr int AREA0 = GBASE + 1;                         // area of Delta0
    static constexpr int VALID = AREA0 + 1;                         // 1 = full-rank stencil
    static constexpr int RAW = VALID + 1;
    static constexpr int LEN = (RAW + 7) / 8 * 8;                   // padded to 64 bytes
};

// Layout of the per-element record of the type-I reconstruction (N = 1, 2):
// the centroid-subcell average functionals, the pseudo-inverses of the
// central stencil (rows piece-major, then face: 9) and of the three sectors
// (faces k, k+1; rows piece-major, then the two faces: 6), the smoothness
// matrix and the projection, in the NM monomials of degree 1..N.
template <int N>
struct OpLayoutT1 {
    using D = Dims<N>;
    static constexpr int NM = N == 1 ? 2 : 5;
    static constexpr int NBP = NM * (NM + 1) / 2;
    static constexpr int AVG = 0;                         // [3][3][NP]
    static constexpr int XC = AVG + 9 * D::NP;            // [NM][9]
    static constexpr int XS = XC + NM * 9;                // [3][NM][6]
    static constexpr int BP = XS + 3 * NM * 6;            // packed upper triangle
    static constexpr int PM = BP + NBP;                   // [NP-1][NM]
    static constexpr int AREA0 = PM + (D::NP - 1) * NM;
    static constexpr int VALID = AREA0 + 1;
    static constexpr int RAW = VALID + 1;
    static constexpr int LEN = (RAW + 7) / 8 * 8;
};

// Layout of the per-element record of the type-II reconstruction (N = 2):
// the centroid-subcell average functionals, the pseudo-inverses of the
// linear fits on the three single-neighbour stencils (rows: the neighbour's
// three pieces) and on the three sectors (faces k, k+1; rows piece-major,
// then the two faces), and at the 9 points of the degree-4 rule on Delta0
// the six linear weights, the two mean-free scaled linear monomials and the
// projection weights w_q psi_i(x_q); BSC = |Delta0| / h0^2 (the smoothness
// indicator of a linear fit is BSC |c|^2 in its scaled coefficients).
struct OpLayoutT2 {
    static constexpr int NP = 6, NQ = 9, NJ = 6;
    static constexpr int AVG = 0;                 // [3][3][NP]
    static constexpr int XF = AVG + 9 * NP;       // [3][2][3]
    static constexpr int XS = XF + 3 * 2 * 3;     // [3][2][6]
    static constexpr int GAM = XS + 3 * 2 * 6;    // [NQ][NJ]
    static constexpr int PHI = GAM + NQ * NJ;     // [NQ][2]
    static constexpr int PMQ = PHI + NQ * 2;      // [NP-1][NQ]
    static constexpr int BSC = PMQ + (NP - 1) * NQ;
    static constexpr int VALID = BSC + 1;
    static constexpr int RAW = VALID + 1;
    static constexpr int LEN = (RAW + 7) / 8 * 8;
};

// Layout of the per-element record of the mixed reconstruction (N = 2):
// the centroid-subcell average functionals and the linear fits of the
// type-II record, the pseudo-inverse of the quadratic fit on the nine
// pieces (rows piece-major: piece p of face f is row 3 p + f), the packed
// upper triangle of the smoothness matrix of a quadratic (derivative
// orders 1 and 2), the projection PM[i-1][j] = sum_q w_q phi_j(x_q)
// psi_i(x_q) of the scaled monomials onto psi_1..psi_5 (degree-4 rule of the
// reference triangle, where the basis is orthonormal), and BSC = |Delta0| /
// h0^2.
struct OpLayoutMX {
    static constexpr int NP = 6, NM = 5;
    static constexpr int AVG = 0;               // [3][3][NP]
    static constexpr int XF = AVG + 9 * NP;     // [3][2][3]
    static constexpr int XS = XF + 3 * 2 * 3;   // [3][2][6]
    static constexpr int X3 = XS + 3 * 2 * 6;   // [NM][9]
    static constexpr int BP = X3 + NM * 9;      // [NM (NM + 1) / 2]
    static constexpr int PM = BP + NM * (NM + 1) / 2;  // [NP-1][NM]
    static constexpr int BSC = PM + (NP - 1) * NM;
    static constexpr int VALID = BSC + 1;
    static constexpr int RAW = VALID + 1;
    static constexpr int LEN = (RAW + 7) / 8 * 8;
};

}  // namespace cswdg
