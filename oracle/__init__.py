"""FP64 CPU oracle for the RKDG + compact subcell WENO (CSWENO) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP library; the only common
module is the seeded input generator (paper_2106_06280_amd.inputs), which
holds no method arithmetic.

The oracle follows the paper step by step in plain numpy float64,
vectorised over elements (residual, indicator) and over troubled cells
(limiter).  Every function cites the section / equation it follows.

Parity status per function is stated in each module header, as are the
readings taken where the paper is silent or garbled.
"""
