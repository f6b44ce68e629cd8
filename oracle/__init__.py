"""FP64 CPU oracle for velocity-gauge real-time TDDFTB propagation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference against
which the HIP library is checked.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the library itself never
does, and the two share no code (only the seeded input generator feeds both).

Every function cites the passage of the paper (arXiv 2308.09782, Section 2)
whose computation it writes out.  Where the paper is silent the reading used
is stated in the docstring.  All arithmetic is complex128 / float64.

Pinned by tests/test_oracle_*.py (closed-form leapfrog solution, brute-force
matrix-exponential propagation, invariants, the gauge identity, textbook sp3
and single-orbital-chain models, SCC special cases and the work theorem,
spectrum closed forms: a filtered sinusoid, the mean subtraction, and the damped
free-electron (Drude) dielectric function for Eq. 16; a k-point split into two
halves of its weight; for the momentum-matrix coupling of Eq. 12: Hermiticity,
the closed-form diamagnetic current, the |A|^2 term as a pure phase, the
orthogonal-basis limit, energy conservation at constant A, the work theorem of
its current matrix under an SCC pulse and brute-force propagation; for the
Crank-Nicolson propagation of the coefficients (Eq. 5): the closed-form
Cayley-transform solution, exact S-unitarity, stationarity of the ground state
and second-order convergence towards independent fine-step integrators).
"""
from .tddftb import (  # noqa: F401
    C_LIGHT,
    bloch_sum,
    overlap_k,
    overlap_inverse,
    h0_k,
    momentum_k,
    overlap_momentum_k,
    h_ext_k,
    field_hamiltonian_k,
    current_matrix_k,
    scc_potential,
    hamiltonian_k,
    mulliken,
    ground_state,
    occupations,
    density_derivative,
    density_derivative_columns,
    observables,
    propagate,
    OracleState,
    make_state,
)
from .coefficients import (  # noqa: F401
    density_from_coefficients,
    ground_state_coefficients,
    propagate_crank_nicolson,
    crank_nicolson_step,
    CoefficientState,
    make_coefficient_state,
)
from .spectrum import conductivity, dielectric, absorption  # noqa: F401
