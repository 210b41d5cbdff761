"""Plain FP64 CPU oracle for the FE-DVR second-Born ground-state path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP path;
the only common ground is the seeded input generators in ``workloads``.

Each function follows the paper (Balzer, Bauch, Bonitz, "Finite elements and
the discrete variable representation in nonequilibrium Green's function
calculations") step by step, citing the section and equation it implements.
Everything is NumPy float64; library primitives used as single steps are
``numpy.linalg.eigh``, matrix products and ``numpy.fft``.

Modules
    fedvr   -- Gauss-Lobatto elements, DVR basis, T, v, V; tau grids
    hf      -- Hartree-Fock self-energy, HF ground state, chemical potential, G0(tau)
    sigma   -- second-Born self-energy (literal, general-basis and factorized forms)
    dyson   -- tau-convolution quadrature, Dyson step, Galitskii-Migdal energy
    scf     -- the self-consistent second-Born loop
    ed      -- exact two-electron diagonalisation and closed-shell MP2 (pins)
    mlp     -- the learned initial guess (features, network, gradients, Adam)
"""
from . import fedvr, hf, sigma, dyson, scf, ed  # noqa: F401
