"""Plain FP64 / complex128 CPU oracle for the sampled finite-PEPS + minSR path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import or call
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it. It shares no code with the HIP library or its Python
binding; both sides only share the seeded input generators in ``synth``.

Every function follows the paper (arXiv 2503.12557, "Efficient optimization
and conceptual barriers in variational finite Projected Entangled-Pair
States") step by step and cites the passage it implements. Where the paper
is silent the reading taken is stated at the function.

Parity status of each part:
  * exact-contraction amplitudes, local energies, log-derivatives and the
    minSR solve are pinned by brute force, exact enumeration, closed forms
    and identities (tests/test_oracle_*.py);
  * amplitudes, energies and log-derivatives at a truncating contraction
    bond (chi below the exact Schmidt rank) are "parity unpinned" beyond the
    invariants that hold at any chi (product-state limit, uniform amplitude,
    homogeneity of O, finite differences of the strip amplitude, agreement
    of the two truncation algorithms).
"""
