"""CPU correctness oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, complex128 numpy simulator of what the GPU path computes:
batched state vectors evolved through uniform layers of gates, the <Z_i>
readout and exact gradients.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the GPU library; it takes its inputs from the ``workloads`` module, which holds
no simulation arithmetic.

Modules
-------
gates  -- the gate matrices of the paper's Appendix A (with the readings of the
          garbled ECR and MS entries), their analytic parameter derivatives.
sim    -- tier O1 (full 2^n x 2^n layer unitaries from Kronecker products, the
          paper's "Unitary operation", Sec. 2.2.1) and tier O2 (per-gate tensor
          contraction, the paper's "Sequential Einsum", Sec. 2.2.2); the <Z_i>
          readout through the paper's K_Rz = 1 - 2J matrix (Sec. 2.4.1); and
          gradients by three independent routes (adjoint sweep, parameter shift,
          central finite differences).

Every function here is pinned by tests under ``tests/test_oracle_*.py``
against values the paper prints, closed forms, library special cases and
invariants.
"""
