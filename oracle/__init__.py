"""CPU FP64 oracle for the boundary-MPS branch-and-bound method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; both sides take the same seeded instances from ``tnb_inputs``.

Modules
  ising   -- Eq. (1), (6), (10): energies, brute-force Z / marginals / ground
             states, closed forms.
  potts   -- Eq. (3)-(5): cluster tables E_n[x], projectors, compressed bond
             tables.
  bmps    -- Sec. III.B: PEPS row transfer, variational zipper with randomized SVD,
             truncation, log Z.
  search  -- Sec. III.A, Eq. (7)-(9): conditional marginals from the
             boundary MPS and branch and bound with boundary merging.
  droplets -- Sec. III.A, Fig. 4: excitations above each main branch from
             the members its merge discards.
  lbp     -- Sec. IV, Fig. 9: loopy belief propagation on projected cluster
             states and the reduction to the most probable states.
"""
