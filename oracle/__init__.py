"""Plain, slow FP64 CPU oracle for the batched DC N-1 topology screen.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only the test suite, the package smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP library (no kernels, headers, helpers, tables or pre/post-processing);
the only common dependency is the seeded input generator ``gridgen``, which
holds none of the method's arithmetic.

What it computes, per candidate topology (Problem formulation and Fitness
function heuristics sections of the paper; DC linearisation from the Importer
and DC-Optimizer sections):

  1. the post-switch bus-branch network: opened branches removed, every bus
     split creates a second busbar that receives the moved branches and the
     moved part of the injection (two-node operation),
  2. islanding by connected components over the in-service branches,
  3. N-0 flows and the flows of every single-branch contingency by solving the
     reduced nodal equations B' theta = P from scratch (slack angle 0), with
     f_e = b_e (theta_from - theta_to),
  4. the congestion metrics lambda_o, lambda_c, lambda_c0, the maximum loading
     and its arg-max, the fitness lambda_f1 and a MapElites descriptor cell,
  5. the per-cell elite archive by one-at-a-time strict-improvement insertion.

Pins (tests/test_oracle_pins.py) tie every part to facts that do not come from
the oracle itself: radial-grid closed forms, Kirchhoff's laws, superposition,
the parallel-line current divider, exhaustive islanding enumeration, the
line-outage distribution factor identity, split/outage equivalences and
hand-worked metric examples under tests/golden/.
"""
from .dcflow import (  # noqa: F401
    Candidate, CandidateResult, candidate_from_batch, validate_candidate,
    post_switch_network, is_connected, solve_flows, evaluate_candidate,
    evaluate_batch, busbar_outage_flows, busbar_metrics, fitness_f2,
)
from .metrics import (  # noqa: F401
    n1_metrics, fitness_f1, descriptor_cell, archive_insert_sequential,
    contingency_energies, worst_k, descriptor_cell_paper,
)
