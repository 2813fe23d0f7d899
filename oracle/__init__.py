"""CPU oracle for sliced bucket-elimination contraction -- TEST INFRASTRUCTURE.

This package is the slow, plain, obviously-correct reference that the GPU
library is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the GPU library (``paper_2004_10892_amd``): the two
only consume the same seeded inputs from ``circuitgen``.

Modules
-------
statevector  -- textbook dense statevector simulation of the circuits
                (the plain definition of <x|C|0^n>).
planner      -- simple graph, greedy min-fill order, Alg. 1 (treewidth of an
                order), the clique tree of App. A (Alg. 4, maximal-bag
                reading), the tree-trimming score of Sec. 3.2, the degree,
                betweenness and Alg. 3 scores of Sec. 3.1, and the greedy
                mu-treewidth deletion of Alg. 2.
contract     -- brute-force summation (Eq. 1 as a plain sum), and bucket
                elimination with sliced variables (Eqs. 2-4) in complex128.
cost         -- per-bucket FLOP / byte counts and peak memory of a schedule
                (Sec. 4 cost statements; exact formulas are this project's).

Parity status: every function is pinned by a test under ``tests/`` against
something other than itself (the worked example of Eq. 2, Figs. 3, 4 and 6,
brute force, statevector simulation, closed forms); the only unpinned item is
the *quality* of tree-trimming against the paper's figures, whose values are
not available ("parity unpinned" for that aspect only).
"""
