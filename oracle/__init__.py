"""CPU oracle for the supernodal Cholesky hot path.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything under ``oracle/``. The product (``paper_2409_13090_amd``) never
imports it, and the two share no code.

* ``osym``  -- naive symbolic analysis (ordering, etree, supernodes, merging,
  within-supernode reordering, relind / blocks / relindB), from the
  definitions of Section 2.1.2, Section 2.2.2 and Section 3.1.
* ``onum``  -- the paper's Algorithm 1 (Section 2.1.1) in plain C, FP64.
"""
