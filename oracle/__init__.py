"""CPU oracle for the failure-less Aho-Corasick matcher.

TEST INFRASTRUCTURE ONLY. This package is imported, called or executed only by the test
suite, by ``__graft_entry__.smoke()`` (to check the GPU result) and by the benchmark's
``cpu_baseline`` leg. The product path (the HIP library and its Python binding) never
touches it, and it shares no code with that path: the only inputs both sides take come
from the seeded generators in ``paper_1704_02272_amd.workloads``, which hold none of the
method's arithmetic.

Contents
--------
* ``literal``  -- the match set written out from its definition (every pattern compared
                  at every start position), pure Python, for small inputs.
* ``native``   -- ctypes wrapper over ``oracle.c``: a length-bucketed brute force and a
                  textbook Aho-Corasick (failure + dictionary links, overlapped chunks).
* ``trie``     -- the paper's storage model for the trie (Section 3.1 and Eq. 1):
                  breadth-first node numbering of the sorted patterns, one first-child
                  offset and one alphabet-wide child bitmap per node; plus a walker that
                  applies Eq. 1 to that array, and the byte accounting of the model.
* ``reduce``   -- the trie compression of Section 3.2 as a node count (merging nodes of
                  the bottom levels whose suffixes agree; Eq. 2; Eqs. 3-4 read as an
                  occupancy law).
* ``prefix``   -- prefix depths: for every start, the longest pattern prefix the text
                  spells there, as a histogram (the quantity behind the truncated trie
                  of Section 2.4 and the prefix-length study of Section 4.2).

Parity status: every function here is pinned by tests under ``tests/`` against hand
derived answers, printed values of the paper, closed forms and cross-algorithm checks.
No function is "parity unpinned".
"""
