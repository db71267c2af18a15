"""CPU oracle for STTSV on the blowup adjacency tensor and for the NQZ
H-eigenvector iteration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers); the two meet only through
the seeded input arrays produced by ``paper_2311_08595_amd.workloads``, which
holds none of the method's arithmetic.

Modules
-------
``blowup``     exact-rational definitions: Stirling numbers, |beta(e)|, the
               blowup tensor entries enumerated one by one (Sec. II), TTSV1
               by the tensor definition (Eq. (2)) and AAY (Alg. 2) in exact
               rationals.
``sttsv_ref``  FP64 AAY (Alg. 2) vectorised per edge size, in the ordinary
               power-series basis with full-length truncated convolutions,
               correctly rounded per-node sums (math.fsum).
``nqz_ref``    Alg. 1 (NQZ) on top of ``sttsv_ref``.
``plan_ref``   the canonical edge order, size buckets, member layout and
               node-major incidence lists, written independently of the C++
               planner so the two can be compared bit for bit.
``mpnn_ref``   FP64 forward/backward of the warm-start message-passing net.
``ccss_ref``   the CCSS forest (Sec. III) and Alg. 4's memoised STTSV over it.
``sshopm_ref`` the full contraction B x^r and SS-HOPM Z-eigenpairs.
``cp_ref``     symmetric CP decomposition of B by Armijo gradient descent.

Every function names the passage of the paper it follows.  Where the paper is
silent or garbled the reading taken is stated in the docstring.
"""
