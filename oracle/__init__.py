"""CPU oracle for the PAC stochastic-aggregation path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call, link or execute anything in this package.  The
GPU library never routes through it, and it shares no code, header, table or
constant generator with the GPU sources: every formula here is written again
from the paper.

Modules
-------
``pac_ref``     plain, slow, obviously correct Python/numpy definitions:
                the keyed PU hash, the m-execution brute force over sampled
                databases (Sec. 4.1 compile procedure), the per-world
                aggregate definition (Sec. 4.2 ``pac_agg``) and the sequential
                noise / posterior release (Sec. 4.1 ``pac_noised``, Sec. 3.2
                NULLs, Sec. 5 diversity check).
``onepass.c``   the same per-world definition as a multi-threaded C loop
                (``native``), used for full-size inputs and timed as the CPU
                baseline.
``approx_sum.c`` the approximate integer SUM of Sec. 5 (16-bit counters in
                25 levels cascading every 4 bits, two-sided or signed), one
                sequential pass per block of rows (``native.approx_sum``).
"""
