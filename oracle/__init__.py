"""CPU oracle for the Multiscale Robin Coupled Method (MRCM) — TEST INFRASTRUCTURE.

A plain, slow, FP64 implementation (NumPy/SciPy) of what the HIP library
computes, written from the paper's Section 2 ("Mathematical model and
numerical schemes").  It exists only to check the library: it is imported by
``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py``, and by nothing else.  It shares no code, header, table or
helper with the HIP path.

Modules
-------
geometry    subdomains, interfaces, patches (Sec. 2.2 "Domain decomposition";
            interface space V_H and its cardinality, eq. (2.24))
fine        two-point-flux finite volumes and the global fine-grid solve
            (eqs. (2.9)-(2.12))
mrcm        the MRCM algorithm (Algorithm 2): local Robin problems (2.13),
            (2.14) and their MBF systems (2.25), (2.26); interface system
            (2.15)-(2.22); interface solve; reconstruction (2.23)
monolithic  independent formulations used only as pins: the whole MRCM as one
            sparse system, and its alpha -> 0 / alpha -> infinity limits
banded      textbook banded Cholesky / band solves (used to pin the band
            factor the library stores)
norms       the error norms of Sec. 3.1 (relative L2 for pressure,
            K^-1-weighted L2 for velocity)

Where the paper is silent or garbled, each module states the reading it
adopts next to the code that depends on it; each function names the passage
it follows.
"""
