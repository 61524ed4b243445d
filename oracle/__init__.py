"""Plain FP64 CPU oracle for the windowed Fourier projection (WFP) march.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constant generators); the
only thing both sides consume is the seeded input generator, which holds none
of the method's arithmetic.

The oracle computes the fully discrete scheme of the paper (Sections 2-4:
eqs. (periodicIE_disc), (alphakEvolutionFormulas), (hkcompdisc), the local
quadrature of Section 4.1 and the RBC projection of Section 4.4) with every
fast component replaced by its plain definition:

* exponential sums are evaluated directly (no NUFFT),
* the RBC uses direct real DFTs of length 2K (no FFT),
* neighbours are found by brute-force distance tests,
* local weights Q_m(d) are evaluated from their definition per pair,
* the implicit system is solved with a sparse LU factorisation.

Independent pins (closed forms, identities, brute force) live in
``oracle.exact`` / ``oracle.volterra`` and are exercised by ``tests/``.

Modules
-------
window    Kaiser-Bessel blending window phi, phi', phi'' (eqs. KB, phi, b)
params    derived parameters (b, W, delta, K, m_max, ...)
history   influence kernels Psi_k, p_k, q_k, one-step mode propagator
local     periodic distance, neighbour classes, local weights Q_m(d)
march     the fully discrete march (Tier A), incident-field driving data
rbc       the free-space radiation-boundary projection P
exact     closed-form solutions used as pins (Tier B)
volterra  naive marching of the unwindowed Volterra equation (brute force)
"""
