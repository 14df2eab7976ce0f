"""CPU FP64 oracle for the stable FDTD method with embedded reduced-order models.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, NumPy/SciPy
implementation written from the paper (Zhang, Bekmambetova, Triverio, IEEE
TAP 2017).  It is imported only by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``.  The GPU library never
imports, links or calls anything in here, and this package shares no code
with it: the only common module is ``workloads`` (seeded problem
descriptions, no method arithmetic).

Modules
  constants  physical constants
  yee        coarse TEz Yee grid: coefficients, masks, leap-frog step (Sec. II-A, eqs. (3)-(5))
  fine       fine-region descriptor system R, F, B, L, S (eqs. (6)-(8), (24)-(25))
  rom        SPRIM-style congruence reduction and the CFL-extending clip (eqs. (9)-(12), (27))
  coupling   coarse/ROM interface: literal A1/A2 system and its closed form (eqs. (13)-(23))
  sim        whole coupled run: probes, energy (Sec. IV, Sec. V, Appendix)
  subgrid    direct merged-edge subgridding (an independent check of the coupling)
  adjoint    discrete adjoint of the coupled run (gradients w.r.t. cell materials)
  model_grad gradients through the reduced models: eq. (23) closed form, ring
             cells, the eq. (27) clip and the congruence (fine-cell materials)

Parity status per function is stated in each module header.
"""
