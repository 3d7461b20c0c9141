"""FP64 CPU oracle for the LEE + ghost-point IBM + ADE impedance stage.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package; the
GPU library never does, and this package never imports the library.  The two
share no code: only the plain problem descriptions in ``lee_cases`` serve both.

The oracle follows the paper step by step, in its order and notation:

* ``schemes``   DRP first-derivative stencils (Sec. 2.2, eq. DRP_s), the
                11-point selective filter and the low-storage RK4 stage
                coefficients (readings listed in the module);
* ``geometry``  mask, ghost selection, boundary point / normal / r, and the
                elliptical cloud (Sec. 3.1, eqs. ns-rotation, ns-ellipse);
* ``weights``   Vandermonde least squares and read-out at P_0..P_4
                (eqs. ns-poly2d .. ns-readout) and the 1-D Lagrange and
                Birkhoff extrapolation weights (eq. ns-ghost);
* ``ade``       mass-spring-damper poles, residues and ADE matrices
                (Secs. 2.3 and 2.5);
* ``core.c``    the time stepping (Sec. 3.2, six coupling steps per stage),
                plain C loops in FP64;
* ``solver``    glue: builds everything for a case and runs the core.

Parity status of each function is stated in its module header.
"""
