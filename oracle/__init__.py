"""CPU FP64 oracle for the SAA smoothed-CVaR objective and gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
binding imports, calls or links this package; only the tests, the smoke check
and the CPU-baseline leg of the benchmark do.  It shares no code with the HIP
path: every quantity here is computed from the paper's definitions with plain
numpy / scipy in float64 (textbook element loops, sparse direct solves,
bisection), so that a reader can check it against the paper by eye.

Modules
-------
fem2d      P1 finite elements for the semilinear elliptic state equation
           (Sec. 4.2), Newton with sparse LU, QoI, adjoint gradient (Sec. 2.3).
fem3d      Q1 finite elements for the same equation on the unit cube.
cvar       smoothed plus function, Rockafellar-Uryasev SAA CVaR, its
           minimiser t* and gradient weights (Sec. 2.1-2.2).
saa        per-sample (q, dq/dz) and the SAA objective + gradient.
surrogate  MR-DINO: KL encoder, MLP, reduced QoI, VJP/JVP (Sec. 3.1, 3.3).
training   weighted POD, DINO loss, its hand-derived gradient, Adam
           (Sec. 3.2-3.4).
"""
