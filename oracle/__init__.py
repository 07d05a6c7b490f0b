"""Plain FP64 CPU oracle for the VtV volume potential on a boundary-concentrated cube mesh.

TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
leg may import, call or execute anything in this package. The product path (the HIP
library and its Python binding) never does, and shares no code, tables or constants with
it; the two meet only through the seeded densities of the `synth` package.

Contents (each function cites the passage of the paper it follows):
  mesh.py      BC refinement (Sec. 2: B_l, M_l, L_l, C_{l+1}, L*_l), neighbours (eq. def:neighbors),
               interaction lists (Sec. 2), extended neighbour lists N* (Sec. 3, Lemma 1).
  touching.py  exact integrals of 1/|x-y| over touching cube pairs (convolution + Duffy), also
               with Legendre polynomial weights on both boxes.
  taylor.py    multi-indices and Taylor coefficients of 1/|r+h| (binomial series).
  direct.py    O1: u = A f by direct O(N^2) evaluation of the Galerkin entries.
  fmm.py       O2: Algorithm 1 step by step (near field, moments, upward pass, interaction
               phase, downward pass, evaluation) in FP64.
  mlp.py       the touching-pair surrogate's network in FP64: forward pass, training loss and its
               gradient by the chain rule (reference for the GPU kernels' gradients).
  basis.py     degree-p leaf bases (p_l = L - l, Legendre tensor polynomials): O1 and O2 with
               polynomial leaf spaces, entry blocks (exact where the cubes touch, via
               touching.box_pair_poly), projection of a density onto the leaf spaces.
  mapped.py    mapped (curved) meshes, the BC octree pushed through a map (the cube-to-ball map;
               plain-C loops in mapped.c): entries with a singular rule for touching curved cells,
               O1 by direct summation and O2 step by step with Taylor translations between the
               images of the cell centres.
  boundary.py  BtV (Algorithm 3): single- and double-layer entries of (leaf, boundary face) pairs
               (exact by convolution where they touch, point rule elsewhere), O1 by direct
               summation and O2 step by step.

Readings of the paper used here (all for the cube-octree form of the method):
  * marking rule: M_l = B_l (cells with a face on the boundary), l < L;
  * separation ratio uses rho_w + rho_w' (the printed rho_w' + rho_w' is a typo);
  * eta = eta0 is not a neighbour (strict inequality), decided by an integer test;
  * basis degree p = 0 with the indicator basis 1_w, so u_w = <1_w, N f>;
  * non-touching cell pairs use the 2x2x2 Gauss point rule; touching pairs the exact integral;
  * moments and evaluation use the same 2x2x2 point rule, so O2 -> O1 as q grows.
"""
