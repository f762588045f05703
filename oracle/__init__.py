"""CPU oracle for the simultaneous matrix cosine and sine (test infrastructure).

This package is test infrastructure. Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product library and its
Python binding never do, and it never imports them.

Contents, each following the paper (Seydaoglu, Bader, Blanes, Casas,
"Computing the matrix sine and cosine simultaneously with a reduced number of
products", arXiv 2010.00465):

* ``reference``  - a plain, independent algorithm for cos(A), sin(A): exact
  1-norm, scaling to norm <= 1, Horner evaluation of the Taylor series
  (Section 2.1 definitions of T^c_{2m}, T^s_{2m+1}) and the double-angle
  recovery of Section 1; float64 and 80-bit long double.
* ``schemes``    - the paper's factorized schemes with 3, 4, 6 and 7 products
  (Section 2.1) over any algebra (matrices or scalar polynomials), with the
  coefficient sets typed from the paper.
* ``theta``      - the truncation-error bounds of Section 3 and the
  re-derivation of Tables 1 and 2.
* ``plan``       - the choice of scheme and scaling power from the 1-norm.
* ``paper_algorithm`` - the paper's full method (plan + scheme + double angle)
  written out plainly in float64.
* ``frechet``    - derivative references: the block-triangular Frechet
  derivative, a dual-number variant, and central finite differences.

Parity status of every function is stated in its module header.
"""
