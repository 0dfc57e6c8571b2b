"""MI355X (gfx950) implementation of the data-parallel solve of specular
polynomials (Fan et al., ACM TOG 2024): a C-ABI HIP library (csrc/, include/)
and its Python binding (spoly.py).  Scene generators live in scenes.py."""
