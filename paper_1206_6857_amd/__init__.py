"""MI355X (gfx950) Gaussian summation library: Python binding package."""
