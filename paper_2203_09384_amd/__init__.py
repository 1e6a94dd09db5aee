"""mifft: batched 1D complex-to-complex FFTs of power-of-two length on MI355X (gfx950)."""
