"""Ensemble ODE/SDE solving on AMD MI355X (gfx950): Python face of libens.so."""
