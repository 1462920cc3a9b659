"""CPU oracle for the FlashGS rasterizer (test infrastructure only)."""
