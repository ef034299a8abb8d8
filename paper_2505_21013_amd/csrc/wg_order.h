// Workgroup orders of the PCG matrix product (host and device; plain C++ so
// that the host tests can check them).
#pragma once

namespace ppn {

// Panel order within an XCD's chunk of C workgroups: the chunk is cut into
// panels of P consecutive workgroups (the last one possibly shorter), and the
// k-th workgroup the XCD dispatches is offset k / (panels) of panel
// k % (panels), offsets ascending.  Workgroups P apart then run at the same
// time: rows about one matrix bandwidth apart, which read each other's stored
// blocks (each block is read by its owner row and, transposed, by its partner
// row), do so close in time and meet in the L2.  A bijection of [0, C);
// P <= 0 or P >= C gives the identity.
constexpr int panel_order(int k, int C, int P) {
  if (P <= 0 || P >= C) return k;
  const int np = (C + P - 1) / P;  // panels
  const int r = C - (np - 1) * P;  // length of the last panel (1..P)
  if (k < r * np) return (k % np) * P + k / np;
  const int k2 = k - r * np;  // offsets r.. exist in the first np - 1 panels only
  return (k2 % (np - 1)) * P + r + k2 / (np - 1);
}

}  // namespace ppn
